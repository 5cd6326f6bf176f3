// Observables over a population (arXiv:1711.05095, Secs. 2.4 and 3.3): the
// squared modulus of a Fourier mode of the density (eq. fourdens) per clone,
// and the mean and the histogram of a per-clone quantity over the current
// population (the end-time distribution) or over the ancestors of the current
// population at the last origin reset (the ancestral distribution, eq. Opave),
// and the descendant counts of the clones at the last origin reset.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_internal.hpp"
#include "pd_launch.hpp"

namespace pd {

// out[j] = |L^{-1/2} sum_{occupied i} e^{-2 pi i n i / L}|^2 for the clones
// of instance `inst`, population in state[cur] in slot order.
template <int W>
__global__ __launch_bounds__(kTile) void k_density_mode(const InstDev* __restrict__ insts,
                                                        int inst, int cur, int n,
                                                        double* __restrict__ out)
{
    __shared__ double s_cos[kMaxSites], s_sin[kMaxSites];
    const InstDev& I = insts[inst];
    const int L = I.L;
    for (int i = threadIdx.x; i < L; i += kTile) {
        // the phase n i / L taken mod 1 exactly in integers
        int64_t m = ((int64_t)n * i) % L;
        if (m < 0) m += L;
        double sv, cv;
        sincospi(2.0 * (double)m / (double)L, &sv, &cv);
        s_cos[i] = cv;
        s_sin[i] = sv;
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * kTile + threadIdx.x;
    const int64_t Nc = I.Nc;
    if (j >= Nc) return;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t bits = gptr(I.state[cur])[w * Nc + j];
        while (bits) {
            const int i = w * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
            re += s_cos[i];
            im -= s_sin[i];
        }
    }
    out[j] = (re * re + im * im) / (double)L;
}

// Per-block sums of v_j = values[j] (or values[origin[j]] when ancestral),
// written to the instance's tile_sum (one entry per 256 clones).
__global__ __launch_bounds__(kTile) void k_mean_partial(const InstDev* __restrict__ insts, int inst,
                                                        int cur, const double* __restrict__ values,
                                                        int ancestral)
{
    __shared__ double s_red[kTile / 64];
    const InstDev& I = insts[inst];
    const int64_t j = (int64_t)blockIdx.x * kTile + threadIdx.x;
    double v = 0.0;
    if (j < I.Nc) v = values[ancestral ? (int64_t)gptr(I.origin[cur])[j] : j];
    v = block_reduce(v, OpSum(), s_red);
    if (threadIdx.x == 0) gptr(I.tile_sum)[blockIdx.x] = v;
}

// mean = (sum of the partials in block order) / Nc, into tile_off[0].
__global__ __launch_bounds__(kTile) void k_mean_final(const InstDev* __restrict__ insts, int inst,
                                                      int nb)
{
    __shared__ double s_red[kTile / 64];
    const InstDev& I = insts[inst];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kTile) v += gptr(I.tile_sum)[b];
    v = block_reduce(v, OpSum(), s_red);
    if (threadIdx.x == 0) gptr(I.tile_off)[0] = v / (double)I.Nc;
}

__global__ void k_zero_u64(uint64_t* __restrict__ a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

// counts[b] += #{j : floor((v_j - lo) / width) = b}, v_j = values[j] (or
// values[origin[j]] when ancestral); each block counts its clones in LDS and
// adds its nonzero bins to the global counts (integer sums: the result does
// not depend on the order).
__global__ __launch_bounds__(kTile) void k_histogram(const InstDev* __restrict__ insts, int inst,
                                                     int cur, const double* __restrict__ values,
                                                     int ancestral, double lo, double width,
                                                     int nbins, uint64_t* __restrict__ counts)
{
    __shared__ uint32_t s_c[kMaxHistBins];
    const InstDev& I = insts[inst];
    for (int b = threadIdx.x; b < nbins; b += kTile) s_c[b] = 0;
    __syncthreads();
    const int64_t Nc = I.Nc;
    for (int64_t j = (int64_t)blockIdx.x * kTile + threadIdx.x; j < Nc;
         j += (int64_t)gridDim.x * kTile) {
        const double v = values[ancestral ? (int64_t)gptr(I.origin[cur])[j] : j];
        const double t = (v - lo) / width;
        if (t >= 0.0 && t < (double)nbins) atomicAdd(&s_c[(int)t], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += kTile)
        if (s_c[b]) atomicAdd((unsigned long long*)&counts[b], (unsigned long long)s_c[b]);
}

hipError_t launch_density_mode(int W, const InstDev* insts, int inst, int64_t Nc, int cur, int n,
                               double* out, hipStream_t st)
{
    const dim3 grid((unsigned)((Nc + kTile - 1) / kTile));
    switch (W) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL(k_density_mode<w>, grid, dim3(kTile), 0, st, insts, inst, cur, n,  \
                           out);                                                              \
        break;
        PD_CASE(1) PD_CASE(2) PD_CASE(3) PD_CASE(4) PD_CASE(5) PD_CASE(6) PD_CASE(7)
        PD_CASE(8)
#undef PD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mean(const InstDev* insts, int inst, int64_t Nc, int cur, const double* values,
                       int ancestral, hipStream_t st)
{
    const int nb = (int)((Nc + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_mean_partial, dim3(nb), dim3(kTile), 0, st, insts, inst, cur, values,
                       ancestral);
    hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(kTile), 0, st, insts, inst, nb);
    return hipGetLastError();
}

hipError_t launch_histogram(const InstDev* insts, int inst, int64_t Nc, int cur,
                            const double* values, int ancestral, double lo, double width,
                            int nbins, uint64_t* counts, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_u64, dim3((nbins + kTile - 1) / kTile), dim3(kTile), 0, st, counts,
                       nbins);
    const int64_t need = (Nc + kTile - 1) / kTile;
    const int blocks = (int)(need < 2048 ? need : 2048);
    hipLaunchKernelGGL(k_histogram, dim3(blocks), dim3(kTile), 0, st, insts, inst, cur, values,
                       ancestral, lo, width, nbins, counts);
    return hipGetLastError();
}

// counts[k] = #{j : origin[cur][j] = k}: the descendants, among the current
// clones of instance `inst`, of the clone that sat in slot k at the last
// origin reset (Sec. 2.4: after a long lag their expectation is proportional
// to v of its configuration).  Zeroed by k_zero_u32 first.
__global__ void k_zero_u32(uint32_t* __restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

__global__ __launch_bounds__(kTile) void k_descendants(const InstDev* __restrict__ insts, int inst,
                                                       int cur, uint32_t* __restrict__ counts)
{
    const InstDev& I = insts[inst];
    const int64_t j = (int64_t)blockIdx.x * kTile + threadIdx.x;
    if (j < I.Nc) atomicAdd(&counts[gptr(I.origin[cur])[j]], 1u);
}

// d_out[i] = hops of instance i so far, for every instance of the context.
__global__ __launch_bounds__(kTile) void k_hop_counts(const InstDev* __restrict__ insts, int n,
                                                     uint64_t* __restrict__ out)
{
    for (int i = threadIdx.x; i < n; i += kTile) out[i] = insts[i].ctl->hops;
}

hipError_t launch_hop_counts(const InstDev* insts, int n, uint64_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_hop_counts, dim3(1), dim3(kTile), 0, st, insts, n, out);
    return hipGetLastError();
}

hipError_t launch_descendants(const InstDev* insts, int inst, int64_t Nc, int cur,
                              uint32_t* counts, hipStream_t st)
{
    const unsigned blocks = (unsigned)((Nc + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks), dim3(kTile), 0, st, counts, Nc);
    hipLaunchKernelGGL(k_descendants, dim3(blocks), dim3(kTile), 0, st, insts, inst, cur, counts);
    return hipGetLastError();
}

}  // namespace pd
