// The learned guide: a translation-equivariant circular 1D convolutional net
// whose output f(C) = sum_j o_j predicts ln v(C), v the dominant eigenvector
// of the tilted generator, so that differences across a hop predict the
// optimal control of the modified dynamics (Sec. 2.2); it is trained by
// Poisson regression on the descendant counts of plain runs (a clone's
// expected number of descendants is proportional to v, Sec. 2.4).
//
//   a_j  = 2 n_j - 1
//   h1   = tanh(b1[c] + sum_k W1[c][k] a_{j+k-2})                 (1 -> 32 channels)
//   h2   = tanh(b2[c] + sum_{c',k} W2[c][c'][k] h1[c'][j+k-2])     (32 -> 32)
//   o_j  = b3 + sum_{c',k} W3[c'][k] h2[c'][j+k-2]                 (32 -> 1)
//
// Weights enter the arithmetic rounded to bfloat16 (the FP32 master copy is
// what Adam updates); the 32 x 160 x L contractions of layer 2 (forward, the
// weight gradient and the input gradient) run on MFMA 16x16x16 bf16 with FP32
// accumulation; the small layers 1 and 3 run on the vector ALU in FP32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_guide.hpp"
#include "pd_internal.hpp"

namespace pd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32, KS = 5, Q = CH * KS;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + CH * KS, OFF_W2 = OFF_B1 + CH,
              OFF_B2 = OFF_W2 + CH * CH * KS, OFF_W3 = OFF_B2 + CH, OFF_B3 = OFF_W3 + CH * KS,
              OFF_C0 = OFF_B3 + 1;
static_assert(OFF_C0 + 1 == kGuideParams, "parameter layout");

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bfr(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Forward and backward passes, one sample per wave, several waves per block
// sharing the weights.
//
// The layer-2 contraction index is taken tap-major, q = t * 32 + c' (tap t of
// the kernel, input channel c'), so that four consecutive q of an MFMA operand
// are four consecutive channels of one position: with the activations stored
// position-major ([position][channel], bf16) each operand of the forward pass
// and of the input-gradient pass is one 8-byte LDS read.  The weight-gradient
// pass contracts over positions and reads the activations position-contiguous
// ([channel][position]).  Positions carry a circular halo of two sites on each
// side (row i holds position i - 2).
//
// The scalar delta = d loss / d f of a sample is applied after the matrix
// products (in float32): the products run on g2 = w3s (1 - h2^2) and the
// results are scaled by delta, so no operand is converted per element.
// Layer-1 activations in float32 are recomputed where 1 - h1^2 is needed.
// ---------------------------------------------------------------------------
constexpr int kNetShared = 2 * CH * Q * 2 + 4 * (Q + 3 * CH);  // bytes

struct NetShared {
    uint16_t* W2R;   // [c][t * 32 + c']  = W2[c][c'][t]
    uint16_t* W2T;   // [c'][t * 32 + c]  = W2[c][c'][t]
    float* W1;       // [c][t] (bf16 values)
    float* b1;
    float* b2;
    float* w3s;      // sum_t W3[c][t] (bf16 values)
};

struct NetWave {
    float* sa;       // [P] a at row i = position i - 2
    uint16_t* H1P;   // [P][32] bf16 h1
    uint16_t* H1C;   // [32][P] bf16 h1
    uint16_t* G2C;   // [32][LP] bf16 g2 (zero beyond L)
    uint16_t* G2P;   // [P][32] bf16 g2
};

__host__ __device__ inline int net_lp(int L) { return (L + 15) / 16 * 16; }

// Bytes of one wave's region: its arrays, and at least the 32 x 160 floats of
// the end-of-block reduction of the layer-2 weight gradient.
__host__ __device__ inline size_t net_wave_bytes(int L)
{
    const size_t LP = net_lp(L), P = LP + 4;
    const size_t arrays = (4 * P + 15) / 16 * 16 + 2 * P * CH * 2 + 2 * CH * LP + 2 * P * CH;
    const size_t red = sizeof(float) * CH * Q;
    return ((arrays > red ? arrays : red) + 15) / 16 * 16;
}

// Waves per block: as many as fit beside the shared part (at most 4).
__host__ __device__ inline int net_waves(int L)
{
    const size_t avail = 163840 - kNetShared;
    const int w = (int)(avail / net_wave_bytes(L));
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// tanh from one exponential and one reciprocal: 1 - 2 / (e^{2x} + 1), and the
// odd series x - x^3/3 + 2x^5/15 for |x| < 2^-6 where the difference would
// cancel.  The error (a few ulp of float) is far below the bfloat16 rounding
// of the activations that follows.
__device__ __forceinline__ float tanh_fast(float x)
{
    const float e = __expf(2.0f * x);
    const float t = 1.0f - 2.0f * __frcp_rn(e + 1.0f);
    const float x2 = x * x;
    const float sers = x * (1.0f + x2 * (-1.0f / 3.0f + x2 * (2.0f / 15.0f)));
    return fabsf(x) < 0.015625f ? sers : t;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x4 ld4(const uint16_t* p)
{
    return *reinterpret_cast<const bf16x4*>(p);
}

// Circular halo and zero rows of a position-major [P][32] array holding rows
// 2 .. L+1: rows 0, 1 <- L, L+1; rows L+2, L+3 <- 2, 3; rows >= L+4 <- 0.
// For the position-contiguous copy (when C is not null) the same rows.
__device__ void halo_rows(uint16_t* Pm, uint16_t* Cm, int L, int P, int lane)
{
    const int nrow = P - L;
    for (int idx = lane; idx < CH * nrow; idx += 64) {
        const int c = idx / nrow, h = idx % nrow;
        const int i = h < 2 ? h : L + h;
        uint16_t v = 0;
        if (i < 2) v = Pm[(L + i) * CH + c];
        else if (i < L + 4) v = Pm[(i - L) * CH + c];
        Pm[i * CH + c] = v;
        if (Cm) Cm[c * P + i] = v;
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_net(const float* __restrict__ theta,
                                             const uint64_t* __restrict__ states,
                                             const float* __restrict__ counts, int L, int64_t n,
                                             int64_t ld, float inv_n, float* __restrict__ f_out,
                                             float* __restrict__ partial)
{
    extern __shared__ __align__(16) char smem[];
    const int LP = net_lp(L), P = LP + 4;
    const int nw = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, g4 = lane >> 4;

    NetShared S;
    S.W2R = (uint16_t*)smem;
    S.W2T = S.W2R + CH * Q;
    S.W1 = (float*)(S.W2T + CH * Q);
    S.b1 = S.W1 + Q;
    S.b2 = S.b1 + CH;
    S.w3s = S.b2 + CH;
    char* wbase = smem + kNetShared + (size_t)wv * net_wave_bytes(L);
    NetWave V;
    V.sa = (float*)wbase;
    V.H1P = (uint16_t*)(wbase + ((4 * P + 15) / 16) * 16);
    V.H1C = V.H1P + P * CH;
    V.G2C = V.H1C + CH * P;
    V.G2P = V.G2C + CH * LP;

    for (int i = threadIdx.x; i < CH * Q; i += blockDim.x) {
        const int c = i / Q, rest = i % Q, cp = rest / KS, t = rest % KS;   // W2[c][c'][t]
        const uint16_t v = f2bf(theta[OFF_W2 + i]);
        S.W2R[c * Q + t * CH + cp] = v;
        S.W2T[cp * Q + t * CH + c] = v;
    }
    for (int i = threadIdx.x; i < Q; i += blockDim.x) S.W1[i] = bfr(theta[OFF_W1 + i]);
    for (int c = threadIdx.x; c < CH; c += blockDim.x) {
        S.b1[c] = theta[OFF_B1 + c];
        S.b2[c] = theta[OFF_B2 + c];
        float w = 0.0f;
        for (int t = 0; t < KS; ++t) w += bfr(theta[OFF_W3 + c * KS + t]);
        S.w3s[c] = w;
    }
    __syncthreads();
    const float b3 = theta[OFF_B3], c0 = theta[OFF_C0];

    // per-lane accumulators over the block's samples; the lane's channels are
    // c = mt * 16 + 4 * g4 + v, its weight-gradient columns q = qt * 16 + r
    f32x4 acc[2][10];
    float gW1[2][4][KS], gb1[2][4], gW3[2][4], gb2[2][4];
    float gb3 = 0.0f, gc0 = 0.0f, gloss = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 10; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            gb1[a][v] = gW3[a][v] = gb2[a][v] = 0.0f;
#pragma unroll
            for (int t = 0; t < KS; ++t) gW1[a][v][t] = 0.0f;
        }
    }

    const int64_t stride = (int64_t)gridDim.x * nw;
    for (int64_t smp = (int64_t)blockIdx.x * nw + wv; smp < n; smp += stride) {
        // inputs a = 2 n - 1, circular rows
        for (int i = lane; i < P; i += 64) {
            int site = i - 2;
            site = site < 0 ? site + L : (site >= L ? site - L : site);
            float v = 0.0f;
            if (i < L + 4)
                v = ((states[(int64_t)(site >> 6) * ld + smp] >> (site & 63)) & 1ull) ? 1.0f : -1.0f;
            V.sa[i] = v;
        }
        wave_sync();
        // layer 1
        for (int j = lane; j < L; j += 64) {
            float a5[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) a5[t] = V.sa[j + t];
            for (int c = 0; c < CH; ++c) {
                float z = S.b1[c];
#pragma unroll
                for (int t = 0; t < KS; ++t) z += S.W1[c * KS + t] * a5[t];
                const uint16_t hb = f2bf(tanh_fast(z));
                V.H1P[(j + 2) * CH + c] = hb;
                V.H1C[c * P + j + 2] = hb;
            }
        }
        wave_sync();
        halo_rows(V.H1P, V.H1C, L, P, lane);
        wave_sync();
        // layer 2 and 3: both channel tiles of a position tile share each B operand
        float fpart = 0.0f;
        float s2p[2][4], g2p[2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) s2p[mt][v] = g2p[mt][v] = 0.0f;
        for (int nt = 0; nt < LP / 16; ++nt) {
            const int j = nt * 16 + r;
            f32x4 z[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
            for (int kt = 0; kt < Q / 16; ++kt) {
                const int t = kt >> 1, cb = (kt & 1) * 16 + 4 * g4;
                const bf16x4 B = ld4(V.H1P + (j + t) * CH + cb);
                z[0] = mfma16(ld4(S.W2R + r * Q + kt * 16 + 4 * g4), B, z[0]);
                z[1] = mfma16(ld4(S.W2R + (16 + r) * Q + kt * 16 + 4 * g4), B, z[1]);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = mt * 16 + 4 * g4 + v;
                    uint16_t gb = 0;
                    if (j < L) {
                        const float h2 = tanh_fast(z[mt][v] + S.b2[c]);
                        const float g2 = S.w3s[c] * (1.0f - h2 * h2);
                        fpart += S.w3s[c] * h2;
                        s2p[mt][v] += h2;
                        g2p[mt][v] += g2;
                        gb = f2bf(g2);
                        V.G2P[(j + 2) * CH + c] = gb;
                    }
                    V.G2C[c * LP + j] = gb;
                }
        }
        const float f = (float)L * b3 + wave_reduce(fpart, OpSum());
        if (MODE == 0) {
            if (lane == 0) f_out[smp] = f;
            wave_sync();
            continue;
        }
        const float cnt = counts[smp];
        const float zf = f + c0, ez = expf(zf);
        const float delta = (ez - cnt) * inv_n;
        if (lane == 0) {
            gb3 += delta * (float)L;
            gc0 += delta;
            gloss += (ez - cnt * zf) * inv_n;
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                gW3[mt][v] += delta * s2p[mt][v];
                gb2[mt][v] += delta * g2p[mt][v];
            }
        wave_sync();
        halo_rows(V.G2P, nullptr, L, P, lane);
        wave_sync();
        // weight gradient of layer 2: sum over positions of g2[c][j] h1[c'][j + t - 2]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int qt = 0; qt < 10; ++qt) {
                const int q = qt * 16 + r, t = q >> 5, cp = q & 31;
                f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int jt = 0; jt < LP / 16; ++jt) {
                    const int j0 = jt * 16 + 4 * g4;
                    const uint16_t* hb = V.H1C + cp * P + j0 + t;
                    bf16x4 B;
                    B[0] = (short)hb[0];
                    B[1] = (short)hb[1];
                    B[2] = (short)hb[2];
                    B[3] = (short)hb[3];
                    d = mfma16(ld4(V.G2C + (mt * 16 + r) * LP + j0), B, d);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[mt][qt][v] += delta * d[v];
            }
        // input gradient of layer 2, then layer 1 (both channel tiles per B operand)
        for (int nt = 0; nt < LP / 16; ++nt) {
            const int j = nt * 16 + r;
            f32x4 d[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
            for (int kt = 0; kt < Q / 16; ++kt) {
                const int t = kt >> 1, cb = (kt & 1) * 16 + 4 * g4;
                const bf16x4 B = ld4(V.G2P + (j - t + 4) * CH + cb);
                d[0] = mfma16(ld4(S.W2T + r * Q + kt * 16 + 4 * g4), B, d[0]);
                d[1] = mfma16(ld4(S.W2T + (16 + r) * Q + kt * 16 + 4 * g4), B, d[1]);
            }
            if (j < L) {
                float a5[KS];
#pragma unroll
                for (int t = 0; t < KS; ++t) a5[t] = V.sa[j + t];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int c = mt * 16 + 4 * g4 + v;
                        float z = S.b1[c];
#pragma unroll
                        for (int t = 0; t < KS; ++t) z += S.W1[c * KS + t] * a5[t];
                        const float h = tanh_fast(z);
                        const float dz1 = delta * d[mt][v] * (1.0f - h * h);
                        gb1[mt][v] += dz1;
#pragma unroll
                        for (int t = 0; t < KS; ++t) gW1[mt][v][t] += dz1 * a5[t];
                    }
            }
        }
        wave_sync();
    }
    if (MODE == 0) return;

    // Block sums in a fixed order (no atomics, so the result is reproducible):
    // first the layer-2 weight gradient, then the small parameters, each
    // through the per-wave regions.
    __syncthreads();   // every wave is done with its region
    float* red = (float*)wbase;   // at least CH * Q floats per wave
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int qt = 0; qt < 10; ++qt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = mt * 16 + 4 * g4 + v, q = qt * 16 + r;
                red[c * Q + q] = acc[mt][qt][v];
            }
    __syncthreads();
    float* out = partial + (int64_t)blockIdx.x * (kGuideParams + 1);
    for (int i = threadIdx.x; i < CH * Q; i += blockDim.x) {
        const int c = i / Q, q = i % Q, t = q >> 5, cp = q & 31;
        float sum = 0.0f;
        for (int w = 0; w < nw; ++w)
            sum += ((const float*)(smem + kNetShared + (size_t)w * net_wave_bytes(L)))[i];
        out[OFF_W2 + c * Q + cp * KS + t] = sum;
    }
    __syncthreads();
    // small parameters: lane l of a wave writes its 8 channels x 8 slots
    // (5 taps of W1, b1, b2, W3) at red[l * 64 + (mt * 4 + v) * 8 + slot] and
    // its scalars at red[4096 + l * 3 + k]
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float* o = red + lane * 64 + (mt * 4 + v) * 8;
#pragma unroll
            for (int t = 0; t < KS; ++t) o[t] = gW1[mt][v][t];
            o[5] = gb1[mt][v];
            o[6] = gb2[mt][v];
            o[7] = gW3[mt][v];
        }
    red[4096 + lane * 3 + 0] = gb3;
    red[4096 + lane * 3 + 1] = gc0;
    red[4096 + lane * 3 + 2] = gloss;
    __syncthreads();
    // channel c = mt * 16 + 4 * g4 + v lives in lanes g4 * 16 + r, r = 0..15
    for (int i = threadIdx.x; i < CH * 8; i += blockDim.x) {
        const int c = i >> 3, slot = i & 7;
        const int mt = c >> 4, g = (c >> 2) & 3, v = c & 3;
        float sum = 0.0f;
        for (int w = 0; w < nw; ++w) {
            const float* R = (const float*)(smem + kNetShared + (size_t)w * net_wave_bytes(L));
            for (int rr = 0; rr < 16; ++rr) sum += R[(g * 16 + rr) * 64 + (mt * 4 + v) * 8 + slot];
        }
        if (slot < KS) out[OFF_W1 + c * KS + slot] = sum;
        else if (slot == 5) out[OFF_B1 + c] = sum;
        else if (slot == 6) out[OFF_B2 + c] = sum;
        else for (int t = 0; t < KS; ++t) out[OFF_W3 + c * KS + t] = sum;
    }
    if (threadIdx.x < 3) {
        float sum = 0.0f;
        for (int w = 0; w < nw; ++w) {
            const float* R = (const float*)(smem + kNetShared + (size_t)w * net_wave_bytes(L));
            sum += R[4096 + threadIdx.x];   // lane 0 of each wave holds the scalars
        }
        out[threadIdx.x == 0 ? OFF_B3 : (threadIdx.x == 1 ? OFF_C0 : kGuideParams)] = sum;
    }
}

// Sum of the per-block partials: 16 parameters per block, 16 lanes per
// parameter each summing every 16th block in double precision, then the 16
// lane sums combined in a fixed order.
__global__ __launch_bounds__(256) void k_net_reduce(const float* __restrict__ partial, int blocks,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss)
{
    __shared__ double s[16][17];
    const int pl = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int p = blockIdx.x * 16 + pl;
    double acc = 0.0;
    if (p <= kGuideParams)
        for (int b = part; b < blocks; b += 16) acc += partial[(int64_t)b * (kGuideParams + 1) + p];
    s[pl][part] = acc;
    __syncthreads();
    if (part == 0 && p <= kGuideParams) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += s[pl][k];
        if (p < kGuideParams) grad[p] = (float)t;
        else if (loss) *loss = (float)t;
    }
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float bc1, float bc2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kGuideParams) return;
    const float g = grad[p];
    const float mm = 0.9f * m[p] + 0.1f * g;
    const float vv = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// Window table: h(w) for all 8192 windows of 13 sites (site c-6 in bit 0), the
// net evaluated on the window alone (valid convolutions 13 -> 9 -> 5 -> 1).
// One wave per 16 windows; layer 2 is a 32 x 160 x 80 MFMA contraction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_window_table(const float* __restrict__ theta,
                                                     float* __restrict__ table)
{
    __shared__ uint16_t sW2[CH * Q];
    __shared__ float sW1[Q], sb1[CH], sb2[CH], sW3[Q];
    __shared__ float sh1[16][CH][9];
    __shared__ float sh2[16][CH][5];
    const int lane = threadIdx.x;
    for (int i = lane; i < CH * Q; i += 64) sW2[i] = f2bf(theta[OFF_W2 + i]);
    for (int i = lane; i < Q; i += 64) {
        sW1[i] = bfr(theta[OFF_W1 + i]);
        sW3[i] = bfr(theta[OFF_W3 + i]);
    }
    for (int c = lane; c < CH; c += 64) {
        sb1[c] = theta[OFF_B1 + c];
        sb2[c] = theta[OFF_B2 + c];
    }
    __syncthreads();
    const int w0 = blockIdx.x * 16;
    for (int idx = lane; idx < 16 * CH * 9; idx += 64) {
        const int w = idx / (CH * 9), c = (idx / 9) % CH, p = idx % 9;
        float z = sb1[c];
#pragma unroll
        for (int k = 0; k < KS; ++k)
            z += sW1[c * KS + k] * ((((w0 + w) >> (p + k)) & 1) ? 1.0f : -1.0f);
        sh1[w][c][p] = tanhf(z);
    }
    __syncthreads();
    const int r = lane & 15, g4 = lane >> 4;
    for (int mt = 0; mt < 2; ++mt)
        for (int nt = 0; nt < 5; ++nt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            const int col = nt * 16 + r, w = col / 5, p2 = col % 5;
            for (int kt = 0; kt < Q / 16; ++kt) {
                bf16x4 A, B;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = kt * 16 + 4 * g4 + v;
                    A[v] = (short)sW2[(mt * 16 + r) * Q + q];
                    B[v] = (short)f2bf(sh1[w][q / KS][p2 + q % KS]);
                }
                acc = mfma16(A, B, acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = mt * 16 + 4 * g4 + v;
                sh2[w][c][p2] = tanhf(acc[v] + sb2[c]);
            }
        }
    __syncthreads();
    if (lane < 16) {
        float o = theta[OFF_B3];
        for (int c = 0; c < CH; ++c)
#pragma unroll
            for (int k = 0; k < KS; ++k) o += sW3[c * KS + k] * sh2[lane][c][k];
        table[w0 + lane] = o;
    }
}

// ---------------------------------------------------------------------------
// Bond table: for an allowed neighbourhood u of bond b (sites b-6..b+6), the
// log-ratio f(C after the hop) - f(C) = sum over the 14 windows holding b or
// b+1 of h(after) - h(before), averaged over the 13 outer sites b-12..b-7 and
// b+7..b+13 (all 8192 settings, equally weighted), clipped to [-gmax, gmax]:
// eg[u] = rint(2^16 exp(G)).  One block per neighbourhood.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bond_table(const float* __restrict__ H, double gmax,
                                                    uint32_t* __restrict__ eg,
                                                    double* __restrict__ G_out)
{
    __shared__ float sH[8192];
    __shared__ double sred[4];
    const int u = blockIdx.x;
    const bool allowed = ((u >> 6) ^ (u >> 7)) & 1;
    if (!allowed) {
        if (threadIdx.x == 0) {
            eg[u] = 0;
            if (G_out) G_out[u] = 0.0;
        }
        return;
    }
    for (int i = threadIdx.x; i < 8192; i += 256) sH[i] = H[i];
    __syncthreads();
    double d = 0.0;
    for (int ctx = threadIdx.x; ctx < 8192; ctx += 256) {
        const uint32_t s0 = (uint32_t)(ctx & 0x3F) | ((uint32_t)u << 6) | ((uint32_t)(ctx >> 6) << 19);
        const uint32_t s1 = s0 ^ (3u << 12);
        double e = 0.0;
#pragma unroll
        for (int o = 0; o < 14; ++o)
            e += (double)sH[(s1 >> o) & 0x1FFF] - (double)sH[(s0 >> o) & 0x1FFF];
        d += e;
    }
    d = wave_reduce(d, OpSum());
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double G = ((sred[0] + sred[1]) + (sred[2] + sred[3])) / 8192.0;
        if (G_out) G_out[u] = G;
        eg[u] = (uint32_t)rint(65536.0 * exp(fmin(fmax(G, -gmax), gmax)));
    }
}

// ---------------------------------------------------------------------------
// Bond table conditioned on data: for every configuration of a sample set and
// every allowed bond b, d = f(C after the hop) - f(C), exactly the 14 windows
// holding b or b+1 after minus before (the ring has L >= 26 sites, so those
// windows span 26 distinct sites b-12..b+13); d is summed per neighbourhood u
// (sites b-6..b+6).  Sums and counts are privatised per block in LDS and then
// added to the global accumulators.
// ---------------------------------------------------------------------------
constexpr int kStatThreads = 256;
constexpr size_t kStatSmem = 8192 * (sizeof(float) + sizeof(double) + sizeof(uint32_t));

template <int W>
__global__ __launch_bounds__(kStatThreads) void k_bond_stats(const float* __restrict__ H,
                                                             const uint64_t* __restrict__ states,
                                                             int64_t ld, int L, int64_t n,
                                                             double* __restrict__ sums,
                                                             uint32_t* __restrict__ counts)
{
    extern __shared__ __align__(16) char smem[];
    double* s_sum = (double*)smem;
    float* s_H = (float*)(s_sum + 8192);
    uint32_t* s_cnt = (uint32_t*)(s_H + 8192);
    for (int i = threadIdx.x; i < 8192; i += kStatThreads) {
        s_sum[i] = 0.0;
        s_cnt[i] = 0u;
        s_H[i] = H[i];
    }
    __syncthreads();
    const int lb = (L - 1) & 63;
    for (int64_t i = (int64_t)blockIdx.x * kStatThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kStatThreads) {
        uint64_t x[W], m[W];
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = states[w * ld + i];
        bond_mask<W>(x, lb, m);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint64_t bits = m[w];
            while (bits) {
                const int b = w * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
                const uint32_t w0 = ring_bits<W>(x, L, b >= 12 ? b - 12 : b - 12 + L, 26);
                const uint32_t w1 = w0 ^ (3u << 12);
                double d = 0.0;
#pragma unroll
                for (int o = 0; o < 14; ++o)
                    d += ((double)s_H[(w1 >> o) & 0x1FFFu] - (double)s_H[(w0 >> o) & 0x1FFFu]);
                const uint32_t u = (w0 >> 6) & 0x1FFFu;
                atomicAdd(&s_sum[u], d);
                atomicAdd(&s_cnt[u], 1u);
            }
        }
    }
    __syncthreads();
    for (int u = threadIdx.x; u < 8192; u += kStatThreads)
        if (s_cnt[u]) {
            atomicAdd(&sums[u], s_sum[u]);
            atomicAdd(&counts[u], s_cnt[u]);
        }
}

__global__ void k_zero_stats(double* __restrict__ sums, uint32_t* __restrict__ counts)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < 8192) {
        sums[u] = 0.0;
        counts[u] = 0u;
    }
}

// G = mean where the neighbourhood was seen at least min_count times, else the
// uniform-context value already in G; then the clipped integer table.
__global__ void k_cond_finish(const double* __restrict__ sums, const uint32_t* __restrict__ counts,
                              uint32_t min_count, double gmax, double* __restrict__ G,
                              uint32_t* __restrict__ eg, uint32_t* __restrict__ counts_out)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= 8192) return;
    const uint32_t c = counts[u];
    if (counts_out) counts_out[u] = c;
    if (!((u >> 6 ^ u >> 7) & 1)) return;   // k_bond_table wrote 0 to eg and G
    double g = G[u];
    if (c >= min_count) g = sums[u] / (double)c;
    G[u] = g;
    eg[u] = (uint32_t)rint(65536.0 * exp(fmin(fmax(g, -gmax), gmax)));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int guide_blocks(int64_t n) { return (int)(n < kGuideBlocks ? n : kGuideBlocks); }

static size_t net_block_smem(int L) { return kNetShared + net_waves(L) * net_wave_bytes(L); }

hipError_t launch_net(int mode, const float* theta, const uint64_t* states, int64_t ld,
                      const float* counts, int L, int64_t n, float* f_out, float* partial,
                      float* grad, float* loss, hipStream_t st)
{
    const int nw = net_waves(L);
    const int64_t want = (n + nw - 1) / nw;
    const int blocks = (int)(want < 512 ? want : 512);   // <= guide_blocks(n): fits the workspace
    const size_t sm = net_block_smem(L);
    if (mode == 0) {
        hipLaunchKernelGGL(k_net<0>, dim3(blocks), dim3(64 * nw), sm, st, theta, states, counts,
                           L, n, ld, 1.0f / (float)n, f_out, partial);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_net<1>, dim3(blocks), dim3(64 * nw), sm, st, theta, states, counts, L, n,
                       ld, 1.0f / (float)n, f_out, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_net_reduce, dim3((kGuideParams + 1 + 15) / 16), dim3(256), 0, st,
                       partial, blocks, grad, loss);
    return hipGetLastError();
}

hipError_t net_set_smem_limit(int L)
{
    (void)L;
    const int sm = 163840;
    hipError_t e = hipFuncSetAttribute((const void*)k_net<0>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, sm);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_net<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               sm);
}

size_t net_smem(int L) { return net_block_smem(L); }

hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int step, float lr,
                       hipStream_t st)
{
    const float bc1 = 1.0f - powf(0.9f, (float)step);
    const float bc2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kGuideParams + 255) / 256), dim3(256), 0, st, theta, m, v,
                       grad, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_window_table(const float* theta, float* table, hipStream_t st)
{
    hipLaunchKernelGGL(k_window_table, dim3(8192 / 16), dim3(64), 0, st, theta, table);
    return hipGetLastError();
}

hipError_t launch_bond_table_cond(const float* H, const uint64_t* states, int64_t ld, int L,
                                  int64_t n, uint32_t min_count, double gmax, uint32_t* eg,
                                  double* G, uint32_t* counts_out, void* work, hipStream_t st)
{
    double* sums = (double*)work;
    uint32_t* counts = (uint32_t*)(sums + 8192);
    double* Gw = G ? G : (double*)(counts + 8192);
    hipLaunchKernelGGL(k_bond_table, dim3(8192), dim3(256), 0, st, H, gmax, eg, Gw);
    hipLaunchKernelGGL(k_zero_stats, dim3(32), dim3(256), 0, st, sums, counts);
    const int64_t want = (n + kStatThreads - 1) / kStatThreads;
    const int blocks = (int)(want < 512 ? want : 512);
    switch ((L + 63) / 64) {
#define PD_STATS(w)                                                                          \
    case w:                                                                                  \
        hipLaunchKernelGGL(k_bond_stats<w>, dim3(blocks), dim3(kStatThreads), kStatSmem, st, \
                           H, states, ld, L, n, sums, counts);                               \
        break;
        PD_STATS(1) PD_STATS(2) PD_STATS(3) PD_STATS(4) PD_STATS(5) PD_STATS(6) PD_STATS(7)
        PD_STATS(8)
#undef PD_STATS
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_cond_finish, dim3(32), dim3(256), 0, st, sums, counts, min_count, gmax,
                       Gw, eg, counts_out);
    return hipGetLastError();
}

hipError_t stats_set_smem_limit()
{
#define PD_ATTR(w)                                                                           \
    {                                                                                        \
        hipError_t e = hipFuncSetAttribute((const void*)k_bond_stats<w>,                     \
                                           hipFuncAttributeMaxDynamicSharedMemorySize,       \
                                           (int)kStatSmem);                                  \
        if (e != hipSuccess) return e;                                                       \
    }
    PD_ATTR(1) PD_ATTR(2) PD_ATTR(3) PD_ATTR(4) PD_ATTR(5) PD_ATTR(6) PD_ATTR(7) PD_ATTR(8)
#undef PD_ATTR
    return hipSuccess;
}

hipError_t launch_bond_table(const float* H, double gmax, uint32_t* eg, double* G, hipStream_t st)
{
    hipLaunchKernelGGL(k_bond_table, dim3(8192), dim3(256), 0, st, H, gmax, eg, G);
    return hipGetLastError();
}

}  // namespace pd
