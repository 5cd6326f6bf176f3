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

struct NetSmem {
    uint16_t* W2;    // [32][160]  W2[c][c'*5+k]
    uint16_t* W2T;   // [32][160]  W2T[c'][c*5+k] = W2[c][c'][k]
    float* W1;       // [160] (bf16 values)
    float* b1;       // [32]
    float* b2;       // [32]
    float* w3s;      // [32]  sum_k W3[c][k] (bf16 values)
    float* a;        // [LP + 4]  a_{i-2}
    float* h1;       // [32][LP + 4]  h1[c][i-2] (later dz1)
    float* h2;       // [32][LP + 4]  h2[c][i-2] (later dz2)
    float* g;        // partial gradient of the small parameters + loss
};

// Per-block sums of the small parameters' gradients (g below):
//   [0,160) W1 | [160,192) b1 | [192,224) b2 | [224,256) S2 = sum_j h2[c][j] of the
//   current sample | [256,288) sum over samples of delta S2 (the W3 gradient, equal
//   for the 5 taps) | 288 b3 | 289 c0 | 290 loss
constexpr int kSmallGrad = 291;

__host__ __device__ inline size_t net_smem_bytes(int L)
{
    const int LP = (L + 15) / 16 * 16;
    return 2 * (size_t)CH * Q * 2 + sizeof(float) * ((size_t)Q + 3 * CH + (LP + 4) +
                                                     2 * (size_t)CH * (LP + 4) + kSmallGrad);
}

__device__ NetSmem carve(char* base, int L)
{
    const int LP = (L + 15) / 16 * 16;
    NetSmem s;
    s.W2 = (uint16_t*)base;
    s.W2T = s.W2 + CH * Q;
    float* f = (float*)(s.W2T + CH * Q);
    s.W1 = f; f += Q;
    s.b1 = f; f += CH;
    s.b2 = f; f += CH;
    s.w3s = f; f += CH;
    s.a = f; f += LP + 4;
    s.h1 = f; f += CH * (LP + 4);
    s.h2 = f; f += CH * (LP + 4);
    s.g = f;
    return s;
}

__device__ void load_weights(const float* __restrict__ theta, const NetSmem& s, bool transpose)
{
    const int t = threadIdx.x;
    for (int i = t; i < CH * Q; i += blockDim.x) {
        const int c = i / Q, q = i % Q;              // q = c'*5 + k
        const uint16_t v = f2bf(theta[OFF_W2 + i]);
        s.W2[i] = v;
        if (transpose) {
            const int cp = q / KS, k = q % KS;
            s.W2T[cp * Q + c * KS + k] = v;
        }
    }
    for (int i = t; i < Q; i += blockDim.x) s.W1[i] = bfr(theta[OFF_W1 + i]);
    for (int c = t; c < CH; c += blockDim.x) {
        s.b1[c] = theta[OFF_B1 + c];
        s.b2[c] = theta[OFF_B2 + c];
        float w = 0.0f;
        for (int k = 0; k < KS; ++k) w += bfr(theta[OFF_W3 + c * KS + k]);
        s.w3s[c] = w;
    }
}

// Circular halo of a [32][LP+4] array holding x[c][i-2] for i in [2, L+2):
// columns 0,1 <- x[L-2], x[L-1]; L+2, L+3 <- x[0], x[1]; further columns 0.
__device__ void halo(float* x, int L, int LP)
{
    const int W = LP + 4;
    for (int idx = threadIdx.x; idx < CH * (W - L); idx += blockDim.x) {
        const int c = idx / (W - L), h = idx % (W - L);
        float* row = x + c * W;
        if (h == 0) row[0] = row[L];
        else if (h == 1) row[1] = row[L + 1];
        else if (h == 2) row[L + 2] = row[2];
        else if (h == 3) row[L + 3] = row[3];
        else row[L + h] = 0.0f;
    }
}

// Forward pass of one sample (its occupancy bits in words[w * stride]); f is
// returned to every thread.  Block = one wave.
__device__ float net_forward(const NetSmem& s, const uint64_t* __restrict__ words, int64_t stride,
                             int L, float b3)
{
    const int LP = (L + 15) / 16 * 16, W = LP + 4;
    const int lane = threadIdx.x;
    for (int i = lane; i < W; i += 64) {
        int site = i - 2;
        site = site < 0 ? site + L : (site >= L ? site - L : site);
        float v = 0.0f;
        if (i < L + 4) v = ((words[(int64_t)(site >> 6) * stride] >> (site & 63)) & 1ull) ? 1.0f : -1.0f;
        s.a[i] = v;
    }
    __syncthreads();
    for (int idx = lane; idx < CH * L; idx += 64) {
        const int c = idx / L, j = idx % L;
        float z = s.b1[c];
#pragma unroll
        for (int k = 0; k < KS; ++k) z += s.W1[c * KS + k] * s.a[j + k];
        s.h1[c * W + j + 2] = tanhf(z);
    }
    __syncthreads();
    halo(s.h1, L, LP);
    __syncthreads();
    const int r = lane & 15, g4 = lane >> 4;
    for (int mt = 0; mt < 2; ++mt)
        for (int nt = 0; nt < LP / 16; ++nt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            const int j = nt * 16 + r;
            for (int kt = 0; kt < Q / 16; ++kt) {
                const int q0 = kt * 16 + 4 * g4;
                bf16x4 A, B;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = q0 + v;
                    A[v] = (short)s.W2[(mt * 16 + r) * Q + q];
                    B[v] = (short)f2bf(s.h1[(q / KS) * W + j + q % KS]);
                }
                acc = mfma16(A, B, acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = mt * 16 + 4 * g4 + v;
                if (j < L) s.h2[c * W + j + 2] = tanhf(acc[v] + s.b2[c]);
            }
        }
    __syncthreads();
    halo(s.h2, L, LP);
    __syncthreads();
    // f = L b3 + sum_c (sum_k W3[c][k]) (sum_j h2[c][j])
    float part = 0.0f;
    if (lane < CH) {
        float S2 = 0.0f;
        for (int j = 0; j < L; ++j) S2 += s.h2[lane * W + j + 2];
        part = s.w3s[lane] * S2;
        s.g[CH * KS + 2 * CH + lane] = S2;     // kept for the W3 gradient
    }
    part = wave_reduce(part, OpSum());
    return (float)L * b3 + part;
}

// Gradient pass of one sample given delta = d loss / d f; layer-2 weight
// gradient accumulates into acc (2 x 10 tiles of 16 x 16, MFMA layout).
__device__ void net_backward(const NetSmem& s, int L, float delta, f32x4 (&acc)[2][10])
{
    const int LP = (L + 15) / 16 * 16, W = LP + 4;
    const int lane = threadIdx.x;
    const int r = lane & 15, g4 = lane >> 4;
    // dz2 = delta * w3s[c] * (1 - h2^2), in place of h2
    for (int idx = lane; idx < CH * L; idx += 64) {
        const int c = idx / L, j = idx % L;
        const float h = s.h2[c * W + j + 2];
        s.h2[c * W + j + 2] = delta * s.w3s[c] * (1.0f - h * h);
    }
    __syncthreads();
    halo(s.h2, L, LP);
    __syncthreads();
    // dW2[c][q] += sum_j dz2[c][j] X[q][j],  X[q][j] = h1[q/5][j + q%5 - 2]
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int qt = 0; qt < Q / 16; ++qt) {
            const int q = qt * 16 + r;
            for (int jt = 0; jt < LP / 16; ++jt) {
                bf16x4 A, B;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = jt * 16 + 4 * g4 + v;
                    const float dz = j < L ? s.h2[(mt * 16 + r) * W + j + 2] : 0.0f;
                    A[v] = (short)f2bf(dz);
                    B[v] = (short)f2bf(s.h1[(q / KS) * W + j + q % KS]);
                }
                acc[mt][qt] = mfma16(A, B, acc[mt][qt]);
            }
        }
    // small gradients of this sample
    if (lane < CH) {
        float db2 = 0.0f;
        for (int j = 0; j < L; ++j) db2 += s.h2[lane * W + j + 2];
        s.g[CH * KS + CH + lane] += db2;                       // b2
    }
    // dh1[c'][j] = sum_{c,k} W2[c][c'][k] dz2[c][j-k+2]; dz1 = dh1 (1 - h1^2) in place of h1
    __syncthreads();
    for (int mt = 0; mt < 2; ++mt)
        for (int nt = 0; nt < LP / 16; ++nt) {
            f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
            const int j = nt * 16 + r;
            for (int kt = 0; kt < Q / 16; ++kt) {
                const int p0 = kt * 16 + 4 * g4;
                bf16x4 A, B;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int p = p0 + v;
                    A[v] = (short)s.W2T[(mt * 16 + r) * Q + p];
                    B[v] = (short)f2bf(s.h2[(p / KS) * W + j - p % KS + 4]);
                }
                d = mfma16(A, B, d);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = mt * 16 + 4 * g4 + v;
                if (j < L) {
                    const float h = s.h1[c * W + j + 2];
                    s.h1[c * W + j + 2] = d[v] * (1.0f - h * h);
                }
            }
        }
    __syncthreads();
    for (int idx = lane; idx < CH * KS; idx += 64) {
        const int c = idx / KS, k = idx % KS;
        float acc1 = 0.0f;
        for (int j = 0; j < L; ++j) acc1 += s.h1[c * W + j + 2] * s.a[j + k];
        s.g[idx] += acc1;                                      // W1
    }
    if (lane < CH) {
        float db1 = 0.0f;
        for (int j = 0; j < L; ++j) db1 += s.h1[lane * W + j + 2];
        s.g[CH * KS + lane] += db1;                            // b1
    }
    __syncthreads();
}

// mode 0: f of every sample; mode 1: loss and gradient partial sums per block.
template <int MODE>
__global__ __launch_bounds__(64) void k_net(const float* __restrict__ theta,
                                            const uint64_t* __restrict__ states,
                                            const float* __restrict__ counts, int L, int64_t n,
                                            int64_t ld, float inv_n, float* __restrict__ f_out,
                                            float* __restrict__ partial)
{
    extern __shared__ __align__(16) char smem[];
    const NetSmem s = carve(smem, L);
    load_weights(theta, s, MODE == 1);
    const float b3 = theta[OFF_B3];
    const float c0 = theta[OFF_C0];
    const int lane = threadIdx.x;
    for (int i = lane; i < kSmallGrad; i += 64) s.g[i] = 0.0f;
    __syncthreads();
    f32x4 acc[2][10];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 10; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const float f = net_forward(s, states + i, ld, L, b3);
        if (MODE == 0) {
            if (lane == 0) f_out[i] = f;
            __syncthreads();
            continue;
        }
        const float cnt = counts[i];
        const float ez = expf(f + c0);
        const float delta = (ez - cnt) * inv_n;
        if (lane < CH) s.g[256 + lane] += delta * s.g[224 + lane];
        if (lane == 0) {
            s.g[288] += delta * (float)L;
            s.g[289] += delta;
            s.g[290] += (ez - cnt * (f + c0)) * inv_n;
        }
        __syncthreads();
        net_backward(s, L, delta, acc);
    }
    if (MODE == 0) return;
    float* out = partial + (int64_t)blockIdx.x * (kGuideParams + 1);
    const int r = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int qt = 0; qt < 10; ++qt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = mt * 16 + 4 * g4 + v, q = qt * 16 + r;
                out[OFF_W2 + c * Q + q] = acc[mt][qt][v];
            }
    for (int i = lane; i < CH * KS; i += 64) out[OFF_W1 + i] = s.g[i];
    for (int c = lane; c < CH; c += 64) {
        out[OFF_B1 + c] = s.g[160 + c];
        out[OFF_B2 + c] = s.g[192 + c];
        for (int k = 0; k < KS; ++k) out[OFF_W3 + c * KS + k] = s.g[256 + c];
    }
    if (lane == 0) {
        out[OFF_B3] = s.g[288];
        out[OFF_C0] = s.g[289];
        out[kGuideParams] = s.g[290];
    }
}

__global__ void k_net_reduce(const float* __restrict__ partial, int blocks,
                             float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kGuideParams) return;
    double acc = 0.0;
    for (int b = 0; b < blocks; ++b) acc += partial[(int64_t)b * (kGuideParams + 1) + p];
    if (p < kGuideParams) grad[p] = (float)acc;
    else if (loss) *loss = (float)acc;
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

hipError_t launch_net(int mode, const float* theta, const uint64_t* states, int64_t ld,
                      const float* counts, int L, int64_t n, float* f_out, float* partial,
                      float* grad, float* loss, hipStream_t st)
{
    const int blocks = guide_blocks(n);
    const size_t sm = net_smem_bytes(L);
    if (mode == 0) {
        hipLaunchKernelGGL(k_net<0>, dim3(blocks), dim3(64), sm, st, theta, states, counts, L, n,
                           ld, 1.0f / (float)n, f_out, partial);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_net<1>, dim3(blocks), dim3(64), sm, st, theta, states, counts, L, n,
                       ld, 1.0f / (float)n, f_out, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_net_reduce, dim3((kGuideParams + 1 + 255) / 256), dim3(256), 0, st,
                       partial, blocks, grad, loss);
    return hipGetLastError();
}

hipError_t net_set_smem_limit(int L)
{
    const size_t sm = net_smem_bytes(L);
    hipError_t e = hipFuncSetAttribute((const void*)k_net<0>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_net<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sm);
}

size_t net_smem(int L) { return net_smem_bytes(L); }

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
