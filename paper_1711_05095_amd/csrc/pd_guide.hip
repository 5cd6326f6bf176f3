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
// what Adam updates, biases stay FP32); the 32 x 160 x L contractions of
// layer 2 (forward, the weight gradient and the input gradient) and layer 1
// (exact: its inputs are +-1; in the training kernel over its 32 possible
// input windows, once per block) run on the matrix cores in bf16 with FP32
// accumulation; layer 3 and the activations run on the vector ALU in FP32.
#include <hip/hip_runtime.h>

#include <atomic>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_guide.hpp"
#include "pd_internal.hpp"

namespace pd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row strides chosen so that the operand reads of a wave spread over all LDS
// banks: W2R / W2T rows of WS halves (336 bytes) and position-major rows of RS
// halves (80 bytes) put 8 consecutive rows of a 16-byte read on 8 disjoint
// 16-byte bank groups; channel-major rows of P = LP + 4 halves (2 x odd
// dwords) do the same for the 8-byte reads of the weight-gradient pass.
constexpr int WS = 168, RS = 40;
constexpr int kWindows = 32;        // input windows of layer 1 (5 sites of +-1)
constexpr int kNetShared = 2 * CH * WS * 2 + 4 * (3 * CH) + kWindows * CH * (4 + 2);  // bytes

struct NetShared {
    uint16_t* W2R;   // [c][t * 32 + c']  = W2[c][c'][t]   (row stride WS)
    uint16_t* W2T;   // [c'][t * 32 + c]  = W2[c][c'][t]   (row stride WS)
    float* b1;
    float* b2;
    float* w3s;      // sum_t W3[c][t] (bf16 values)
    float* D1;       // [w][2 r + mt]: 1 - h1^2 of channel mt * 16 + r at input window w
    uint16_t* T1;    // [w][2 r + mt]: h1 (bfloat16) of channel mt * 16 + r at input window w
};

__host__ __device__ inline int net_lp(int L) { return (L + 15) / 16 * 16; }

// The inputs a = 2 n - 1 of a sample as a circular bit string: bit i is
// site (i - 4) mod L, so that the 5-site window of layer 1 at row R (site
// R - 2) is bits R .. R + 4.  Rows up to LP + 1 are evaluated, each reading
// the 32-bit window at its row, and the W1 gradient reads windows from rows up
// to LP + 13 (two 32-bit words from word R / 32).
__host__ __device__ inline int net_ext_words(int L)
{
    return (32 * (((net_lp(L) + 13) >> 5) + 2) + 63) / 64;
}
__host__ __device__ inline size_t net_ext_bytes(int L) { return (8 * net_ext_words(L) + 15) / 16 * 16; }

// Bytes of one wave's region: the bit string, the position-major array (h1,
// then g2 once the forward pass is past a row), the channel-major h1, and at
// least the 16 x 160 floats of one half of the end-of-block reduction.
__host__ __device__ inline size_t net_wave_bytes(int L)
{
    const size_t LP = net_lp(L), P = LP + 4;
    const size_t arrays = net_ext_bytes(L) + P * RS * 2 + CH * P * 2;
    const size_t red = sizeof(float) * 16 * Q;
    return ((arrays > red ? arrays : red) + 15) / 16 * 16;
}

// Waves per block: as many as fit beside the shared part (at most 8: two
// waves per SIMD, the most the kernel's 256 registers allow).
__host__ __device__ inline int net_waves(int L)
{
    const size_t avail = 163840 - kNetShared;
    const int w = (int)(avail / net_wave_bytes(L));
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// tanh(x) = 1 - 2 / (e^{2x} + 1) from the hardware base-2 exponential and
// reciprocal (each within about 1 ulp): absolute error a few 1e-7 for every
// x, saturating to +-1 for large |x|.  Near 0 the relative error grows, but
// the absolute one stays far below the bfloat16 quantum of the activations
// and below what float32 accumulation of the network's sums adds.
__device__ __forceinline__ float tanh_fast(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);   // e^{2x}
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
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
__device__ __forceinline__ bf16x8 ld8(const uint16_t* p)
{
    return *reinterpret_cast<const bf16x8*>(p);
}
__device__ __forceinline__ bf16x4 as_bf16x4(uint32_t lo, uint32_t hi)
{
    return __builtin_bit_cast(bf16x4, u32x2{lo, hi});
}

// Two floats to a pair of bfloat16 (round to nearest even), low half first.
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// The 32 bits of the circular input string starting at bit R.
__device__ __forceinline__ uint32_t ext_window(const uint32_t* ext32, int R)
{
    return __builtin_amdgcn_alignbit(ext32[(R >> 5) + 1], ext32[R >> 5], (uint32_t)(R & 31));
}

// B operand of layer 1 (16x16x16, k = 4 g4 + i): the inputs a_k = +-1 of the
// window bits k < 5 as bfloat16 (0x3F80 / 0xBF80), zero for k >= 5; m0, m1
// are the lane's masks of valid halves.
__device__ __forceinline__ bf16x4 l1_operand(uint32_t x, int g4, uint32_t m0, uint32_t m1)
{
    const uint32_t y = x >> (4 * g4);
    const uint32_t d0 = 0xBF80BF80u ^ (((y & 1u) << 15) | ((y & 2u) << 30));
    const uint32_t d1 = 0xBF80BF80u ^ (((y & 4u) << 13) | ((y & 8u) << 28));
    return as_bf16x4(d0 & m0, d1 & m1);
}

// Positions of one wave's sample, one lane per bit: lane k < W holds word k of
// the sample; bit i = w * 64 + lane of the string is site p (advanced by 64
// per word, modulo L).
__device__ __forceinline__ void build_ext(uint64_t* ext, uint64_t word_of_lane, int p0, int L,
                                          int next, int lane)
{
    int p = p0;
    for (int w = 0; w < next; ++w) {
        const int src = p >> 6;
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)word_of_lane, src);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(word_of_lane >> 32), src);
        const uint32_t wbits = (p & 32) ? hi : lo;
        const uint64_t m = __ballot((wbits >> (p & 31)) & 1u);
        if (lane == 0) ext[w] = m;
        p += 64;
        while (p >= L) p -= L;
    }
}

// Circular halo rows of the position-major h1 and its channel-major copy:
// rows 0, 1 and LP + 2, LP + 3 copied from the rows of their sites; for g2
// (position-major only) rows 0, 1 and L + 2, L + 3 copied, rows LP + 2 and
// LP + 3 zero where they are not those.  dst / src rows per lane slot are
// precomputed (src < 0: zero), packed as two signed 16-bit halves to keep the
// registers they hold through the sample loop few.
struct HaloSlots {
    uint32_t ds[3];
    __device__ void set(int s, int dst, int src) { ds[s] = (uint32_t)(dst & 0xFFFF) | ((uint32_t)src << 16); }
    __device__ int dst(int s) const { return (int)(int16_t)(ds[s] & 0xFFFFu); }
    __device__ int src(int s) const { return (int)(int16_t)(ds[s] >> 16); }
};

// ---------------------------------------------------------------------------
// Forward and backward passes, one sample per wave, up to 8 waves per block
// sharing the weights: two waves per SIMD, which the 256 registers and the
// per-wave LDS below are sized for.
//
// Layer 1 (1 -> 32, K = 5 padded to 16) runs once per block on the matrix
// cores, over the 32 input windows it can see, into a table of h1 and
// 1 - h1^2 that the passes read per position.  Layer 2 (32 -> 32, K = 160)
// runs on the matrix cores with positions as the rows of each product and
// channels as its columns: a lane ends with one channel at 4 consecutive
// positions, so per-channel sums take one register per channel tile and the
// W1 gradient is one more product (bf16 dz1 against the exact +-1 inputs).  The layer-2
// contraction index is taken tap-major, q = t * 32 + c', so that one 16x16x32
// step covers one tap: its A operand is 8 consecutive channels of h1 (or g2)
// at one position, a 16-byte read of the position-major array, and its B
// operand (the weights) a 16-byte read of the shared weights at each product.
// The weight-gradient pass contracts over positions (16x16x16): its A operand
// (4 positions of one g2 channel) is four 2-byte reads of the position-major
// array, its B operand comes from the channel-major copy of h1, the tap shift
// formed from two aligned 8-byte reads with byte alignment, all five taps from
// one pair.
//
// The forward pass reads the A operands of the next tile before the epilogue
// of the current one; the input-gradient pass runs one tile at a time (the
// other wave of the SIMD covers the latency).  The position-major array holds
// h1 during the forward pass and g2 after it: each tile writes its g2 at the
// end of its epilogue, after the reads of the next tile, the only one that
// shares rows with it, were issued.  The scalar delta = d loss / d f of a sample is applied
// after the matrix products (in float32): the products run on
// g2 = w3s (1 - h2^2) and the results are scaled by delta.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(512) void k_net(const float* __restrict__ theta,
                                             const uint64_t* __restrict__ states,
                                             const float* __restrict__ counts, int L, int64_t n,
                                             int64_t ld, float inv_n, float* __restrict__ f_out,
                                             float* __restrict__ partial)
{
    // products and sums may fuse here: the results are compared statistically
#pragma clang fp contract(fast)
    extern __shared__ __align__(16) char smem[];
    const int LP = net_lp(L), P = LP + 4, NT = LP / 16;
    const int W = (L + 63) >> 6, next = net_ext_words(L);
    const int nw = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, g4 = lane >> 4;

    NetShared S;
    S.W2R = (uint16_t*)smem;
    S.W2T = S.W2R + CH * WS;
    S.b1 = (float*)(S.W2T + CH * WS);
    S.b2 = S.b1 + CH;
    S.w3s = S.b2 + CH;
    S.D1 = S.w3s + CH;
    S.T1 = (uint16_t*)(S.D1 + kWindows * CH);
    char* wbase = smem + kNetShared + (size_t)wv * net_wave_bytes(L);
    uint64_t* ext = (uint64_t*)wbase;
    const uint32_t* ext32 = (const uint32_t*)wbase;
    uint16_t* HP = (uint16_t*)(wbase + net_ext_bytes(L));   // [P][RS]: h1, then g2
    uint16_t* H1C = HP + P * RS;                              // [32][P]

    // the wave's first sample word, loaded before the set-up so that its
    // latency overlaps it
    const int64_t stride = (int64_t)gridDim.x * nw;
    int64_t smp = (int64_t)blockIdx.x * nw + wv;
    uint64_t word = (lane < W && smp < n) ? states[(int64_t)lane * ld + smp] : 0ull;
    // W2 as bfloat16, row-major and transposed: each thread issues its loads
    // ten at a time before the stores (a loop of one load per iteration
    // would wait out the memory latency at every element)
    for (int i0 = threadIdx.x; i0 < CH * Q; i0 += 10 * blockDim.x) {
        float v[10];
#pragma unroll
        for (int u = 0; u < 10; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            v[u] = i < CH * Q ? theta[OFF_W2 + i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 10; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < CH * Q) {
                const int c = i / Q, rest = i % Q, cp = rest / KS, t = rest % KS;   // W2[c][c'][t]
                const uint16_t h = f2bf(v[u]);
                S.W2R[c * WS + t * CH + cp] = h;
                S.W2T[cp * WS + t * CH + c] = h;
            }
        }
    }
    for (int c = threadIdx.x; c < CH; c += blockDim.x) {
        S.b1[c] = theta[OFF_B1 + c];
        S.b2[c] = theta[OFF_B2 + c];
        float w = 0.0f;
        for (int t = 0; t < KS; ++t) w += bfr(theta[OFF_W3 + c * KS + t]);
        S.w3s[c] = w;
    }
    // layer-1 B operand: W1[mt * 16 + r][k], k = 4 g4 + i < 5
    bf16x4 W1op[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g4 + i;
            h[i] = k < KS ? f2bf(theta[OFF_W1 + (mt * 16 + r) * KS + k]) : (uint16_t)0;
        }
        W1op[mt] = as_bf16x4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
    }
    const uint32_t m0 = g4 == 0 ? 0xFFFFFFFFu : (g4 == 1 ? 0x0000FFFFu : 0u);
    const uint32_t m1 = g4 == 0 ? 0xFFFFFFFFu : 0u;
    // Layer 1 as tables over its 32 input windows: a position's pre-activation
    // depends only on the 5 inputs (+-1) of its window, so h1 takes one of 32
    // values per channel.  Four products of 16 windows x 16 channels, the
    // product a position tile would use (the same operands and accumulator), give
    // T1 = h1 as bfloat16 and D1 = 1 - h1^2 in float32, the two channels
    // r and 16 + r of a lane side by side (one read serves both channel tiles).
    for (int job = wv; job < 4; job += nw) {
        const int mt = job & 1, wt = job >> 1, c = mt * 16 + r;
        const float b1c = theta[OFF_B1 + c];
        const f32x4 z = mfma16(l1_operand((uint32_t)(wt * 16 + r), g4, m0, m1), W1op[mt],
                               f32x4{b1c, b1c, b1c, b1c});
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int w = wt * 16 + 4 * g4 + v;
            const float h = tanh_fast(z[v]);
            S.T1[w * CH + 2 * r + mt] = (uint16_t)pk_bf16(h, 0.0f);
            if (MODE == 1) S.D1[w * CH + 2 * r + mt] = 1.0f - h * h;
        }
    }
    const uint32_t ma = r < KS ? 0xFFFFFFFFu : 0u;
    // halo slots: idx = lane + 64 s over 4 rows (h1) / 6 rows (g2) of 32 channels
    HaloSlots H1s, G2s;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int idx = lane + 64 * s, k = idx >> 5;
        H1s.set(s, -1, -1);
        if (k < 4) {
            const int R = k < 2 ? k : LP + k;   // 0, 1, LP + 2, LP + 3
            H1s.set(s, R, (R - 2 + 2 * L) % L + 2);
        }
        const int RG = k == 0 ? 0 : k == 1 ? 1 : k == 2 ? LP + 2 : k == 3 ? LP + 3 : L + k - 2;
        G2s.set(s, RG, RG < 2 ? RG + L : (RG == L + 2 || RG == L + 3) ? RG - L : -1);
    }
    const int p0 = (lane - 4 + L) % L;
    __syncthreads();
    const float b3 = theta[OFF_B3], c0 = theta[OFF_C0];
    // the lane's channels c = mt * 16 + r
    float b2s[2], w3c[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        b2s[mt] = S.b2[mt * 16 + r];
        w3c[mt] = S.w3s[mt * 16 + r];
    }
    // the layer-2 B operands of both passes, read from LDS at each product:
    // output channel mt * 16 + r, tap t, input channels 8 g4 .. 8 g4 + 7
    // (forward), and the transposed weights for the input gradient
    const uint16_t* const wf = S.W2R + r * WS + 8 * g4;
    const uint16_t* const wb = S.W2T + r * WS + 8 * g4;

    // per-lane accumulators over the block's samples: the layer-2 weight
    // gradient for c = mt * 16 + 4 g4 + v and q = qt * 16 + r, the layer-1
    // weight gradient for c = mt * 16 + 4 g4 + v and tap r < 5, and per-channel
    // sums for c = mt * 16 + r
    f32x4 acc[2][10], gW1[2];
    float gb1[2], gW3[2], gb2[2];
    float gb3 = 0.0f, gc0 = 0.0f, gloss = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 10; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        gW1[a] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        gb1[a] = gW3[a] = gb2[a] = 0.0f;
    }

    for (; smp < n; smp += stride) {
        const uint64_t word_next =
            (lane < W && smp + stride < n) ? states[(int64_t)lane * ld + smp + stride] : 0ull;
        build_ext(ext, word, p0, L, next, lane);
        word = word_next;
        wave_sync();
        // layer 1 from the table: the lane writes channel mt * 16 + r at rows
        // R0 .. R0 + 3, whose windows are bits v .. v + 4 of the string from R0
        for (int nt = 0; nt < NT; ++nt) {
            const int R0 = nt * 16 + 2 + 4 * g4;
            const uint32_t x = ext_window(ext32, R0);
            uint32_t tp[4];   // h1 of channels r (low half) and 16 + r at row R0 + v
#pragma unroll
            for (int v = 0; v < 4; ++v)
                tp[v] = *reinterpret_cast<const uint32_t*>(S.T1 + (int)((x >> v) & 31u) * CH + 2 * r);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const int c = mt * 16 + r;
                const uint32_t lo = mt == 0 ? (tp[0] & 0xFFFFu) | (tp[1] << 16)
                                            : (tp[0] >> 16) | (tp[1] & 0xFFFF0000u);
                const uint32_t hi = mt == 0 ? (tp[2] & 0xFFFFu) | (tp[3] << 16)
                                            : (tp[2] >> 16) | (tp[3] & 0xFFFF0000u);
                *reinterpret_cast<uint32_t*>(H1C + c * P + R0) = lo;
                *reinterpret_cast<uint32_t*>(H1C + c * P + R0 + 2) = hi;
                HP[R0 * RS + c] = (uint16_t)lo;
                HP[(R0 + 1) * RS + c] = (uint16_t)(lo >> 16);
                HP[(R0 + 2) * RS + c] = (uint16_t)hi;
                HP[(R0 + 3) * RS + c] = (uint16_t)(hi >> 16);
            }
        }
        wave_sync();
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            if (H1s.dst(s) >= 0) {
                const int c = (lane + 64 * s) & 31;
                const uint16_t v = HP[H1s.src(s) * RS + c];
                HP[H1s.dst(s) * RS + c] = v;
                H1C[c * P + H1s.dst(s)] = v;
            }
        }
        wave_sync();
        // layers 2 and 3, positions as rows: one A operand (8 channels of h1 at
        // one position) serves both channel tiles.  The A operands of tile nt+1
        // are read before the epilogue of tile nt (a tile past the last is
        // clamped to it and its reads dropped).  Tile nt writes its g2
        // (position-major, over the h1 rows) at the end of its epilogue: its rows
        // end at row (nt+1)*16 + 1, which only tile nt+1 reads, and that read was
        // issued before; LDS operations of a wave complete in order.
        float fpart = 0.0f, s2p[2] = {0.0f, 0.0f}, g2p[2] = {0.0f, 0.0f};
        auto load_h = [&](bf16x8 (&A)[KS], int nt) {
            const int row = min(nt, NT - 1) * 16 + r;
#pragma unroll
            for (int t = 0; t < KS; ++t) A[t] = ld8(HP + (row + t) * RS + 8 * g4);
        };
        auto mm_f = [&](const bf16x8 (&A)[KS], f32x4 (&z)[2]) {
            z[0] = f32x4{b2s[0], b2s[0], b2s[0], b2s[0]};
            z[1] = f32x4{b2s[1], b2s[1], b2s[1], b2s[1]};
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                z[0] = mfma32(A[t], ld8(wf + t * 32), z[0]);
                z[1] = mfma32(A[t], ld8(wf + 16 * WS + t * 32), z[1]);
            }
        };
        auto epi_f = [&](const f32x4 (&z)[2], int nt) {
            const int jo = nt * 16 + 4 * g4;
            float vm[4];   // 1 for positions of the ring, 0 for the padding
#pragma unroll
            for (int v = 0; v < 4; ++v) vm[v] = jo + v < L ? 1.0f : 0.0f;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                float g2[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float h2 = tanh_fast(z[mt][v]);
                    const float hv = vm[v] * h2;
                    g2[v] = vm[v] * w3c[mt] * (1.0f - h2 * h2);
                    s2p[mt] += hv;
                    g2p[mt] += g2[v];
                }
                if (MODE == 1) {
                    const u32x2 pk{pk_bf16(g2[0], g2[1]), pk_bf16(g2[2], g2[3])};
                    uint16_t* hp = HP + (jo + 2) * RS + mt * 16 + r;
                    hp[0] = (uint16_t)pk[0];
                    hp[RS] = (uint16_t)(pk[0] >> 16);
                    hp[2 * RS] = (uint16_t)pk[1];
                    hp[3 * RS] = (uint16_t)(pk[1] >> 16);
                }
            }
        };
        {
            bf16x8 A0[KS], A1[KS];
            f32x4 z[2];
            load_h(A0, 0);
            for (int nt = 0; nt < NT; nt += 2) {
                mm_f(A0, z);           // tile nt
                load_h(A1, nt + 1);    // before tile nt's epilogue writes over rows it reads
                epi_f(z, nt);
                if (nt + 1 < NT) {
                    mm_f(A1, z);       // tile nt+1
                    load_h(A0, nt + 2);
                    epi_f(z, nt + 1);
                }
            }
        }
        fpart = w3c[0] * s2p[0] + w3c[1] * s2p[1];
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
        for (int mt = 0; mt < 2; ++mt) {
            gW3[mt] += delta * s2p[mt];
            gb2[mt] += delta * g2p[mt];
        }
        wave_sync();
        // weight gradient of layer 2: sum over positions of g2[c][j] h1[c'][j + t - 2]
        // for c = mt * 16 + 4 g4 + v and c' = h * 16 + r; A (4 positions of one g2
        // channel) from four 2-byte reads of the position-major array, which holds
        // g2 at row j + 2 and zeros for j >= L until the halo copy below; the five
        // taps of B from one aligned pair of 8-byte reads of the channel-major h1
#pragma unroll
        for (int hm = 0; hm < 4; ++hm) {
            const int h = hm >> 1, mt = hm & 1;
            f32x4 d[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) d[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const uint16_t* hrow = H1C + (h * 16 + r) * P + 4 * g4;
            const uint16_t* gcol = HP + (4 * g4 + 2) * RS + mt * 16 + r;
            for (int jt = 0; jt < NT; ++jt) {
                const uint16_t* gp = gcol + jt * 16 * RS;
                const bf16x4 A = as_bf16x4((uint32_t)gp[0] | ((uint32_t)gp[RS] << 16),
                                           (uint32_t)gp[2 * RS] | ((uint32_t)gp[3 * RS] << 16));
                const u32x2 lo = *reinterpret_cast<const u32x2*>(hrow + jt * 16);
                const u32x2 hi = *reinterpret_cast<const u32x2*>(hrow + jt * 16 + 4);
                d[0] = mfma16(A, as_bf16x4(lo[0], lo[1]), d[0]);
                d[1] = mfma16(A, as_bf16x4(__builtin_amdgcn_alignbit(lo[1], lo[0], 16),
                                           __builtin_amdgcn_alignbit(hi[0], lo[1], 16)), d[1]);
                d[2] = mfma16(A, as_bf16x4(lo[1], hi[0]), d[2]);
                d[3] = mfma16(A, as_bf16x4(__builtin_amdgcn_alignbit(hi[0], lo[1], 16),
                                           __builtin_amdgcn_alignbit(hi[1], hi[0], 16)), d[3]);
                d[4] = mfma16(A, as_bf16x4(hi[0], hi[1]), d[4]);
            }
#pragma unroll
            for (int t = 0; t < KS; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[mt][2 * t + h][v] += delta * d[t][v];
        }
        wave_sync();
        // circular halo rows of g2 for the input gradient
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int c = (lane + 64 * s) & 31;
            const uint16_t v = G2s.src(s) >= 0 ? HP[G2s.src(s) * RS + c] : (uint16_t)0;
            HP[G2s.dst(s) * RS + c] = v;
        }
        wave_sync();
        // input gradient of layer 2 and the layer-1 backward, positions as rows
        // (this pass only reads the arrays)
        auto load_g = [&](bf16x8 (&A)[KS], int nt) {
            const int row = min(nt, NT - 1) * 16 + r;
#pragma unroll
            for (int t = 0; t < KS; ++t) A[t] = ld8(HP + (row - t + 4) * RS + 8 * g4);
        };
        auto mm_b = [&](const bf16x8 (&A)[KS], f32x4 (&d)[2]) {
            d[0] = d[1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                d[0] = mfma32(A[t], ld8(wb + t * 32), d[0]);
                d[1] = mfma32(A[t], ld8(wb + 16 * WS + t * 32), d[1]);
            }
        };
        auto epi_b = [&](const f32x4 (&d)[2], int nt) {
            const int jo = nt * 16 + 4 * g4;
            float vm[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) vm[v] = jo + v < L ? delta : 0.0f;
            // 1 - h1^2 at positions jo + v from the table (windows: bits v .. v + 4
            // of the string from row jo + 2)
            const uint32_t xw = ext_window(ext32, jo + 2);
            f32x2 dp[4];   // channels r and 16 + r
#pragma unroll
            for (int v = 0; v < 4; ++v)
                dp[v] = *reinterpret_cast<const f32x2*>(S.D1 + (int)((xw >> v) & 31u) * CH + 2 * r);
            // inputs a at positions jo + i + t - 2 for tap t = r (B of the W1 gradient)
            const uint32_t xa = ext_window(ext32, jo + r + 2);
            const bf16x4 Ba = as_bf16x4((0xBF80BF80u ^ (((xa & 1u) << 15) | ((xa & 2u) << 30))) & ma,
                                        (0xBF80BF80u ^ (((xa & 4u) << 13) | ((xa & 8u) << 28))) & ma);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                float dz[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    dz[v] = vm[v] * d[mt][v] * dp[v][mt];
                    gb1[mt] += dz[v];
                }
                gW1[mt] = mfma16(as_bf16x4(pk_bf16(dz[0], dz[1]), pk_bf16(dz[2], dz[3])), Ba,
                                 gW1[mt]);
            }
        };
        // one tile at a time: the other wave of the SIMD covers the latency
        for (int nt = 0; nt < NT; ++nt) {
            bf16x8 A[KS];
            f32x4 dc[2];
            load_g(A, nt);
            mm_b(A, dc);
            epi_b(dc, nt);
        }
        wave_sync();
    }
    if (MODE == 0) return;

    // Block sums in a fixed order (no atomics, so the result is reproducible):
    // the layer-2 weight gradient in two halves of 16 output channels, then the
    // small parameters, each through the per-wave regions.
    __syncthreads();   // every wave is done with its region
    float* red = (float*)wbase;   // at least 16 * Q floats per wave
    float* out = partial + (int64_t)blockIdx.x * (kGuideParams + 1);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int qt = 0; qt < 10; ++qt)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(4 * g4 + v) * Q + qt * 16 + r] = acc[mt][qt][v];
        __syncthreads();
        for (int i = threadIdx.x; i < 16 * Q; i += blockDim.x) {
            const int c = mt * 16 + i / Q, q = i % Q, t = q >> 5, cp = q & 31;
            float v[8];   // the waves' values read at once (nw <= 8), summed in wave order
#pragma unroll
            for (int w = 0; w < 8; ++w)
                v[w] = w < nw ? ((const float*)(smem + kNetShared + (size_t)w * net_wave_bytes(L)))[i]
                              : 0.0f;
            float sum = 0.0f;
#pragma unroll
            for (int w = 0; w < 8; ++w)
                if (w < nw) sum += v[w];
            out[OFF_W2 + c * Q + cp * KS + t] = sum;
        }
        __syncthreads();   // the half is read before the next one is written
    }
    // small parameters: the W1 gradient at red[c * 5 + t] (lanes r < 5), the
    // per-channel partials of b1, b2 and W3 at red[160 + (k * 4 + g4) * 32 + c]
    // and the scalars at red[544 + k]
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        if (r < KS) {
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(mt * 16 + 4 * g4 + v) * KS + r] = gW1[mt][v];
        }
        const int c = mt * 16 + r;
        red[160 + (0 * 4 + g4) * 32 + c] = gb1[mt];
        red[160 + (1 * 4 + g4) * 32 + c] = gb2[mt];
        red[160 + (2 * 4 + g4) * 32 + c] = gW3[mt];
    }
    if (lane == 0) {
        red[544] = gb3;
        red[545] = gc0;
        red[546] = gloss;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CH * KS + 3 * CH + 3; i += blockDim.x) {
        // the cnt values of parameter i in each wave's region, every wave's
        // read at once (nw <= 8), then summed wave by wave in order
        int o[4] = {0, 0, 0, 0}, cnt = 1;
        if (i < CH * KS) {
            o[0] = i;
        } else if (i < CH * KS + 3 * CH) {
            const int k = (i - CH * KS) >> 5, c = (i - CH * KS) & 31;
#pragma unroll
            for (int g = 0; g < 4; ++g) o[g] = 160 + (k * 4 + g) * 32 + c;
            cnt = 4;
        } else {
            o[0] = 544 + (i - CH * KS - 3 * CH);
        }
        float v[8][4];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            const float* R = (const float*)(smem + kNetShared + (size_t)w * net_wave_bytes(L));
#pragma unroll
            for (int g = 0; g < 4; ++g) v[w][g] = (w < nw && g < cnt) ? R[o[g]] : 0.0f;
        }
        float sum = 0.0f;
#pragma unroll
        for (int w = 0; w < 8; ++w)
#pragma unroll
            for (int g = 0; g < 4; ++g)
                if (w < nw && g < cnt) sum += v[w][g];
        if (i < CH * KS) {
            out[OFF_W1 + i] = sum;
        } else if (i < CH * KS + 3 * CH) {
            const int k = (i - CH * KS) >> 5, c = (i - CH * KS) & 31;
            if (k == 0) out[OFF_B1 + c] = sum;
            else if (k == 1) out[OFF_B2 + c] = sum;
            else
                for (int t = 0; t < KS; ++t) out[OFF_W3 + c * KS + t] = sum;
        } else {
            const int k = i - CH * KS - 3 * CH;
            out[k == 0 ? OFF_B3 : (k == 1 ? OFF_C0 : kGuideParams)] = sum;
        }
    }
}

// Adam (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8) on parameter p with
// gradient g; bc1, bc2 are the bias corrections 1 - beta^step.
__device__ __forceinline__ void adam_update(float* __restrict__ theta, float* __restrict__ m,
                                            float* __restrict__ v, int p, float g, float lr,
                                            float bc1, float bc2)
{
    const float mm = 0.9f * m[p] + 0.1f * g;
    const float vv = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

// Sum of the per-block partials: 16 parameters per block, 16 lanes per
// parameter each summing every 16th block in double precision, then the 16
// lane sums combined in a fixed order.  The float gradient then goes to grad
// (if not null) and, when theta is not null, straight into one Adam step; the
// loss to `loss` (if not null) and, as a double, added to *loss_sum (if not
// null) by the one thread that owns it.
__global__ __launch_bounds__(256) void k_net_reduce(const float* __restrict__ partial, int blocks,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss, float* theta,
                                                    float* m, float* v, float lr, float bc1,
                                                    float bc2, double* __restrict__ loss_sum)
{
    __shared__ double s[16][17];
    const int pl = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int p = blockIdx.x * 16 + pl;
    double acc = 0.0;
    if (p <= kGuideParams) {
        // eight loads in flight at a time; the sum keeps the order of b
#pragma unroll 8
        for (int b = part; b < blocks; b += 16) acc += partial[(int64_t)b * (kGuideParams + 1) + p];
    }
    s[pl][part] = acc;
    __syncthreads();
    if (part == 0 && p <= kGuideParams) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += s[pl][k];
        const float tf = (float)t;
        if (p < kGuideParams) {
            if (grad) grad[p] = tf;
            if (theta) adam_update(theta, m, v, p, tf, lr, bc1, bc2);
        } else {
            if (loss) *loss = tf;
            if (loss_sum) *loss_sum += (double)tf;
        }
    }
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float bc1, float bc2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kGuideParams) return;
    adam_update(theta, m, v, p, grad[p], lr, bc1, bc2);
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

constexpr int kNetBlocks = 256;   // the compute units of the chip
static_assert(kNetBlocks <= kGuideBlocks, "partials of k_net fit the guide workspace");

static void adam_corrections(int step, float* bc1, float* bc2)
{
    *bc1 = 1.0f - powf(0.9f, (float)step);
    *bc2 = 1.0f - powf(0.999f, (float)step);
}

// Forward (mode 0) or the per-block partial gradients (mode 1); returns the
// grid used through *blocks_out.
static hipError_t launch_net_pass(int mode, const float* theta, const uint64_t* states, int64_t ld,
                                  const float* counts, int L, int64_t n, float* f_out,
                                  float* partial, int* blocks_out, hipStream_t st)
{
    const int nw = net_waves(L);
    const int64_t want = (n + nw - 1) / nw;
    // one block per CU (its waves fill the LDS and the registers), a single
    // round of blocks: each block pays its set-up and its reduction once, and
    // the partials to sum are as few as can be
    const int blocks = (int)(want < kNetBlocks ? want : kNetBlocks);   // fits the workspace
    const size_t sm = net_block_smem(L);
    if (blocks_out) *blocks_out = blocks;
    if (mode == 0)
        hipLaunchKernelGGL(k_net<0>, dim3(blocks), dim3(64 * nw), sm, st, theta, states, counts,
                           L, n, ld, 1.0f / (float)n, f_out, partial);
    else
        hipLaunchKernelGGL(k_net<1>, dim3(blocks), dim3(64 * nw), sm, st, theta, states, counts,
                           L, n, ld, 1.0f / (float)n, f_out, partial);
    return hipGetLastError();
}

static constexpr int kReduceBlocks = (kGuideParams + 1 + 15) / 16;

hipError_t launch_net(int mode, const float* theta, const uint64_t* states, int64_t ld,
                      const float* counts, int L, int64_t n, float* f_out, float* partial,
                      float* grad, float* loss, hipStream_t st)
{
    int blocks = 0;
    hipError_t e = launch_net_pass(mode, theta, states, ld, counts, L, n, f_out, partial, &blocks, st);
    if (e != hipSuccess || mode == 0) return e;
    hipLaunchKernelGGL(k_net_reduce, dim3(kReduceBlocks), dim3(256), 0, st, partial, blocks, grad,
                       loss, nullptr, nullptr, nullptr, 0.0f, 1.0f, 1.0f, nullptr);
    return hipGetLastError();
}

hipError_t launch_train_epoch(float* theta, float* m, float* v, const uint64_t* states,
                              int64_t ld, const float* counts, int L, int64_t n, int64_t batch,
                              int step0, float lr, double* loss_sum, float* partial,
                              hipStream_t st)
{
    int k = 0;
    for (int64_t a = 0; a < n; a += batch, ++k) {
        const int64_t nb = (n - a < batch) ? n - a : batch;
        int blocks = 0;
        hipError_t e = launch_net_pass(1, theta, states + a, ld, counts + a, L, nb, nullptr,
                                       partial, &blocks, st);
        if (e != hipSuccess) return e;
        float bc1, bc2;
        adam_corrections(step0 + k + 1, &bc1, &bc2);
        hipLaunchKernelGGL(k_net_reduce, dim3(kReduceBlocks), dim3(256), 0, st, partial, blocks,
                           nullptr, nullptr, theta, m, v, lr, bc1, bc2, loss_sum);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
    float bc1, bc2;
    adam_corrections(step, &bc1, &bc2);
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

// Scratch of the allocation-free conditional distillation: the sums, counts
// and (when the caller passes no G) the uniform-context table of
// launch_bond_table_cond, kCondWorkBytes whatever the number of samples.  One
// copy per GPU, held until the process ends and shared by every call on that
// GPU (calls that overlap on one GPU race on it; k_zero_stats clears the sums
// and counts at the start of every call).  Host code never passes `scratch`
// itself to a kernel: its device address comes from hipGetSymbolAddress,
// looked up once per device.
static __device__ __align__(256) unsigned char scratch[kCondWorkBytes];

namespace {
constexpr int kScratchDevices = 64;
std::atomic<void*> g_scratch_addr[kScratchDevices];
}  // namespace

hipError_t cond_scratch(void** out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    void* p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        // with `dev` current: each GPU holds its own copy at its own address
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return hipSuccess;
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
