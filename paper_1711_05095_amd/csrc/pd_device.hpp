// Device building blocks: Philox4x32-10, bit-packed ring occupancy, and
// wave64 / block reductions and scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pd_internal.hpp"

namespace pd {

// Global address-space view of a pointer read from a descriptor in memory.
// Such pointers are generic to the compiler, which then emits flat memory
// instructions; flat stores are counted with LDS operations, so every LDS
// read after a store in a loop would wait for the store to reach memory.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by the published constants, xor with the Weyl key.
// Each product is one v_mad_u64_u32 and each three-way xor one v_bitop3_b32
// (truth table 0x96 = a ^ b ^ c).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// X = 53 bits of (a, b) plus one, an integer in [1, 2^53]: the uniform
// variate u = X 2^-53 in (0, 1] without its scale (log_unit takes the scale as
// an exponent offset).  Every step is exact.
__device__ __forceinline__ double unit_scaled(uint32_t a, uint32_t b)
{
    return fma((double)a, 2097152.0, (double)((b >> 11) + 1u));   // a 2^21 + lo <= 2^53
}

// ln(x 2^-eoff) for x 2^-eoff in (0, 1] (Tang's table-driven method).  x =
// m 2^e with m in [0.75, 1.5); the table row i covers m in [0.75 + 0.75 i/128,
// 0.75 + 0.75 (i+1)/128) (the row index is rounded once, so m may lie an ulp
// outside its row) and holds c ~ 1/centre (exactly 1 on the row that holds 1,
// so the result is accurate to the last bit near 1), -ln c split into a part
// that is a multiple of 2^-42 and a remainder.  With r = m c - 1 (one
// rounding, |r| <= 2^-8), the logarithm is (e - eoff) ln2 - ln c + log1p(r);
// (e - eoff) ln2_hi - ln c_hi is exact and log1p(r) is its Taylor series to
// r^7, coefficients pc = 1/7, -1/6, ..., -1/2 (passed in as values uniform
// over the wave, so the fma take them from scalar registers; the truncation is
// below 2^-59 relative).  The result is within about one ulp.
__device__ __forceinline__ double log_unit(double x, const double* __restrict__ tab,
                                           double ln2_hi, double ln2_lo,
                                           const double (&pc)[kLogPoly], int eoff)
{
    const int e0 = __builtin_amdgcn_frexp_exp(x);
    const double f = __builtin_amdgcn_frexp_mant(x);   // [0.5, 1)
    const bool low = f < 0.75;
    const double m = low ? f * 2.0 : f;                 // [0.75, 1.5), exact
    const double e = (double)(e0 - eoff - (low ? 1 : 0));
    const int i = (int)fma(m, 128.0 / 0.75, -128.0);   // in [0, 127]
    const double c = tab[kLogCols * i];
    const double nlc_hi = tab[kLogCols * i + 1];
    const double nlc_lo = tab[kLogCols * i + 2];
    const double r = fma(m, c, -1.0);
    double p = pc[0];
#pragma unroll
    for (int k = 1; k < kLogPoly; ++k) p = fma(p, r, pc[k]);
    const double l1p = fma(r * r, p, r);
    const double t = fma(e, ln2_hi, nlc_hi);            // exact
    return t + (fma(e, ln2_lo, nlc_lo) + l1p);
}

// e^x for x <= 0 (Cody and Waite's reduction): x = k ln2 + r with k the
// integer nearest x / ln2 and |r| <= ln2 / 2; k ln2_hi is exact (ln2_hi is a
// multiple of 2^-42 and |k| < 2^11), e^r is its Taylor series to r^13
// (coefficients pc = 1/13!, ..., 1/1!, 1, uniform over the wave so the fma
// take them from scalar registers; the truncation is below 2^-56 relative) and
// 2^k is applied exactly by ldexp.  Arguments below -1000 are taken as -1000:
// the result is zero either way.
__device__ __forceinline__ double exp_nonpos(double x, double ln2_hi, double ln2_lo,
                                             const double (&pc)[14])
{
    x = fmax(x, -1000.0);
    const double k = rint(x * 1.4426950408889634);
    const double r = fma(-k, ln2_lo, fma(-k, ln2_hi, x));
    double p = pc[0];
#pragma unroll
    for (int i = 1; i < 14; ++i) p = fma(p, r, pc[i]);
    return ldexp(p, (int)k);
}

// floor(((a << 32) | b) * r / 2^64) for r < 2^31: a uniform index in [0, r).
__device__ __forceinline__ uint32_t mulhi64_small(uint32_t a, uint32_t b, uint32_t r)
{
    const uint64_t ph = (uint64_t)a * r;
    const uint64_t pl = (uint64_t)b * r;
    return (uint32_t)((ph + (pl >> 32)) >> 32);
}

// ---------------------------------------------------------------------------
// Ring occupancy: W words of 64 sites, site i is bit (i & 63) of word i >> 6,
// bits >= L are zero.  Bond i joins sites i and (i+1) mod L.
// ---------------------------------------------------------------------------

// Bit i of the result is n_i xor n_{(i+1) mod L}: the allowed hops.
template <int W>
__device__ __forceinline__ void bond_mask(const uint64_t (&x)[W], int lb, uint64_t (&m)[W])
{
    const uint64_t n0 = x[0] & 1ull;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t nxt = x[w] >> 1;
        if (w + 1 < W) nxt |= x[w + 1] << 63;
        else nxt |= n0 << lb;   // lb = (L - 1) & 63: site L-1 sees site 0
        m[w] = x[w] ^ nxt;
    }
}

template <int W>
__device__ __forceinline__ int popcount_words(const uint64_t (&m)[W])
{
    int r = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) r += __popcll(m[w]);
    return r;
}

// Byte table of select_bit_lut: entry b * 8 + q is the position of the q-th
// set bit (0-based, ascending) of the byte b for q < popcount(b), else 0.  The
// host builds it once (2 KB in the shared workspace); a block copies it into
// LDS (8-byte aligned), 8 bytes per thread.
__device__ __forceinline__ void load_select_table(uint8_t* t, const uint8_t* src, int tid,
                                                  int nthr)
{
    const auto s = gptr((const uint64_t*)src);
    for (int e = tid; e < 256; e += nthr) ((uint64_t*)t)[e] = s[e];
}

// Position of the q-th set bit (0-based, ascending) of the W-word mask, for
// q < its popcount: the word, then halvings down to a byte, then one lookup
// in the byte table (load_select_table, in LDS).
template <int W>
__device__ __forceinline__ int select_bit_lut(const uint64_t (&m)[W], uint32_t q,
                                              const uint8_t* __restrict__ sel)
{
    uint64_t word = m[W - 1];
    int base = (W - 1) * 64;
    bool found = false;
#pragma unroll
    for (int w = 0; w < W - 1; ++w) {
        const uint32_t c = (uint32_t)__popcll(m[w]);
        const bool here = !found && q < c;
        if (here) { word = m[w]; base = w * 64; }
        if (!found && !here) q -= c;
        found = found || here;
    }
    uint32_t v = (uint32_t)word;
    uint32_t c = (uint32_t)__popc(v);
    int pos = 0;
    if (q >= c) { q -= c; v = (uint32_t)(word >> 32); pos = 32; }
    c = (uint32_t)__popc(v & 0xFFFFu);
    if (q >= c) { q -= c; v >>= 16; pos += 16; }
    c = (uint32_t)__popc(v & 0xFFu);
    if (q >= c) { q -= c; v >>= 8; pos += 8; }
    return base + pos + sel[((v & 0xFFu) << 3) | (q & 7u)];
}

// Word i (0 <= i < W) of the register array, i not known at compile time.
template <int W>
__device__ __forceinline__ uint64_t word_at(const uint64_t (&x)[W], int i)
{
    uint64_t v = x[0];
#pragma unroll
    for (int w = 1; w < W; ++w)
        if (i == w) v = x[w];
    return v;
}

// Occupancies of sites p .. p+n-1 (bit k = site p+k), for p + n <= L, n <= 32.
template <int W>
__device__ __forceinline__ uint32_t lin_bits(const uint64_t (&x)[W], int p, int n)
{
    const int wi = p >> 6, sh = p & 63;
    uint64_t v = word_at<W>(x, wi) >> sh;
    if (sh + n > 64) v |= word_at<W>(x, wi + 1) << (64 - sh);
    return (uint32_t)v & (n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u));
}

// Occupancies of sites p, p+1, ..., p+n-1 taken mod L (0 <= p < L, n <= 32).
template <int W>
__device__ __forceinline__ uint32_t ring_bits(const uint64_t (&x)[W], int L, int p, int n)
{
    uint32_t bits = 0;
    int got = 0;
    while (got < n) {
        const int take = min(n - got, L - p);
        bits |= lin_bits<W>(x, p, take) << got;
        got += take;
        p = 0;
    }
    return bits;
}

// Exchange the occupancies across bond b (the two sites differ, so both flip).
template <int W>
__device__ __forceinline__ void hop(uint64_t (&x)[W], int b, int L)
{
    const int wb = b >> 6;
    const int sb = b & 63;
    const bool wrap = (b == L - 1);               // partner is site 0
    const bool cross = (sb == 63) && !wrap;       // partner is bit 0 of word wb+1
    const uint64_t f = wrap ? (1ull << sb) : (3ull << sb);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t t = (w == wb) ? f : 0ull;
        if ((w == wb + 1 && cross) || (w == 0 && wrap)) t |= 1ull;
        x[w] ^= t;
    }
}

// ---------------------------------------------------------------------------
// Wave64 and block (kTile threads) reductions and scans.
// ---------------------------------------------------------------------------
struct OpSum {
    template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
    __device__ __forceinline__ double operator()(double a, double b) const { return fmax(a, b); }
};

template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
    return v;
}

template <class T, class Op>
__device__ __forceinline__ T wave_scan_incl(T v, Op op)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T u = __shfl_up(v, o, 64);
        if (lane >= o) v = op(u, v);
    }
    return v;
}

// One DPP move of a double (both halves); lanes without a source, and rows
// that ROWS leaves out, get id.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v, double id)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v), o = (uint64_t)__double_as_longlong(id);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, CTRL, ROWS,
                                               0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32),
                                               CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Inclusive wave64 scan of doubles on DPP (all 64 lanes active; id is the
// identity of op): shifts by 1, 2, 4 and 8 lanes within each row of 16, then
// rows 1 and 3 take lane 15 and 47 of their left neighbour row, then rows 2
// and 3 take lane 31.  The association is fixed, so the result is too.
template <class Op>
__device__ __forceinline__ double wave_scan_dpp(double v, Op op, double id)
{
    v = op(v, dpp_f64<0x111, 0xF>(v, id));   // row_shr:1
    v = op(v, dpp_f64<0x112, 0xF>(v, id));   // row_shr:2
    v = op(v, dpp_f64<0x114, 0xF>(v, id));   // row_shr:4
    v = op(v, dpp_f64<0x118, 0xF>(v, id));   // row_shr:8
    v = op(v, dpp_f64<0x142, 0xA>(v, id));   // row_bcast:15 into rows 1, 3
    v = op(v, dpp_f64<0x143, 0xC>(v, id));   // row_bcast:31 into rows 2, 3
    return v;
}

// Block-wide reduction; every thread gets the result.  `sh` holds kTile/64 Ts.
template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T* sh)
{
    const int wave = threadIdx.x >> 6;
    v = wave_reduce(v, op);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    T r = sh[0];
#pragma unroll
    for (int i = 1; i < kTile / 64; ++i) r = op(r, sh[i]);
    return r;
}

// Block-wide inclusive scan in thread order; `total` gets the last value.
template <class T, class Op>
__device__ __forceinline__ T block_scan_incl(T v, Op op, T* sh, T& total)
{
    const int wave = threadIdx.x >> 6;
    v = wave_scan_incl(v, op);
    __syncthreads();
    if ((threadIdx.x & 63) == 63) sh[wave] = v;
    __syncthreads();
    T carry = v;  // placeholder, replaced below for waves > 0
    bool have = false;
#pragma unroll
    for (int i = 0; i < kTile / 64; ++i) {
        if (i < wave) {
            carry = have ? op(carry, sh[i]) : sh[i];
            have = true;
        }
    }
    if (have) v = op(carry, v);
    T t = sh[0];
#pragma unroll
    for (int i = 1; i < kTile / 64; ++i) t = op(t, sh[i]);
    total = t;
    return v;
}

}  // namespace pd
