// Device building blocks: Philox4x32-10, bit-packed ring occupancy, and
// wave64 / block reductions and scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pd_internal.hpp"

namespace pd {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by the published constants, xor with the Weyl key.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// u in (0, 1]: 53 bits of (a, b) plus one, times 2^-53.  Every step is exact.
__device__ __forceinline__ double unit_open0(uint32_t a, uint32_t b)
{
    const double hi = (double)a * 2097152.0;          // a * 2^21, exact
    const double lo = (double)(b >> 11) + 1.0;        // < 2^21 + 1, exact
    return (hi + lo) * 0x1p-53;                       // < 2^53 + 1, exact
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

// Position of the q-th set bit (0-based, ascending) of the W-word mask.
template <int W>
__device__ __forceinline__ int select_bit(const uint64_t (&m)[W], uint32_t q)
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
    c = (uint32_t)__popc(v & 0xFu);
    if (q >= c) { q -= c; v >>= 4; pos += 4; }
    c = (uint32_t)__popc(v & 0x3u);
    if (q >= c) { q -= c; v >>= 2; pos += 2; }
    c = v & 1u;
    if (q >= c) { pos += 1; }
    return base + pos;
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
