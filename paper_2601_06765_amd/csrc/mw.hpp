// Two-word monomial keys (section "Monomial keys: order-refining encodings
// that make sorting feasible", multiword keys), for 1 <= n <= 30 variables.
// A monomial is the 128-bit number (m[0] high, m[1] low): the degree in bits
// 120..127, then the exponents of x_n, x_{n-1}, ..., x_1 in lanes of w bits,
// a = floor(56 / w) of them in m[0] (from bit 56 down), the rest in m[1]
// (from bit 64 down); no lane is split between the words and unused bits are
// zero.  The order key complements the lanes (not the degree): as 128-bit
// numbers, keys compare as grevlex with x_1 > ... > x_n (degree first, then
// the smaller exponent of the last variable wins), and distinct monomials
// have distinct keys.  The product of two monomials is the word-wise sum
// while no lane overflows.  Host and device.
#pragma once

#include "common.hpp"

__host__ __device__ __forceinline__ u32 mw_lane_bits(u32 n) {
    if (n == 0 || n > 30) return 0;
    for (u32 w = 8; w >= 4; --w)
        if (56 / w + 64 / w >= n) return w;
    return 0;
}

struct MwLayout {
    u32 n, w, a;          // variables, lane width, lanes in word 0
    u64 lanes0, lanes1;   // lane bits of each word
    u64 top0, top1;       // the top bit of every lane
};

__host__ __device__ inline MwLayout mw_layout(u32 n) {
    MwLayout L;
    L.n = n;
    L.w = mw_lane_bits(n);
    L.a = L.w ? (n < 56 / L.w ? n : 56 / L.w) : 0;
    L.lanes0 = L.lanes1 = L.top0 = L.top1 = 0;
    for (u32 p = 0; p < n && L.w; ++p) {  // p = 0 is x_n
        const u64 lane = ((1ull << L.w) - 1);
        if (p < L.a) {
            const u32 sh = 56 - (p + 1) * L.w;
            L.lanes0 |= lane << sh;
            L.top0 |= 1ull << (sh + L.w - 1);
        } else {
            const u32 sh = 64 - (p - L.a + 1) * L.w;
            L.lanes1 |= lane << sh;
            L.top1 |= 1ull << (sh + L.w - 1);
        }
    }
    return L;
}

// exponent of x_{v+1} (v = 0 .. n-1)
__host__ __device__ __forceinline__ u32 mw_exp(const MwLayout& L, u64 m0, u64 m1, u32 v) {
    const u32 p = L.n - 1 - v;
    if (p < L.a) return (u32)((m0 >> (56 - (p + 1) * L.w)) & ((1u << L.w) - 1));
    return (u32)((m1 >> (64 - (p - L.a + 1) * L.w)) & ((1u << L.w) - 1));
}

__host__ __device__ __forceinline__ u32 mw_deg(u64 m0) { return (u32)(m0 >> 56); }

// a word pair is a monomial: no bits outside the lanes and the degree byte,
// lanes adding up to the degree
__host__ __device__ inline bool mw_valid(const MwLayout& L, u64 m0, u64 m1) {
    if ((m0 & ~(L.lanes0 | (0xffull << 56))) || (m1 & ~L.lanes1)) return false;
    u32 d = 0;
    for (u32 v = 0; v < L.n; ++v) d += mw_exp(L, m0, m1, v);
    return d == mw_deg(m0);
}

// t * g would overflow a lane (or the degree byte)
__host__ __device__ inline bool mw_mul_overflows(const MwLayout& L, u64 t0, u64 t1, u64 g0, u64 g1) {
    if (mw_deg(t0) + mw_deg(g0) > 255) return true;
    if (!((t0 | g0) & L.top0) && !((t1 | g1) & L.top1)) return false;  // lane sums stay below 2^w
    for (u32 v = 0; v < L.n; ++v)
        if (mw_exp(L, t0, t1, v) + mw_exp(L, g0, g1, v) >= (1u << L.w)) return true;
    return false;
}
