// Signature admissibility of a shifted reducer t * g_k (section "Signature
// regime: correctness under admissibility predicates", Theorem
// "Signature-sound compilation"; section "Discussion: Integrating
// Signatures, Admissibility, and GPU Scheduling").  Element k carries the
// signature s_k e_{i_k}; the row's signature is (t s_k) e_{i_k}.  The row is
// rejected by the syzygy test when a listed syzygy monomial of index i_k
// divides t s_k, else by the rewrite test when a newer element k' > k of the
// same index has s_{k'} dividing t s_k.  Device side, shared by the bulk
// filter and the reducer search of the symbolic preprocessing.
#pragma once

#include "common.hpp"

#define SIG_OK 0u
#define SIG_SYZYGY 1u
#define SIG_REWRITTEN 2u
#define SIG_OVERFLOW 4u  // t s_k does not fit the exponent lanes

struct SigDev {
    const u32* sidx;     // signature index of each element
    const u64* smon;     // signature monomial of each element (P word)
    const u32* syz_off;  // per index: [syz_off[i], syz_off[i+1]) in syz_mon
    const u64* syz_mon;
    const u32* rw_off;   // per index: its elements, ascending, with their signature monomials
    const u32* rw_k;
    const u64* rw_mon;
    u32 nindex, npolys, n, w;
    u64 lanes, H;        // exponent lanes and their top bits
};

// a | b on the exponent lanes (degree fields ignored)
__device__ __forceinline__ bool sig_div(const SigDev& S, u64 a, u64 b) {
    a &= S.lanes;
    b &= S.lanes;
    if (((a | b) & S.H) == 0) return (((b | S.H) - a) & S.H) == S.H;
    for (u32 i = 0; i < S.n; ++i)
        if (mono_exp(a, i, S.w) > mono_exp(b, i, S.w)) return false;
    return true;
}

// t * s as a P word; sets *ovf when a lane would overflow
__device__ __forceinline__ u64 sig_mul(const SigDev& S, u64 t, u64 s, bool* ovf) {
    // no lane's top bit set in either word: lane sums stay below 2^w, so the
    // word sum is the product (degree fields add too)
    if (((t | s) & S.H) == 0 && mono_deg(t) + mono_deg(s) <= 255) return t + s;
    u64 r = 0;
    u32 d = 0;
    for (u32 i = 0; i < S.n; ++i) {
        const u32 e = mono_exp(t, i, S.w) + mono_exp(s, i, S.w);
        if (e >> S.w) *ovf = true;
        r |= (u64)(e & ((1u << S.w) - 1)) << (S.w * i);
        d += e;
    }
    if (d > 255) *ovf = true;
    return r | ((u64)(d & 255) << 56);
}

// first element of index i newer than k (rw_k ascending within the index)
__device__ __forceinline__ u32 sig_rw_first(const SigDev& S, u32 i, u32 k) {
    u32 lo = S.rw_off[i], hi = S.rw_off[i + 1];
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (S.rw_k[mid] <= k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The flag of row (t, k), by one thread, with the tables read through the
// given arrays (the descriptor's, or copies of them in LDS).
__device__ __forceinline__ u32 sig_adm_thread(const SigDev& S, const u32* sidx, const u64* smon, const u32* soff,
                                              const u64* syzm, const u32* roff, const u32* rwk, const u64* rwm,
                                              u64 t, u32 k) {
    bool ovf = false;
    const u32 i = sidx[k];
    const u64 u = sig_mul(S, t, smon[k], &ovf);
    if (ovf) return SIG_OVERFLOW;
    for (u32 q = soff[i]; q < soff[i + 1]; ++q)
        if (sig_div(S, syzm[q], u)) return SIG_SYZYGY;
    u32 lo = roff[i], hi = roff[i + 1];
    while (lo < hi) {  // first element of index i newer than k
        const u32 mid = (lo + hi) >> 1;
        if (rwk[mid] <= k)
            lo = mid + 1;
        else
            hi = mid;
    }
    for (u32 q = lo; q < roff[i + 1]; ++q)
        if (sig_div(S, rwm[q], u)) return SIG_REWRITTEN;
    return SIG_OK;
}

// The flag of row (t, k), by a whole wave (lanes over the lists); every lane
// returns the same value.
__device__ __forceinline__ u32 sig_adm_wave(const SigDev& S, u64 t, u32 k) {
    const u32 lane = threadIdx.x & (F4_WAVE - 1);
    bool ovf = false;
    const u32 i = S.sidx[k];
    const u64 u = sig_mul(S, t, S.smon[k], &ovf);
    if (ovf) return SIG_OVERFLOW;
    const u32 s0 = S.syz_off[i], s1 = S.syz_off[i + 1];
    for (u32 q0 = s0; q0 < s1; q0 += F4_WAVE) {
        const u32 q = q0 + lane;
        if (__ballot(q < s1 && sig_div(S, S.syz_mon[q], u))) return SIG_SYZYGY;
    }
    const u32 r0 = sig_rw_first(S, i, k), r1 = S.rw_off[i + 1];
    for (u32 q0 = r0; q0 < r1; q0 += F4_WAVE) {
        const u32 q = q0 + lane;
        if (__ballot(q < r1 && sig_div(S, S.rw_mon[q], u))) return SIG_REWRITTEN;
    }
    return SIG_OK;
}
