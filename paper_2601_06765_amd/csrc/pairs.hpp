// Host side of the pair set: packed-monomial helpers for the CPU and the
// Gebauer-Moeller update (section "Pair management and the normal
// strategy").  Host code only; included by the C-ABI driver.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.hpp"

// ----------------------------------------------------- packed monomials (host)
// SWAR forms are valid while every exponent is below 2^(w-1) (the lane's top
// bit free as a guard), which holds when the degree is below 2^(w-1); above
// that the lanes are compared one by one.
struct MonoOps {
    u32 n, w, guard;
    u64 lanes, H, ones;  // lane bits, lane top bits, lane low bits
    void init(u32 n_) {
        n = n_;
        w = lane_bits(n);
        guard = 1u << (w - 1);
        lanes = (n * w >= 64) ? ~0ull : ((1ull << (n * w)) - 1);
        H = 0;
        ones = 0;
        for (u32 i = 0; i < n; ++i) {
            H |= 1ull << (w * i + w - 1);
            ones |= 1ull << (w * i);
        }
    }
    // every exponent below 2^(w-1): the lane-parallel forms below are exact
    bool clean(u64 a) const { return (a & H) == 0; }
    // lane-parallel forms for clean operands (no degree field in the result)
    bool divides_c(u64 a, u64 b) const { return ((((b & lanes) | H) - (a & lanes)) & H) == H; }
    u64 lcm_c(u64 a, u64 b) const {
        const u64 ge = (((a & lanes) | H) - (b & lanes)) & H;
        const u64 m = (ge >> (w - 1)) * ((1ull << w) - 1);
        return (a & m) | (b & ~m & lanes);
    }
    // sum of the exponents of a clean word whose sum is below 2^w: the
    // product by `ones` accumulates the lanes into lane n-1 without carries
    u32 lane_sum(u64 a) const { return (u32)((((a & lanes) * ones) >> (w * (n - 1))) & ((1ull << w) - 1)); }
    // top bit of every nonzero lane of a clean word
    u64 nonzero_lanes(u64 a) const { return (((a & lanes) | H) - ones) & H; }
    bool divides(u64 a, u64 b) const {  // a | b
        if ((u32)(a >> 56) >= guard || (u32)(b >> 56) >= guard) return mono_divides(a, b, n, w);
        return ((((b & lanes) | H) - (a & lanes)) & H) == H;
    }
    u64 lcm(u64 a, u64 b) const {
        if ((u32)(a >> 56) >= guard || (u32)(b >> 56) >= guard) return mono_lcm(a, b, n, w);
        u64 ge = (((a & lanes) | H) - (b & lanes)) & H;  // lanes where a >= b
        u64 m = (ge >> (w - 1)) * ((1ull << w) - 1);
        u64 l = (a & m) | (b & ~m & lanes);
        u32 d = 0;
        for (u32 i = 0; i < n; ++i) d += (u32)((l >> (w * i)) & ((1u << w) - 1));
        return l | ((u64)d << 56);
    }
    bool coprime(u64 a, u64 b) const {
        for (u32 i = 0; i < n; ++i)
            if (mono_exp(a, i, w) && mono_exp(b, i, w)) return false;
        return true;
    }
    u64 order_key(u64 P) const { return P ^ lanes; }
};

struct HPair {
    u32 i, j;
    u64 lcm;
};

// Gebauer-Moeller update inserting basis element h (Becker-Weispfenning):
// new pairs (h, g) are pruned by the chain and product criteria, old pairs
// whose lcm is a proper multiple witnessed by LM(h) are removed, and basis
// elements whose leading monomial LM(h) divides become inactive.
static void gm_update(const MonoOps& mo, std::vector<u64>& lm, std::vector<u8>& active, std::vector<HPair>& P,
                      u32 h) {
    const u64 lh = lm[h];
    std::vector<u32> C;
    for (u32 g = 0; g < h; ++g)
        if (active[g]) C.push_back(g);
    const size_t nc = C.size();
    std::vector<u64> L(nc);
    for (size_t a = 0; a < nc; ++a) L[a] = mo.lcm(lh, lm[C[a]]);
    std::vector<u8> kept(nc, 0);
    for (size_t a = 0; a < nc; ++a) {
        bool keep = mo.coprime(lh, lm[C[a]]);
        if (!keep) {
            bool covered = false;
            // still-pending pairs (b > a) and already kept ones (b < a)
            for (size_t b = 0; b < nc && !covered; ++b) {
                if (b == a) continue;
                if ((b > a || kept[b]) && mo.divides(L[b], L[a])) covered = true;
            }
            keep = !covered;
        }
        kept[a] = keep;
    }
    std::vector<HPair> Pn;
    Pn.reserve(P.size() + nc);
    for (const HPair& q : P) {
        bool drop = mo.divides(lh, q.lcm) && mo.lcm(lm[q.i], lh) != q.lcm && mo.lcm(lh, lm[q.j]) != q.lcm;
        if (!drop) Pn.push_back(q);
    }
    for (size_t a = 0; a < nc; ++a)
        if (kept[a] && !mo.coprime(lh, lm[C[a]])) Pn.push_back({C[a], h, L[a]});
    P.swap(Pn);
    for (u32 g = 0; g < h; ++g)
        if (active[g] && mo.divides(lh, lm[g])) active[g] = 0;
    active[h] = 1;
}


// Vector forms of the two inner loops of the fast update (x86-64 hosts with
// AVX2, chosen at run time; the scalar loops are the reference and give the
// same bits).
#if defined(__x86_64__) && !defined(__HIP_DEVICE_COMPILE__)
#include <immintrin.h>
#define GM_HAVE_AVX2 1
static bool gm_avx2() {
    static const bool ok = __builtin_cpu_supports("avx2");
    return ok;
}
// E[a] = lcm(lh, A[a]) - lhl for a < n (clean words, lane forms)
__attribute__((target("avx2"))) static void gm_excess_avx2(const u64* A, size_t n, u64 lh, u64 lanes, u64 H, u32 w,
                                                            u64* E) {
    const __m256i vl = _mm256_set1_epi64x((long long)(lh & lanes)), vlanes = _mm256_set1_epi64x((long long)lanes),
                  vH = _mm256_set1_epi64x((long long)H), vlh = _mm256_set1_epi64x((long long)(lh & lanes));
    const __m256i vlhH = _mm256_or_si256(vl, vH);
    size_t a = 0;
    for (; a + 4 <= n; a += 4) {
        const __m256i b = _mm256_and_si256(_mm256_loadu_si256((const __m256i*)(A + a)), vlanes);
        const __m256i ge = _mm256_and_si256(_mm256_sub_epi64(vlhH, b), vH);
        const __m256i m = _mm256_sub_epi64(_mm256_slli_epi64(ge, 1), _mm256_srli_epi64(ge, (int)(w - 1)));
        const __m256i l = _mm256_or_si256(_mm256_and_si256(vl, m), _mm256_andnot_si256(m, b));
        _mm256_storeu_si256((__m256i*)(E + a), _mm256_sub_epi64(l, vlh));
    }
    for (; a < n; ++a) {
        const u64 b = A[a] & lanes;
        const u64 ge = (((lh & lanes) | H) - b) & H;
        const u64 m = (ge << 1) - (ge >> (w - 1));
        E[a] = (((lh & lanes) & m) | (b & ~m)) - (lh & lanes);
    }
}
// bit k of the result: LH[t0 + k] divides the clean word q (k < 8, t0 + 8 <= nh)
__attribute__((target("avx2"))) static inline u32 gm_div8_avx2(const u64* LH, u64 qm, u64 lanes, u64 H) {
    const __m256i vq = _mm256_set1_epi64x((long long)qm), vlanes = _mm256_set1_epi64x((long long)lanes),
                  vH = _mm256_set1_epi64x((long long)H);
    const __m256i a0 = _mm256_and_si256(_mm256_loadu_si256((const __m256i*)LH), vlanes);
    const __m256i a1 = _mm256_and_si256(_mm256_loadu_si256((const __m256i*)(LH + 4)), vlanes);
    const __m256i r0 = _mm256_cmpeq_epi64(_mm256_and_si256(_mm256_sub_epi64(vq, a0), vH), vH);
    const __m256i r1 = _mm256_cmpeq_epi64(_mm256_and_si256(_mm256_sub_epi64(vq, a1), vH), vH);
    return (u32)_mm256_movemask_pd(_mm256_castsi256_pd(r0)) | ((u32)_mm256_movemask_pd(_mm256_castsi256_pd(r1)) << 4);
}
#else
#define GM_HAVE_AVX2 0
#endif

// Scratch of the fast update, one per system.
struct GmScratch {
    bool generic = false;  // some leading monomial is outside the fast forms
    std::vector<u32> act;  // active basis indices, ascending
    std::vector<u64> actlm;  // their leading monomials (same order)
    std::vector<u64> E;
    std::vector<u32> big;  // candidates with an excess of degree >= 2 not covered by a degree-one one
    struct Min {
        u64 e;
        u32 de, a;
        u8 coprime;
    };
    std::vector<Min> M;
    std::vector<HPair> Pn;
};

// lcm of clean words without a multiply: the lane mask of the lanes where
// a >= b is (ge << 1) - (ge >> (w - 1)) for the lane top bits ge (each set
// top bit becomes 2^(w(i+1)) - 2^(wi), the full lane; the lanes end below bit
// 57, so nothing leaves the word)
static inline u64 gm_lcm_lanes(const MonoOps& mo, u64 a, u64 b) {
    const u64 ge = (((a & mo.lanes) | mo.H) - (b & mo.lanes)) & mo.H;
    const u64 m = (ge << 1) - (ge >> (mo.w - 1));
    return (a & m) | (b & ~m & mo.lanes);
}

// The new pairs (g, h) that gm_update creates for element h, pushed onto P
// (born: their element index relative to h0, when given), computed without
// the quadratic scan.  With E(g) = lcm(LM(h), LM(g)) / LM(h) (the excess of
// g over h), lcm(h, g') | lcm(h, g) iff E(g') | E(g), and the sequential rule
// of gm_update reduces to: the pair (g, h) is created iff E(g) has no proper
// divisor among the excesses, g has the largest index among the candidates
// with the same excess, and no candidate with that excess is coprime to
// LM(h).  (A proper divisor always covers: if its pair was not kept, the pair
// that covered it also properly divides, and following such pairs ends at a
// kept pair or at a later candidate.)  Excess 1 (LM(g) | LM(h)) divides every
// other excess; a single variable divides every excess that contains it, so
// after one pass only the remaining excesses of degree >= 2 are compared,
// in order of degree, with the minimal ones found so far.
static void gm_new_pairs(const MonoOps& mo, GmScratch& X, const std::vector<u64>& lm, std::vector<HPair>& P,
                         u32 h, std::vector<u32>* born, u32 tag) {
    const u64 lh = lm[h];
    const u32 dh = (u32)(lh >> 56);
    const u64 lhl = lh & mo.lanes;
    const std::vector<u32>& C = X.act;
    const u64* A = X.actlm.data();
    const size_t nc = C.size();
    X.E.resize(nc);
    u64* E = X.E.data();
#if GM_HAVE_AVX2
    if (gm_avx2())
        gm_excess_avx2(A, nc, lh, mo.lanes, mo.H, mo.w, E);
    else
#endif
        for (size_t a = 0; a < nc; ++a) E[a] = gm_lcm_lanes(mo, lh, A[a]) - lhl;
    X.M.clear();
    // excess 1: the pair with the last such candidate, unless one is coprime
    // (only a constant LM(g) is); every other excess is a proper multiple
    {
        long last = -1;
        u8 cop = 0;
        for (size_t a = 0; a < nc; ++a)
            if (E[a] == 0) {
                last = (long)a;
                cop |= (u8)((u32)(A[a] >> 56) == 0);
            }
        if (last >= 0) {
            X.M.push_back({0, 0, (u32)last, cop});
            goto emit;
        }
    }
    {
        // single variables: lane index -> last candidate, coprime flag
        u32 last1[16];
        u8 cop1[16];
        for (u32 i = 0; i < mo.n; ++i) last1[i] = 0xffffffffu, cop1[i] = 0;
        u64 m1 = 0;
        for (size_t a = 0; a < nc; ++a) {
            const u64 e = E[a];
            if ((e & (e - 1)) == 0 && (e & mo.ones) == e) {  // one lane, value 1
                const u32 i = (u32)(__builtin_ctzll(e) / mo.w);
                last1[i] = (u32)a;
                cop1[i] |= (u8)((u32)(A[a] >> 56) == 1);
                m1 |= mo.nonzero_lanes(e);
            }
        }
        for (u32 i = 0; i < mo.n; ++i)
            if (last1[i] != 0xffffffffu) X.M.push_back({E[last1[i]], 1, last1[i], cop1[i]});
        const size_t m2 = X.M.size();
        // the rest, by degree then index
        X.big.clear();
        for (size_t a = 0; a < nc; ++a) {
            const u64 e = E[a];
            if (mo.nonzero_lanes(e) & m1) continue;  // covered (also drops the degree-one ones)
            X.big.push_back((u32)a);
        }
        auto deg_of_e = [&](u32 a) { return mo.lane_sum(E[a]); };
        std::sort(X.big.begin(), X.big.end(), [&](u32 x, u32 y) {
            const u32 dx = deg_of_e(x), dy = deg_of_e(y);
            return dx != dy ? dx < dy : x < y;
        });
        for (u32 a : X.big) {
            const u64 e = E[a];
            const u32 d = deg_of_e(a);
            bool cov = false;
            long eq = -1;
            for (size_t k = m2; k < X.M.size(); ++k) {
                const GmScratch::Min& m = X.M[k];
                if (m.de < d) {
                    if (mo.divides_c(m.e, e)) {
                        cov = true;
                        break;
                    }
                } else if (m.e == e) {
                    eq = (long)k;
                    break;
                }
            }
            if (cov) continue;
            const u8 cop = (u8)((u32)(A[a] >> 56) == d);
            if (eq >= 0) {
                X.M[eq].a = a;
                X.M[eq].coprime |= cop;
                continue;
            }
            X.M.push_back({e, d, a, cop});
        }
    }
emit:
    for (const GmScratch::Min& m : X.M)
        if (!m.coprime) {
            P.push_back({C[m.a], h, (lhl + m.e) | ((u64)(dh + m.de) << 56)});
            if (born) born->push_back(tag);
        }
}

// LM(h) retires the active elements it divides; h becomes active.
static void gm_retire(const MonoOps& mo, GmScratch& X, std::vector<u64>& lm, std::vector<u8>& active, u32 h) {
    const u64 lh = lm[h];
    size_t k = 0;
    for (size_t a = 0; a < X.act.size(); ++a) {
        const u32 g = X.act[a];
        if (mo.divides_c(lh, X.actlm[a])) {
            active[g] = 0;
        } else {
            X.act[k] = g;
            X.actlm[k] = X.actlm[a];
            ++k;
        }
    }
    X.act.resize(k);
    X.actlm.resize(k);
    X.act.push_back(h);
    X.actlm.push_back(lh);
    active[h] = 1;
}

static inline bool gm_fast_form(const MonoOps& mo, u64 l) { return mo.clean(l) && (u32)(l >> 56) < (1u << mo.w); }

// Whether a pair is removed by LM(h): LM(h) divides its lcm and differs from
// both of the lcms the pair is formed of.
static inline bool gm_witness(const MonoOps& mo, const std::vector<u64>& lm, const HPair& q, u64 lh) {
    const u64 ql = q.lcm & mo.lanes;
    return mo.divides_c(lh, q.lcm) && gm_lcm_lanes(mo, lm[q.i], lh) != ql && gm_lcm_lanes(mo, lh, lm[q.j]) != ql;
}

// gm_update for element h with the fast forms (falls back to gm_update for
// leading monomials outside them).
static void gm_insert(const MonoOps& mo, GmScratch& X, std::vector<u64>& lm, std::vector<u8>& active,
                      std::vector<HPair>& P, u32 h) {
    const u64 lh = lm[h];
    if (!X.generic && !gm_fast_form(mo, lh)) X.generic = true;
    if (X.generic) {
        gm_update(mo, lm, active, P, h);
        return;
    }
    const size_t p0 = P.size();
    gm_new_pairs(mo, X, lm, P, h, nullptr, 0);
    // old pairs: drop those whose lcm LM(h) properly witnesses
    std::vector<HPair>& Pn = X.Pn;
    Pn.clear();
    Pn.reserve(P.size());
    for (size_t a = 0; a < p0; ++a)
        if (!gm_witness(mo, lm, P[a], lh)) Pn.push_back(P[a]);
    for (size_t a = p0; a < P.size(); ++a) Pn.push_back(P[a]);
    P.swap(Pn);
    gm_retire(mo, X, lm, active, h);
}

// All new elements of one F4 step, h0 .. h1-1 in insertion order, with the
// result of gm_insert on each in turn.  The pairs (h_t, g) are formed per
// element as there (they depend on the active set at t only); the removal of
// existing pairs is order-independent (a pair present before the step is
// removed iff some new LM(h_t) witnesses it; a pair born at t iff some later
// one does), so it runs once per step over the pair set instead of once per
// element, eight new elements at a time with a branch-free divisibility test.
static void gm_insert_step(const MonoOps& mo, GmScratch& X, std::vector<u64>& lm, std::vector<u8>& active,
                           std::vector<HPair>& P, u32 h0, u32 h1) {
    for (u32 h = h0; h < h1 && !X.generic; ++h)
        if (!gm_fast_form(mo, lm[h])) X.generic = true;
    if (X.generic) {
        for (u32 h = h0; h < h1; ++h) gm_update(mo, lm, active, P, h);
        return;
    }
    const size_t p0 = P.size();
    std::vector<u32> born;  // insertion index of each pair created in this step
    for (u32 h = h0; h < h1; ++h) {
        gm_new_pairs(mo, X, lm, P, h, &born, h - h0);
        gm_retire(mo, X, lm, active, h);
    }
    // removals: a pair is dropped when some new LM(h_t) inserted after it
    // (all of them for the pairs that predate the step) witnesses it
    const u32 nh = h1 - h0;
    const u64* LH = lm.data() + h0;
#if GM_HAVE_AVX2
    const bool vec = gm_avx2();
#else
    const bool vec = false;
#endif
    auto witnessed = [&](const HPair& q, u32 from) {
        const u64 qm = (q.lcm & mo.lanes) | mo.H;
        u32 t = from;
        for (; t + 8 <= nh; t += 8) {
            u32 any = 0;
#if GM_HAVE_AVX2
            if (vec)
                any = gm_div8_avx2(LH + t, qm, mo.lanes, mo.H);
            else
#endif
                for (u32 k = 0; k < 8; ++k) any |= (u32)(((qm - (LH[t + k] & mo.lanes)) & mo.H) == mo.H) << k;
            while (any) {
                const u32 k = (u32)__builtin_ctz(any);
                any &= any - 1;
                if (gm_witness(mo, lm, q, LH[t + k])) return true;
            }
        }
        for (; t < nh; ++t)
            if (gm_witness(mo, lm, q, LH[t])) return true;
        return false;
    };
    std::vector<HPair>& Pn = X.Pn;
    Pn.clear();
    Pn.reserve(P.size());
    for (size_t a = 0; a < p0; ++a)
        if (!witnessed(P[a], 0)) Pn.push_back(P[a]);
    for (size_t a = p0; a < P.size(); ++a)
        if (!witnessed(P[a], born[a - p0] + 1)) Pn.push_back(P[a]);
    P.swap(Pn);
}
