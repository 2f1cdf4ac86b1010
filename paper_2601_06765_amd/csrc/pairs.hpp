// Host side of the pair set: packed-monomial helpers for the CPU and the
// Gebauer-Moeller update (section "Pair management and the normal
// strategy").  Host code only; included by the C-ABI driver.
#pragma once
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


// Scratch of the fast update, one per system.
struct GmScratch {
    bool generic = false;  // some leading monomial is outside the fast forms
    std::vector<u32> act;  // active basis indices, ascending
    std::vector<u64> L, E;
    std::vector<u32> de, order, cnt;
    std::vector<u8> cop;
    struct Min {
        u64 e;
        u32 de, a;
        u8 coprime;
    };
    std::vector<Min> M;
    std::vector<HPair> Pn;
};

// The same update as gm_update, computed without the quadratic scan.  With
// E(g) = lcm(LM(h), LM(g)) / LM(h) (the excess of g over h), lcm(h, g') |
// lcm(h, g) iff E(g') | E(g), and the sequential rule of gm_update reduces to:
// the pair (g, h) is created iff E(g) has no proper divisor among the
// excesses, g has the largest index among the candidates with the same
// excess, and no candidate with that excess is coprime to LM(h).  (A proper
// divisor always covers: if its pair was not kept, the pair that covered it
// also properly divides, and following such pairs ends at a kept pair or at a
// later candidate.)  The minimal excesses are found in order of degree,
// testing each candidate only against the minimal ones found so far; a
// minimal excess of degree one (a single variable) covers every larger
// excess that contains the variable, which a mask tests at once.
static void gm_insert(const MonoOps& mo, GmScratch& X, std::vector<u64>& lm, std::vector<u8>& active,
                      std::vector<HPair>& P, u32 h) {
    const u64 lh = lm[h];
    const u32 wmax = 1u << mo.w;
    if (!X.generic && (!mo.clean(lh) || (u32)(lh >> 56) >= wmax)) X.generic = true;
    if (X.generic) {
        gm_update(mo, lm, active, P, h);
        return;
    }
    const u32 dh = (u32)(lh >> 56);
    const u64 lhl = lh & mo.lanes;
    std::vector<u32>& C = X.act;
    const size_t nc = C.size();
    X.L.resize(nc);
    X.E.resize(nc);
    X.de.resize(nc);
    X.cop.resize(nc);
    X.order.resize(nc);
    X.cnt.assign(wmax + 1, 0);
    for (size_t a = 0; a < nc; ++a) {
        const u64 g = lm[C[a]];
        const u64 l = mo.lcm_c(lh, g);
        const u64 e = l - lhl;
        const u32 d = mo.lane_sum(e);
        X.L[a] = l | ((u64)(dh + d) << 56);
        X.E[a] = e;
        X.de[a] = d;
        X.cop[a] = d == (u32)(g >> 56);
        ++X.cnt[d];
    }
    for (u32 d = 0, run = 0; d <= wmax; ++d) {
        const u32 k = X.cnt[d];
        X.cnt[d] = run;
        run += k;
    }
    for (size_t a = 0; a < nc; ++a) X.order[X.cnt[X.de[a]]++] = (u32)a;
    X.M.clear();
    u64 m1 = 0;         // nonzero-lane mask of the degree-one minimal excesses
    size_t m2 = 0;      // M[m2..] have degree >= 2
    bool zero = false;  // an excess 1 (LM(g) | LM(h)) divides every other one
    for (size_t o = 0; o < nc; ++o) {
        const u32 a = X.order[o];
        const u64 e = X.E[a];
        const u32 d = X.de[a];
        if (zero && d >= 1) continue;
        if (d >= 2 && (mo.nonzero_lanes(e) & m1)) continue;
        bool cov = false;
        long eq = -1;
        for (size_t k = (d >= 2 ? m2 : 0); k < X.M.size(); ++k) {
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
        if (eq >= 0) {
            X.M[eq].a = a;
            X.M[eq].coprime |= X.cop[a];
            continue;
        }
        X.M.push_back({e, d, a, X.cop[a]});
        if (d == 0) zero = true;
        if (d <= 1) {
            m1 |= mo.nonzero_lanes(e);
            m2 = X.M.size();
        }
    }
    // old pairs: drop those whose lcm LM(h) properly witnesses
    std::vector<HPair>& Pn = X.Pn;
    Pn.clear();
    Pn.reserve(P.size() + X.M.size());
    for (const HPair& q : P) {
        const u64 ql = q.lcm & mo.lanes;
        const bool drop = mo.divides_c(lh, q.lcm) && mo.lcm_c(lm[q.i], lh) != ql && mo.lcm_c(lh, lm[q.j]) != ql;
        if (!drop) Pn.push_back(q);
    }
    for (const GmScratch::Min& m : X.M)
        if (!m.coprime) Pn.push_back({C[m.a], h, X.L[m.a]});
    P.swap(Pn);
    // LM(h) retires the active elements it divides
    size_t k = 0;
    for (size_t a = 0; a < nc; ++a) {
        const u32 g = C[a];
        if (mo.divides_c(lh, lm[g]))
            active[g] = 0;
        else
            C[k++] = g;
    }
    C.resize(k);
    C.push_back(h);
    active[h] = 1;
}

// All new elements of one F4 step, h0 .. h1-1 in insertion order, with the
// result of gm_insert on each in turn.  The pairs (h_t, g) are formed per
// element as there (they depend on the active set at t only); the removal of
// existing pairs is order-independent (a pair present before the step is
// removed iff some new LM(h_t) witnesses it; a pair born at t iff some later
// one does), so it runs once per step over the pair set instead of once per
// element.
static void gm_insert_step(const MonoOps& mo, GmScratch& X, std::vector<u64>& lm, std::vector<u8>& active,
                           std::vector<HPair>& P, u32 h0, u32 h1) {
    const u32 wmax = 1u << mo.w;
    for (u32 h = h0; h < h1 && !X.generic; ++h)
        if (!mo.clean(lm[h]) || (u32)(lm[h] >> 56) >= wmax) X.generic = true;
    if (X.generic) {
        for (u32 h = h0; h < h1; ++h) gm_update(mo, lm, active, P, h);
        return;
    }
    const size_t p0 = P.size();
    std::vector<u32> born;  // insertion index of each pair created in this step
    std::vector<HPair> keep_old;
    for (u32 h = h0; h < h1; ++h) {
        const u64 lh = lm[h];
        const u32 dh = (u32)(lh >> 56);
        const u64 lhl = lh & mo.lanes;
        std::vector<u32>& C = X.act;
        const size_t nc = C.size();
        X.L.resize(nc);
        X.E.resize(nc);
        X.de.resize(nc);
        X.cop.resize(nc);
        X.order.resize(nc);
        X.cnt.assign(wmax + 1, 0);
        for (size_t a = 0; a < nc; ++a) {
            const u64 g = lm[C[a]];
            const u64 l = mo.lcm_c(lh, g);
            const u64 e = l - lhl;
            const u32 d = mo.lane_sum(e);
            X.L[a] = l | ((u64)(dh + d) << 56);
            X.E[a] = e;
            X.de[a] = d;
            X.cop[a] = d == (u32)(g >> 56);
            ++X.cnt[d];
        }
        for (u32 d = 0, run = 0; d <= wmax; ++d) {
            const u32 k = X.cnt[d];
            X.cnt[d] = run;
            run += k;
        }
        for (size_t a = 0; a < nc; ++a) X.order[X.cnt[X.de[a]]++] = (u32)a;
        X.M.clear();
        u64 m1 = 0;
        size_t m2 = 0;
        bool zero = false;
        for (size_t o = 0; o < nc; ++o) {
            const u32 a = X.order[o];
            const u64 e = X.E[a];
            const u32 d = X.de[a];
            if (zero && d >= 1) continue;
            if (d >= 2 && (mo.nonzero_lanes(e) & m1)) continue;
            bool cov = false;
            long eq = -1;
            for (size_t k = (d >= 2 ? m2 : 0); k < X.M.size(); ++k) {
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
            if (eq >= 0) {
                X.M[eq].a = a;
                X.M[eq].coprime |= X.cop[a];
                continue;
            }
            X.M.push_back({e, d, a, X.cop[a]});
            if (d == 0) zero = true;
            if (d <= 1) {
                m1 |= mo.nonzero_lanes(e);
                m2 = X.M.size();
            }
        }
        for (const GmScratch::Min& m : X.M)
            if (!m.coprime) {
                P.push_back({C[m.a], h, X.L[m.a]});
                born.push_back(h - h0);
            }
        size_t k = 0;
        for (size_t a = 0; a < nc; ++a) {
            const u32 g = C[a];
            if (mo.divides_c(lh, lm[g]))
                active[g] = 0;
            else
                C[k++] = g;
        }
        C.resize(k);
        C.push_back(h);
        active[h] = 1;
    }
    // removals: a pair is dropped when some new LM(h_t) inserted after it
    // (all of them for the pairs that predate the step) divides its lcm
    // without being one of the two lcms it is formed of
    const u32 nh = h1 - h0;
    auto witnessed = [&](const HPair& q, u32 from) {
        const u64 ql = q.lcm & mo.lanes;
        for (u32 t = from; t < nh; ++t) {
            const u64 lh = lm[h0 + t];
            if (mo.divides_c(lh, q.lcm) && mo.lcm_c(lm[q.i], lh) != ql && mo.lcm_c(lh, lm[q.j]) != ql) return true;
        }
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
