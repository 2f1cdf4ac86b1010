// The pair set on the device (section "Pair management and the normal
// strategy"): the Gebauer-Moeller update of one F4 step and the normal
// selection with its halves, for a batch of systems, so that a system's pair
// set, leading monomials and activity flags never leave the device between
// steps.
//
// Update.  The new elements h_0 .. h_{rho-1} of a step enter the set in that
// order, each as in the sequential update (Becker-Weispfenning's form of
// Gebauer-Moeller): pairs (g, h_t) with the active elements g, pruned by the
// chain and product criteria; old pairs whose lcm LM(h_t) properly witnesses
// removed; active elements that LM(h_t) divides retired.  The sequential
// order only matters through the active set, and whether g is active when
// h_t is inserted is a divisibility fact: g (an old active element, or h_s
// with s < t) is active at t unless some h_u with u < t (and u > s for h_s)
// has LM(h_u) | LM(g).  So every element's window [start, end) of insertion
// indices is found first (k_gm_ends), and the pairs of all h_t are then formed
// independently, one workgroup per new element (k_gm_pairs).  For one h_t,
// with E(g) = lcm(LM(h_t), LM(g)) / LM(h_t): the pair (g, h_t) is created iff
// E(g) has no proper divisor among the candidates' excesses, g has the largest
// index among the candidates with the same excess, and no candidate with that
// excess is coprime to LM(h_t) (the pair kept in that class would be dropped
// by the product criterion).  Excess 1 divides every other excess, and a single
// variable every excess that contains it; the rest are compared pairwise.
// Removal is order-free: a pair is removed iff some element inserted after it
// witnesses it (k_gm_prune), which also counts the surviving pairs by lcm
// degree (k_gm_summary reads the least degree and its count off that).
//
// Selection (k_gm_select, one workgroup per system): the pairs of the least
// degree d give their two halves (lcm / LM(i), i) and (lcm / LM(j), j); the
// halves are sorted by (rank of the lcm, element) and deduplicated, and the
// other pairs move to the second buffer.  The active list (descending index)
// for the reducer search is written beside the rows.
//
// Exponents are compared lane by lane whenever a word has a lane's top bit
// set; the lane-parallel forms below are used only where they are exact.
#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "sort_lds.hpp"

#define GM_DEAD 0xffffffffu   // i of a removed pair
#define GM_THREADS 256
#define GM_CAND_LDS 2048      // candidates of one new element held in LDS
#define GM_SEL_THREADS 1024
#define GM_SEL_LDS 4096       // halves of one system sorted in LDS
#define GM_NO_DEG 0xffffffffu

struct GmLanes {
    u32 n, w;
    u64 lanes, H;
};

__device__ __forceinline__ GmLanes gm_lanes(u32 n) {
    GmLanes m;
    m.n = n;
    m.w = lane_bits(n);
    m.lanes = (n * m.w >= 64) ? ~0ull : ((1ull << (n * m.w)) - 1);
    m.H = 0;
    for (u32 i = 0; i < n; ++i) m.H |= 1ull << (m.w * i + m.w - 1);
    return m;
}

// every lane of a at most the same lane of b
__device__ __forceinline__ bool gm_div(const GmLanes& m, u64 a, u64 b) {
    a &= m.lanes;
    b &= m.lanes;
    if (((a | b) & m.H) == 0) return (((b | m.H) - a) & m.H) == m.H;
    for (u32 i = 0; i < m.n; ++i)
        if (mono_exp(a, i, m.w) > mono_exp(b, i, m.w)) return false;
    return true;
}

// lane-wise maximum (no degree field)
__device__ __forceinline__ u64 gm_lcm(const GmLanes& m, u64 a, u64 b) {
    a &= m.lanes;
    b &= m.lanes;
    if (((a | b) & m.H) == 0) {
        const u64 ge = ((a | m.H) - b) & m.H;          // top bit of the lanes where a >= b
        const u64 k = (ge << 1) - (ge >> (m.w - 1));  // those lanes, whole
        return (a & k) | (b & ~k);
    }
    u64 r = 0;
    for (u32 i = 0; i < m.n; ++i) {
        const u32 x = mono_exp(a, i, m.w), y = mono_exp(b, i, m.w);
        r |= (u64)(x > y ? x : y) << (m.w * i);
    }
    return r;
}

// One system's update: its basis, its pair buffer and its scratch.
struct GmSeg {
    const u64* lm;
    u32* act;      // activity flag per element
    u32* se;       // window [start, end) of each element (2 words per element)
    u64* plcm;
    u32* pij;
    u32* pborn;
    u32* ctr;      // [0] pairs in the buffer (insertion counter), [1] overflow bits
    u32* hist;     // surviving pairs per lcm degree (256 words, zero on entry)
    u32* sum;      // 8 summary words out
    u64* cE;       // candidate scratch in global memory (nullptr: LDS), ccap per workgroup
    u32* cI;
    u32* cInfo;
    u32* cBig;
    u32 n, h0, rho, p0;
    u32 cap, ccap;
};

// Windows of every element of the system, new activity flags, and the
// insertion counter set to the pairs already present.
__global__ void k_gm_ends(const GmSeg* segs) {
    const GmSeg G = segs[blockIdx.y];
    const GmLanes m = gm_lanes(G.n);
    const u32 np = G.h0 + G.rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        G.ctr[0] = G.p0;
        G.ctr[1] = 0;
    }
    for (u32 g = blockIdx.x * blockDim.x + threadIdx.x; g < np; g += gridDim.x * blockDim.x) {
        const bool old = g < G.h0;
        u32 start = old ? 0u : g - G.h0 + 1, end = G.rho + 1;
        if (old && !G.act[g]) {
            start = 1;
            end = 0;  // never a candidate
        } else {
            const u64 l = G.lm[g];
            for (u32 t = start; t < G.rho; ++t)
                if (gm_div(m, G.lm[G.h0 + t], l)) {
                    end = t + 1;  // h_t still pairs with g, then retires it
                    break;
                }
        }
        G.se[2 * g] = start;
        G.se[2 * g + 1] = end;
        G.act[g] = end == G.rho + 1 ? 1u : 0u;
    }
}

__device__ __forceinline__ void gm_emit(const GmSeg& G, u32 g, u32 h, u64 l, u32 t) {
    const u32 k = atomicAdd(&G.ctr[0], 1u);
    if (k < G.cap) {
        G.plcm[k] = l;
        G.pij[2 * k] = g;
        G.pij[2 * k + 1] = h;
        G.pborn[k] = t;
    } else {
        atomicOr(&G.ctr[1], 1u);
    }
}

// candidate info word: excess degree (bits 0..11), support (bits 12..25: one
// bit per variable), coprime to LM(h) (bit 31)
#define GM_INFO_DEG(x) ((x) & 0xfffu)
#define GM_INFO_SUP(x) (((x) >> 12) & 0x3fffu)
#define GM_INFO_COP(x) ((x) >> 31)

// The new pairs of h_t, t = blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ __launch_bounds__(GM_THREADS) void k_gm_pairs(const GmSeg* segs) {
    __shared__ u64 sE[GM_CAND_LDS];
    __shared__ u32 sI[GM_CAND_LDS], sInfo[GM_CAND_LDS], sBig[GM_CAND_LDS];
    __shared__ u32 s_wave[33];
    __shared__ u32 s_last1[16], s_cop1[16];
    __shared__ u32 s_m1, s_last0, s_cop0, s_nb;
    const GmSeg G = segs[blockIdx.y];
    const GmLanes m = gm_lanes(G.n);
    const u32 tid = threadIdx.x;
    const bool glob = G.cE != nullptr;
    u64* E = glob ? G.cE + (size_t)blockIdx.x * G.ccap : sE;
    u32* I = glob ? G.cI + (size_t)blockIdx.x * G.ccap : sI;
    u32* Info = glob ? G.cInfo + (size_t)blockIdx.x * G.ccap : sInfo;
    u32* Big = glob ? G.cBig + (size_t)blockIdx.x * G.ccap : sBig;
    const u32 cap = glob ? G.ccap : GM_CAND_LDS;
    for (u32 t = blockIdx.x; t < G.rho; t += gridDim.x) {
        const u32 h = G.h0 + t;
        const u64 lh = G.lm[h];
        const u32 dh = mono_deg(lh);
        const u64 lhl = lh & m.lanes;
        if (tid < 16) {
            s_last1[tid] = 0;
            s_cop1[tid] = 0;
        }
        if (tid == 0) {
            s_m1 = 0;
            s_last0 = 0;
            s_cop0 = 0;
            s_nb = 0;
        }
        __syncthreads();
        // candidates: the elements active when h_t is inserted, in index order
        u32 nc = 0;
        for (u32 base = 0; base < h; base += GM_THREADS) {
            const u32 g = base + tid;
            bool pred = false;
            if (g < h) pred = G.se[2 * g] <= t && t < G.se[2 * g + 1];
            u32 tot;
            const u32 pos = nc + block_exclusive_scan(pred ? 1u : 0u, s_wave, &tot);
            if (pred) {
                const u64 lg = G.lm[g];
                u64 e = 0;
                u32 de = 0, sup = 0;
                for (u32 i = 0; i < m.n; ++i) {
                    const u32 a = mono_exp(lh, i, m.w), b = mono_exp(lg, i, m.w);
                    const u32 x = b > a ? b - a : 0u;
                    e |= (u64)x << (m.w * i);
                    de += x;
                    sup |= (x ? 1u : 0u) << i;
                }
                const u32 cop = mono_deg(lg) == de ? 1u : 0u;  // E(g) = LM(g): coprime
                if (pos < cap) {
                    E[pos] = e;
                    I[pos] = g;
                    Info[pos] = de | (sup << 12) | (cop << 31);
                }
                if (de == 0) {
                    atomicMax(&s_last0, g + 1);
                    if (cop) atomicOr(&s_cop0, 1u);
                } else if (de == 1) {
                    const u32 i = (u32)(__ffs(sup) - 1);
                    atomicMax(&s_last1[i], g + 1);
                    if (cop) atomicOr(&s_cop1[i], 1u);
                    atomicOr(&s_m1, sup);
                }
            }
            nc += tot;
        }
        __syncthreads();
        if (nc > cap) {  // the host sizes cap above any candidate count
            if (tid == 0) atomicOr(&G.ctr[1], 2u);
            __syncthreads();
            continue;
        }
        if (s_last0) {
            // LM(g) | LM(h): every other excess is a proper multiple of 1
            if (tid == 0 && !s_cop0) gm_emit(G, s_last0 - 1, h, lh, t);
            __syncthreads();
            continue;
        }
        const u32 m1 = s_m1;
        for (u32 a = tid; a < nc; a += GM_THREADS) {
            const u32 inf = Info[a];
            if (GM_INFO_DEG(inf) >= 2 && !(GM_INFO_SUP(inf) & m1)) Big[atomicAdd(&s_nb, 1u)] = a;
        }
        __syncthreads();
        const u32 nb = s_nb;
        for (u32 x = tid; x < nb; x += GM_THREADS) {
            const u32 a = Big[x];
            const u64 ea = E[a];
            const u32 ia = Info[a], da = GM_INFO_DEG(ia), ga = I[a];
            bool ok = !GM_INFO_COP(ia);
            for (u32 y = 0; y < nb && ok; ++y) {
                const u32 b = Big[y];
                if (b == a) continue;
                const u32 ib = Info[b], db = GM_INFO_DEG(ib);
                if (db < da) {
                    if (gm_div(m, E[b], ea)) ok = false;  // a proper divisor
                } else if (db == da && E[b] == ea) {
                    if (I[b] > ga || GM_INFO_COP(ib)) ok = false;  // not the last, or the class is coprime
                }
            }
            if (ok) gm_emit(G, ga, h, (lhl + ea) | ((u64)(dh + da) << 56), t);
        }
        if (tid < m.n && s_last1[tid] && !s_cop1[tid])
            gm_emit(G, s_last1[tid] - 1, h, (lhl + (1ull << (m.w * tid))) | ((u64)(dh + 1) << 56), t);
        __syncthreads();
    }
}

// Removal of the pairs that a later element witnesses (LM(h_u) divides the
// lcm and differs from both lcm(LM(i), LM(h_u)) and lcm(LM(h_u), LM(j))), and
// the degree histogram of the pairs that stay.
__global__ void k_gm_prune(const GmSeg* segs) {
    __shared__ u32 sh[256];
    const GmSeg G = segs[blockIdx.y];
    const GmLanes m = gm_lanes(G.n);
    sh[threadIdx.x] = 0;
    __syncthreads();
    const u32 cnt = min(G.ctr[0], G.cap);
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
        const u32 i = G.pij[2 * q];
        if (i == GM_DEAD) continue;
        const u32 j = G.pij[2 * q + 1];
        const u64 l = G.plcm[q], ll = l & m.lanes;
        const u32 from = q < G.p0 ? 0u : G.pborn[q] + 1;
        bool dead = false;
        for (u32 t = from; t < G.rho && !dead; ++t) {
            const u64 lh = G.lm[G.h0 + t];
            if (gm_div(m, lh, l) && gm_lcm(m, G.lm[i], lh) != ll && gm_lcm(m, lh, G.lm[j]) != ll) dead = true;
        }
        if (dead)
            G.pij[2 * q] = GM_DEAD;
        else
            atomicAdd(&sh[mono_deg(l)], 1u);
    }
    __syncthreads();
    if (sh[threadIdx.x]) atomicAdd(&G.hist[threadIdx.x], sh[threadIdx.x]);
}

// Summary of one system: pairs in the buffer, surviving pairs, least lcm
// degree and its count, active elements, overflow bits.
__global__ __launch_bounds__(256) void k_gm_summary(const GmSeg* segs) {
    __shared__ u32 s_wave[33];
    __shared__ u32 s_dmin;
    const GmSeg G = segs[blockIdx.x];
    const u32 tid = threadIdx.x;
    if (tid == 0) s_dmin = GM_NO_DEG;
    __syncthreads();
    const u32 c = G.hist[tid];
    if (c) atomicMin(&s_dmin, tid);
    u32 kept;
    (void)block_exclusive_scan(c, s_wave, &kept);
    u32 na = 0;
    const u32 np = G.h0 + G.rho;
    for (u32 g0 = 0; g0 < np; g0 += 256) {
        u32 tot;
        (void)block_exclusive_scan(g0 + tid < np ? G.act[g0 + tid] : 0u, s_wave, &tot);
        na += tot;
    }
    if (tid == 0) {
        const u32 cnt = G.ctr[0];
        G.sum[0] = min(cnt, G.cap);
        G.sum[1] = kept;
        G.sum[2] = s_dmin;
        G.sum[3] = s_dmin == GM_NO_DEG ? 0u : G.hist[s_dmin];
        G.sum[4] = na;
        G.sum[5] = G.ctr[1] | (cnt > G.cap ? 1u : 0u);
        G.sum[6] = 0;
        G.sum[7] = 0;
    }
}

// One system's selection.
struct GmSel {
    const u64* plcm;
    const u32* pij;
    u64* qlcm;  // the other buffer: the pairs that stay
    u32* qij;
    const u64* lm;
    const u32* act;
    const u32* binom;  // rank table of (n, d)
    u64* keys;         // global scratch (2 * room keys) or nullptr: LDS
    u32* vals;
    u32 room;          // halves expected (2 * pairs of degree d)
    u32 count, npolys, n, d;
    u32 kbits, hibit;
    u32 row_base, act_base, act_room;
    u32* out;  // [0] rows, [1] pairs left, [2] active elements, [3] halves found
};

__global__ __launch_bounds__(GM_SEL_THREADS) void k_gm_select(const GmSel* segs, u64* rows_t, u32* rows_k,
                                                                u32* active_out) {
    extern __shared__ u64 gs_mem[];
    __shared__ u32 run[256];
    __shared__ u32 wcnt[(GM_SEL_THREADS / F4_WAVE) * 256];
    __shared__ u32 s_wave[33];
    const GmSel G = segs[blockIdx.x];
    const u32 tid = threadIdx.x;
    const u32 w = lane_bits(G.n);
    u64 *ka, *kb;
    u32 *va, *vb;
    if (G.keys) {
        ka = G.keys;
        kb = G.keys + G.room;
        va = G.vals;
        vb = G.vals + G.room;
    } else {
        ka = gs_mem;
        kb = gs_mem + GM_SEL_LDS;
        va = (u32*)(gs_mem + 2 * GM_SEL_LDS);
        vb = va + GM_SEL_LDS;
    }
    u32 nk = 0, nrest = 0;
    // halves of the pairs of degree d, the other pairs to the second buffer
    for (u32 base = 0; base < G.count; base += GM_SEL_THREADS) {
        const u32 q = base + tid;
        u32 kind = 0, i = 0, j = 0;
        u64 l = 0;
        if (q < G.count) {
            i = G.pij[2 * q];
            if (i != GM_DEAD) {
                j = G.pij[2 * q + 1];
                l = G.plcm[q];
                kind = mono_deg(l) == G.d ? 1u : 2u;
            }
        }
        u32 tot;
        const u32 pr = nrest + block_exclusive_scan(kind == 2 ? 1u : 0u, s_wave, &tot);
        if (kind == 2) {
            G.qlcm[pr] = l;
            G.qij[2 * pr] = i;
            G.qij[2 * pr + 1] = j;
        }
        nrest += tot;
        const u32 pk = nk + block_exclusive_scan(kind == 1 ? 2u : 0u, s_wave, &tot);
        if (kind == 1 && pk + 1 < G.room) {
            const u64 r = (u64)mono_rank(l, G.n, w, G.d, G.binom) << G.kbits;
            ka[pk] = r | i;
            va[pk] = 2 * q;
            ka[pk + 1] = r | j;
            va[pk + 1] = 2 * q + 1;
        }
        nk += tot;
    }
    if (nk > G.room) {  // the summary counted fewer pairs of degree d: report, write nothing
        if (tid == 0) {
            G.out[0] = 0;
            G.out[1] = nrest;
            G.out[2] = 0;
            G.out[3] = nk;
        }
        return;
    }
    __syncthreads();
    const bool sw = lds_radix_sort(ka, kb, va, vb, nk, 0, G.hibit, 8, GM_SEL_THREADS, run, wcnt, s_wave);
    __syncthreads();
    const u64* K = sw ? kb : ka;
    const u32* V = sw ? vb : va;
    // one row per distinct (lcm, element)
    u32 nr = 0;
    for (u32 base = 0; base < nk; base += GM_SEL_THREADS) {
        const u32 x = base + tid;
        const bool head = x < nk && (x == 0 || K[x] != K[x - 1]);
        u32 tot;
        const u32 pos = nr + block_exclusive_scan(head ? 1u : 0u, s_wave, &tot);
        if (head) {
            const u32 v = V[x], q = v >> 1;
            const u32 k = G.pij[2 * q + (v & 1)];
            rows_t[G.row_base + pos] = G.plcm[q] - G.lm[k];
            rows_k[G.row_base + pos] = k;
        }
        nr += tot;
    }
    // active elements, descending index
    u32 na = 0;
    for (u32 base = 0; base < G.npolys; base += GM_SEL_THREADS) {
        const u32 x = base + tid;
        const u32 g = G.npolys - 1 - x;
        const bool pred = x < G.npolys && G.act[g];
        u32 tot;
        const u32 pos = na + block_exclusive_scan(pred ? 1u : 0u, s_wave, &tot);
        if (pred && pos < G.act_room) active_out[G.act_base + pos] = g;
        na += tot;
    }
    if (tid == 0) {
        G.out[0] = nr;
        G.out[1] = nrest;
        G.out[2] = na;
        G.out[3] = nk;
    }
}

static u32 gm_bitlen(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

static void gm_grow(Ctx& c, DevPairs& P, u64 need) {
    if (need <= P.cap) return;
    const u64 cap = std::max<u64>(need, 2 * P.cap);
    if (cap >= (1ull << 32)) throw F4Error{2, "pair set too large"};
    DevPairs Q;
    for (int b = 0; b < 2; ++b) {
        Q.lcm[b].reset(&c.pool, cap);
        Q.ij[b].reset(&c.pool, 2 * cap);
    }
    Q.born.reset(&c.pool, cap);
    if (P.count) {
        F4_HIP_TRY(hipMemcpyAsync(Q.lcm[0].ptr, P.lcm[P.cur].ptr, (size_t)P.count * 8, hipMemcpyDeviceToDevice,
                                  c.stream));
        F4_HIP_TRY(hipMemcpyAsync(Q.ij[0].ptr, P.ij[P.cur].ptr, (size_t)P.count * 8, hipMemcpyDeviceToDevice,
                                  c.stream));
    }
    for (int b = 0; b < 2; ++b) {
        P.lcm[b] = std::move(Q.lcm[b]);
        P.ij[b] = std::move(Q.ij[b]);
    }
    P.born = std::move(Q.born);
    P.cur = 0;
    P.cap = cap;
}

void gm_insert_batch(Ctx& c, const std::vector<GmInsert>& v) {
    const u32 S = (u32)v.size();
    if (!S) return;
    if (S > 65535) throw F4Error{2, "batch has more than 65535 systems"};
    hipStream_t s = c.stream;
    // room: the pairs present plus, for each new element, one pair per
    // element active when it is inserted (at most nact + t for h_t)
    u64 ntot = 0, ccap = 1;
    u32 maxrho = 0, maxnp = 1;
    bool glob = false;
    for (const GmInsert& a : v) {
        DevPairs& P = *a.P;
        const u64 cand = (u64)P.nact + a.rho;
        const u64 room = (u64)P.count + (u64)a.rho * P.nact + (u64)a.rho * (a.rho ? a.rho - 1 : 0) / 2;
        gm_grow(c, P, std::max<u64>(room, 64));
        ntot += a.h0 + a.rho;
        ccap = std::max<u64>(ccap, cand);
        maxrho = std::max(maxrho, a.rho);
        maxnp = std::max(maxnp, a.h0 + a.rho);
        if (cand > GM_CAND_LDS) glob = true;
    }
    if (ntot >= (1ull << 31)) throw F4Error{2, "basis too large"};
    // the pairs of a system's new elements: grid of up to 256 workgroups per system
    const u32 gx = std::max<u32>(1, std::min<u32>(maxrho, glob ? 64u : 256u));
    DBuf<u32> se(&c.pool, 2 * ntot), small(&c.pool, (u64)S * (2 + 256 + 8));
    fill_u32(small.ptr, (u64)S * (2 + 256 + 8), 0, s);
    DBuf<u64> cE;
    DBuf<u32> cW;
    if (glob) {
        cE.reset(&c.pool, (u64)S * gx * ccap);
        cW.reset(&c.pool, (u64)S * gx * ccap * 3);
    }
    std::vector<GmSeg> segs(S);
    u64 sb = 0;
    for (u32 i = 0; i < S; ++i) {
        const GmInsert& a = v[i];
        DevPairs& P = *a.P;
        GmSeg& g = segs[i];
        std::memset(&g, 0, sizeof(g));
        g.lm = a.lm;
        g.act = a.act;
        g.se = se.ptr + sb;
        sb += 2ull * (a.h0 + a.rho);
        g.plcm = P.lcm[P.cur].ptr;
        g.pij = P.ij[P.cur].ptr;
        g.pborn = P.born.ptr;
        g.ctr = small.ptr + 2ull * i;
        g.hist = small.ptr + 2ull * S + 256ull * i;
        g.sum = small.ptr + 258ull * S + 8ull * i;
        if (glob) {
            const u64 o = (u64)i * gx * ccap;
            g.cE = cE.ptr + o;
            g.cI = cW.ptr + 3 * o;
            g.cInfo = g.cI + (u64)gx * ccap;
            g.cBig = g.cInfo + (u64)gx * ccap;
        }
        g.n = a.n;
        g.h0 = a.h0;
        g.rho = a.rho;
        g.p0 = P.count;
        g.cap = (u32)P.cap;
        g.ccap = glob ? (u32)ccap : GM_CAND_LDS;
    }
    DBuf<GmSeg> dsegs(&c.pool, S);
    upload(c, dsegs.ptr, segs.data(), S * sizeof(GmSeg));
    const u32 bx = std::max<u32>(1, std::min<u32>(64, ceil_div(maxnp, 256)));
    hipLaunchKernelGGL(k_gm_ends, dim3(bx, S), dim3(256), 0, s, dsegs.ptr);
    F4_LAUNCH_CHECK();
    if (maxrho) {
        hipLaunchKernelGGL(k_gm_pairs, dim3(gx, S), dim3(GM_THREADS), 0, s, dsegs.ptr);
        F4_LAUNCH_CHECK();
    }
    u64 maxcap = 1;
    for (const GmInsert& a : v) maxcap = std::max<u64>(maxcap, a.P->cap);
    const u32 px = std::max<u32>(1, std::min<u32>(std::max<u32>(4, 1024 / S), ceil_div(maxcap, 256)));
    hipLaunchKernelGGL(k_gm_prune, dim3(px, S), dim3(256), 0, s, dsegs.ptr);
    F4_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gm_summary, dim3(S), dim3(256), 0, s, dsegs.ptr);
    F4_LAUNCH_CHECK();
    std::vector<u32> sum(8ull * S);
    readback(c, sum.data(), small.ptr + 258ull * S, sum.size() * 4);
    for (u32 i = 0; i < S; ++i) {
        const u32* q = sum.data() + 8ull * i;
        if (q[5]) throw F4Error{5, "pair set overflowed its room"};
        DevPairs& P = *v[i].P;
        P.count = q[0];
        P.kept = q[1];
        P.dmin = q[2];
        P.nsel = q[3];
        P.nact = q[4];
    }
}

void gm_select_batch(Ctx& c, const std::vector<GmSelect>& v, u64* rows_t, u32* rows_k, u32* outs,
                     u32* active_out) {
    const u32 S = (u32)v.size();
    if (!S) return;
    hipStream_t s = c.stream;
    std::vector<GmSel> segs(S);
    u64 gkeys = 0;
    for (const GmSelect& a : v)
        if (2ull * a.P->nsel > GM_SEL_LDS) gkeys += 4ull * a.P->nsel;
    DBuf<u64> gk(&c.pool, std::max<u64>(gkeys, 1));
    DBuf<u32> gv(&c.pool, std::max<u64>(gkeys, 1));
    u64 go = 0;
    bool lds = false;
    for (u32 i = 0; i < S; ++i) {
        const GmSelect& a = v[i];
        DevPairs& P = *a.P;
        if (!P.nsel || P.dmin != a.d) throw F4Error{5, "selection of a degree without pairs"};
        GmSel& g = segs[i];
        std::memset(&g, 0, sizeof(g));
        g.plcm = P.lcm[P.cur].ptr;
        g.pij = P.ij[P.cur].ptr;
        g.qlcm = P.lcm[P.cur ^ 1].ptr;
        g.qij = P.ij[P.cur ^ 1].ptr;
        g.lm = a.lm;
        g.act = a.act;
        g.binom = rank_table(c, a.n, a.d);
        g.room = 2 * P.nsel;
        if (2ull * P.nsel > GM_SEL_LDS) {
            g.keys = gk.ptr + go;
            g.vals = gv.ptr + go;
            go += 4ull * P.nsel;
        } else {
            lds = true;
        }
        g.count = P.count;
        g.npolys = a.npolys;
        g.n = a.n;
        g.d = a.d;
        g.kbits = std::max<u32>(1, gm_bitlen(a.npolys - 1));
        g.hibit = g.kbits + std::max<u32>(1, gm_bitlen(binom_host(a.n + a.d, a.n) - 1));
        if (g.hibit > 64) throw F4Error{2, "half key does not fit 64 bits"};
        g.row_base = a.row_base;
        g.act_base = a.act_base;
        g.act_room = P.nact;
        g.out = outs + 4ull * i;
    }
    DBuf<GmSel> dsegs(&c.pool, S);
    upload(c, dsegs.ptr, segs.data(), S * sizeof(GmSel));
    const size_t shm = lds ? (size_t)GM_SEL_LDS * 2 * (sizeof(u64) + sizeof(u32)) : 0;
    hipLaunchKernelGGL(k_gm_select, dim3(S), dim3(GM_SEL_THREADS), shm, s, dsegs.ptr, rows_t, rows_k, active_out);
    F4_LAUNCH_CHECK();
    for (u32 i = 0; i < S; ++i) {
        DevPairs& P = *v[i].P;
        P.count = P.kept - P.nsel;  // the pairs left, now in the other buffer
        P.kept = P.count;
        P.nsel = 0;
        P.cur ^= 1;
    }
}
