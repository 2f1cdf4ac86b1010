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
// degree and, in the last workgroup of each system, reads the least degree and
// its count off that.
//
// Selection (k_gm_pick): the pairs of the least degree d leave the set and
// give their two halves (lcm / LM(i), i) and (lcm / LM(j), j), deduplicated
// through a hash set keyed by (rank of the lcm, element); the rows come out
// in no particular order, since the symbolic preprocessing orders its rows
// itself.  The pruning kernel compacts the surviving pairs into the second
// buffer and writes the active list (descending index) that the reducer
// search reads.
//
// Exponents are compared lane by lane whenever a word has a lane's top bit
// set; the lane-parallel forms below are used only where they are exact.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

#define GM_DEAD 0xffffffffu   // i of a removed pair
#define GM_THREADS 256
#define GM_CAND_LDS 2048      // candidates of one new element held in LDS
#define GM_EMIT 512           // new pairs of one element collected in LDS before the buffer
#define GM_NO_DEG 0xffffffffu
#define GM_TAB_LDS 2048       // words of the rank table held in LDS

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
    u64* qlcm;     // the other buffer: the pairs that survive, compacted
    u32* qij;
    u32* ctr;      // [0] pairs in the buffer (insertion counter), [1] overflow bits, [2] prune workgroups
                   // done, [3] survivors
    u32* hist;     // surviving pairs per lcm degree (256 words, cleared by k_gm_ends)
    u32* sum;      // 8 summary words out
    u64* cE;       // candidate scratch in global memory (nullptr: LDS), ccap per workgroup
    u32* cI;
    u32* cInfo;
    u32* cBig;
    u32* alist;          // active elements out, descending index (room for h0 + rho)
    const u32* sel_out;  // the selection that preceded this update (4 words) or nullptr
    u32 sel_halves;      // the halves it had to find
    u32 n, h0, rho, p0;
    u32 cap, ccap;
};

// Leading monomials of the step's new elements, staged in LDS when they fit.
#define GM_NEW_LDS 4096
__device__ __forceinline__ const u64* gm_stage_new(const GmSeg& G, u64* buf) {
    const bool fit = G.rho <= GM_NEW_LDS;
    if (fit)
        for (u32 t = threadIdx.x; t < G.rho; t += blockDim.x) buf[t] = G.lm[G.h0 + t];
    __syncthreads();
    return fit ? buf : G.lm + G.h0;
}

// Windows of every element of the system and the new activity flags (one
// wave per element, lanes over the new elements), and the insertion counter
// set to the pairs already present.
__global__ __launch_bounds__(256) void k_gm_ends(const GmSeg* segs) {
    __shared__ u64 s_new[GM_NEW_LDS];
    const GmSeg G = segs[blockIdx.y];
    const GmLanes m = gm_lanes(G.n);
    const u64* LH = gm_stage_new(G, s_new);
    const u32 np = G.h0 + G.rho, lane = lane_id();
    if (blockIdx.x == 0) {
        for (u32 b = threadIdx.x; b < 256; b += blockDim.x) G.hist[b] = 0;
        if (threadIdx.x == 0) {
            G.ctr[0] = G.p0;
            G.ctr[1] = 0;
            G.ctr[2] = 0;
            G.ctr[3] = 0;
            if (G.sel_out && G.sel_out[3] != G.sel_halves) G.ctr[1] = 8u;
        }
    }
    const u32 waves = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 g = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; g < np; g += waves) {
        const bool old = g < G.h0;
        u32 start = old ? 0u : g - G.h0 + 1, end = G.rho + 1;
        if (old && !G.act[g]) {
            start = 1;
            end = 0;  // never a candidate
        } else {
            const u64 l = G.lm[g];
            for (u32 t0 = start; t0 < G.rho; t0 += F4_WAVE) {
                const u32 t = t0 + lane;
                const u64 hit = wave_ballot(t < G.rho && gm_div(m, LH[t], l));
                if (hit) {
                    end = t0 + (u32)__builtin_ctzll(hit) + 1;  // h_t still pairs with g, then retires it
                    break;
                }
            }
        }
        if (lane == 0) {
            G.se[2 * g] = start;
            G.se[2 * g + 1] = end;
            G.act[g] = end == G.rho + 1 ? 1u : 0u;
        }
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
    __shared__ u64 s_el[GM_EMIT];  // this element's new pairs: lcm and partner
    __shared__ u32 s_eg[GM_EMIT];
    __shared__ u32 s_ne, s_eb;
    const GmSeg G = segs[blockIdx.y];
    const GmLanes m = gm_lanes(G.n);
    const u32 tid = threadIdx.x;
    const bool glob = G.cE != nullptr;
    // collect locally; past GM_EMIT, straight to the buffer
    auto emit = [&](u32 g, u32 h, u64 l, u32 t) {
        const u32 k = atomicAdd(&s_ne, 1u);
        if (k < GM_EMIT) {
            s_el[k] = l;
            s_eg[k] = g;
        } else {
            gm_emit(G, g, h, l, t);
        }
    };
    // the element's collected pairs to the buffer: one atomic per element
    auto flush = [&](u32 h, u32 t) {
        __syncthreads();
        const u32 ne = min(s_ne, (u32)GM_EMIT);
        if (tid == 0) s_eb = ne ? atomicAdd(&G.ctr[0], ne) : 0u;
        __syncthreads();
        for (u32 x = tid; x < ne; x += GM_THREADS) {
            const u32 k = s_eb + x;
            if (k < G.cap) {
                G.plcm[k] = s_el[x];
                G.pij[2 * k] = s_eg[x];
                G.pij[2 * k + 1] = h;
                G.pborn[k] = t;
            } else {
                atomicOr(&G.ctr[1], 1u);
            }
        }
        __syncthreads();
    };
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
            s_ne = 0;
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
            if (tid == 0 && !s_cop0) emit(s_last0 - 1, h, lh, t);
            flush(h, t);
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
            if (ok) emit(ga, h, (lhl + ea) | ((u64)(dh + da) << 56), t);
        }
        if (tid < m.n && s_last1[tid] && !s_cop1[tid])
            emit(s_last1[tid] - 1, h, (lhl + (1ull << (m.w * tid))) | ((u64)(dh + 1) << 56), t);
        flush(h, t);
    }
}

// Removal of the pairs that a later element witnesses (LM(h_u) divides the
// lcm and differs from both lcm(LM(i), LM(h_u)) and lcm(LM(h_u), LM(j))):
// GM_GROUP lanes per pair, each taking every GM_GROUP-th candidate witness.
// The pairs that stay are compacted into the other buffer and counted by lcm
// degree.  The last workgroup of a system to finish writes the active list
// (descending index) and the summary: surviving pairs, least lcm degree and
// its count, active elements, overflow bits.
#define GM_GROUP 8
#define GM_SURV 1024  // surviving pairs collected in LDS between flushes
__global__ __launch_bounds__(256) void k_gm_prune(const GmSeg* segs) {
    __shared__ u64 s_new[GM_NEW_LDS];
    __shared__ u64 s_ql[GM_SURV];
    __shared__ u32 s_qi[GM_SURV], s_qj[GM_SURV];
    __shared__ u32 sh[256];
    __shared__ u32 s_wave[33];
    __shared__ u32 s_last, s_dmin, s_n, s_base;
    const GmSeg G = segs[blockIdx.y];
    const GmLanes m = gm_lanes(G.n);
    const u32 tid = threadIdx.x, lane = lane_id();
    const u32 sub = lane % GM_GROUP, grp = lane / GM_GROUP;
    sh[tid] = 0;
    if (tid == 0) s_n = 0;
    const u64* LH = gm_stage_new(G, s_new);  // (synchronizes)
    const u32 cnt = min(G.ctr[0], G.cap);
    // a contiguous range of pairs per workgroup
    const u32 span = (cnt + gridDim.x - 1) / gridDim.x;
    const u32 b0 = min(cnt, blockIdx.x * span), b1 = min(cnt, b0 + span);
    auto flush = [&]() {  // (called by every thread, after a barrier)
        const u32 nq = s_n;
        if (tid == 0) s_base = nq ? atomicAdd(&G.ctr[3], nq) : 0u;
        __syncthreads();
        for (u32 x = tid; x < nq; x += blockDim.x) {
            const u32 k = s_base + x;
            if (k < G.cap) {
                G.qlcm[k] = s_ql[x];
                G.qij[2 * k] = s_qi[x];
                G.qij[2 * k + 1] = s_qj[x];
            }
        }
        __syncthreads();
        if (tid == 0) s_n = 0;
        __syncthreads();
    };
    // no barrier in the loop: survivors past GM_SURV go straight to the
    // buffer (one atomic each; the host aims at ranges of about 256).  Each wave
    // loads 64 pairs at once (a lane each), then its GM_GROUP-lane groups take
    // them GM_GROUP at a time with the data broadcast from the loading lane.
    const u32 wave = tid / F4_WAVE, nwave = blockDim.x / F4_WAVE;
    for (u32 base = b0 + wave * F4_WAVE; base < b1; base += nwave * F4_WAVE) {
        const u32 q = base + lane;
        u32 i = GM_DEAD, j = 0, from = 0;
        u64 l = 0, li = 0, lj = 0;
        if (q < b1) {
            i = G.pij[2 * q];
            if (i != GM_DEAD) {
                j = G.pij[2 * q + 1];
                l = G.plcm[q];
                li = G.lm[i];
                lj = G.lm[j];
                from = q < G.p0 ? 0u : G.pborn[q] + 1;
            }
        }
        for (u32 r = 0; r < F4_WAVE / GM_GROUP; ++r) {
            const int src = (int)(r * GM_GROUP + grp);
            const u32 bi = __shfl(i, src, F4_WAVE), bj = __shfl(j, src, F4_WAVE), bf = __shfl(from, src, F4_WAVE);
            const u64 bl = ((u64)__shfl((u32)(l >> 32), src, F4_WAVE) << 32) | __shfl((u32)l, src, F4_WAVE);
            const u64 bli = ((u64)__shfl((u32)(li >> 32), src, F4_WAVE) << 32) | __shfl((u32)li, src, F4_WAVE);
            const u64 blj = ((u64)__shfl((u32)(lj >> 32), src, F4_WAVE) << 32) | __shfl((u32)lj, src, F4_WAVE);
            const bool live = bi != GM_DEAD;
            bool hit = false;
            if (live) {
                const u64 ll = bl & m.lanes;
                for (u32 t = bf + sub; t < G.rho; t += GM_GROUP) {
                    const u64 lh = LH[t];
                    if (gm_div(m, lh, bl) && gm_lcm(m, bli, lh) != ll && gm_lcm(m, lh, blj) != ll) {
                        hit = true;
                        break;
                    }
                }
            }
            const u64 bal = wave_ballot(hit);
            const bool alive = live && ((bal >> (grp * GM_GROUP)) & ((1ull << GM_GROUP) - 1)) == 0;
            if (alive && sub == 0) {
                const u32 k = atomicAdd(&s_n, 1u);
                if (k < GM_SURV) {
                    s_ql[k] = bl;
                    s_qi[k] = bi;
                    s_qj[k] = bj;
                } else {
                    const u32 x = atomicAdd(&G.ctr[3], 1u);
                    if (x < G.cap) {
                        G.qlcm[x] = bl;
                        G.qij[2 * x] = bi;
                        G.qij[2 * x + 1] = bj;
                    }
                }
                atomicAdd(&sh[mono_deg(bl)], 1u);
            }
        }
    }
    __syncthreads();
    if (tid == 0) s_n = min(s_n, (u32)GM_SURV);
    __syncthreads();
    flush();
    if (sh[tid]) atomicAdd(&G.hist[tid], sh[tid]);
    // the last workgroup of the system sees every histogram update
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&G.ctr[2], 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (tid == 0) s_dmin = GM_NO_DEG;
    __syncthreads();
    const u32 c = atomicAdd(&G.hist[tid], 0u);
    if (c) atomicMin(&s_dmin, tid);
    u32 kept;
    (void)block_exclusive_scan(c, s_wave, &kept);
    u32 na = 0;
    const u32 np = G.h0 + G.rho;
    for (u32 x0 = 0; x0 < np; x0 += 256) {
        const u32 x = x0 + tid;
        const u32 g = np - 1 - x;
        const bool a = x < np && G.act[g];
        u32 tot;
        const u32 pos = na + block_exclusive_scan(a ? 1u : 0u, s_wave, &tot);
        if (a) G.alist[pos] = g;
        na += tot;
    }
    if (tid == 0) {
        const u32 cn = G.ctr[0], sv = atomicAdd(&G.ctr[3], 0u);
        G.sum[0] = sv;
        G.sum[1] = kept;
        G.sum[2] = s_dmin;
        G.sum[3] = s_dmin == GM_NO_DEG ? 0u : atomicAdd(&G.hist[s_dmin], 0u);
        G.sum[4] = na;
        G.sum[5] = G.ctr[1] | (cn > G.cap ? 1u : 0u) | (sv > G.cap || sv != kept ? 4u : 0u);
        G.sum[6] = 0;
        G.sum[7] = 0;
    }
}

// One system's selection.
struct GmSel {
    u64* plcm;
    u32* pij;
    const u64* lm;
    const u32* binom;  // rank table of (n, d)
    u32 tabn;          // its words
    u64* table;        // hash set of the halves' keys (key + 1; 0 empty), tsize entries, zero on entry
    u32 tsize;         // a power of two, at least twice the halves
    u32 room;          // halves expected (2 * pairs of degree d)
    u32 count, n, d, kbits;
    u32 row_base;
    u32* out;  // [0] rows, [3] halves found (zero on entry)
};

// The pairs of degree d leave the set (marked removed in place); each of
// their halves (lcm / LM(k), k) is entered in the system's hash set under the
// key (rank of the lcm, k), and the first to enter a key writes the row.  The
// rows come out unordered (the symbolic preprocessing orders them).  Each
// workgroup takes a contiguous range of pairs and collects its rows in LDS.
#define GM_ROWBUF 1024
__global__ __launch_bounds__(256) void k_gm_pick(const GmSel* segs, u64* rows_t, u32* rows_k) {
    __shared__ u32 s_tab[GM_TAB_LDS];
    __shared__ u64 s_rt[GM_ROWBUF];
    __shared__ u32 s_rk[GM_ROWBUF];
    __shared__ u32 s_n, s_base, s_halves;
    const GmSel G = segs[blockIdx.y];
    const u32 tid = threadIdx.x;
    const u32 w = lane_bits(G.n);
    const bool tab_lds = G.tabn <= GM_TAB_LDS;
    if (tab_lds)
        for (u32 i = tid; i < G.tabn; i += blockDim.x) s_tab[i] = G.binom[i];
    if (tid == 0) {
        s_n = 0;
        s_halves = 0;
    }
    __syncthreads();
    const u32* tab = tab_lds ? s_tab : G.binom;
    const u32 tbits = 31 - __clz(G.tsize);
    const u32 span = (G.count + gridDim.x - 1) / gridDim.x;
    const u32 b0 = min(G.count, blockIdx.x * span), b1 = min(G.count, b0 + span);
    auto flush = [&]() {  // (called by every thread, after a barrier)
        const u32 nr = s_n;
        if (tid == 0) s_base = nr ? atomicAdd(&G.out[0], nr) : 0u;
        __syncthreads();
        for (u32 x = tid; x < nr; x += blockDim.x) {
            const u32 k = s_base + x;
            if (k < G.room) {
                rows_t[G.row_base + k] = s_rt[x];
                rows_k[G.row_base + k] = s_rk[x];
            }
        }
        __syncthreads();
        if (tid == 0) s_n = 0;
        __syncthreads();
    };
    for (u32 q0 = b0; q0 < b1; q0 += blockDim.x) {
        if (s_n + 2 * blockDim.x > GM_ROWBUF) flush();  // (s_n is uniform here: read after a barrier)
        const u32 q = q0 + tid;
        if (q < b1) {
            const u32 i = G.pij[2 * q];
            const u64 l = i != GM_DEAD ? G.plcm[q] : 0ull;
            if (i != GM_DEAD && mono_deg(l) == G.d) {
                const u32 j = G.pij[2 * q + 1];
                G.pij[2 * q] = GM_DEAD;
                atomicAdd(&s_halves, 2u);
                const u64 r = (u64)mono_rank(l, G.n, w, G.d, tab) << G.kbits;
                for (int side = 0; side < 2; ++side) {
                    const u32 k = side ? j : i;
                    const u64 key = (r | k) + 1;
                    u32 h = (u32)((key * 0x9e3779b97f4a7c15ull) >> (64 - tbits));
                    for (u32 probe = 0; probe < G.tsize; ++probe) {
                        const u64 prev =
                            atomicCAS((unsigned long long*)&G.table[h], 0ull, (unsigned long long)key);
                        if (prev == 0) {  // first: this half is a row
                            const u32 x = atomicAdd(&s_n, 1u);
                            s_rt[x] = l - G.lm[k];
                            s_rk[x] = k;
                            break;
                        }
                        if (prev == key) break;
                        h = (h + 1) & (G.tsize - 1);
                    }
                }
            }
        }
        __syncthreads();
    }
    flush();
    if (tid == 0 && s_halves) atomicAdd(&G.out[3], s_halves);
}

static u32 gm_bitlen(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// Growth copies of a batch, done by one launch (the old buffers are kept
// until it is enqueued).
struct GmCopies {
    std::vector<u64> src, dst, words;  // device pointers (as integers) and 4-byte words
    std::vector<DBuf<u64>> keep64;
    std::vector<DBuf<u32>> keep32;
};

__global__ void k_gm_copies(const u64* src, const u64* dst, const u64* words, u32 njobs) {
    const u32 jb = blockIdx.y;
    if (jb >= njobs) return;
    const u32* a = (const u32*)src[jb];
    u32* b = (u32*)dst[jb];
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < words[jb]; i += (u64)gridDim.x * blockDim.x)
        b[i] = a[i];
}

static void gm_copies_flush(Ctx& c, GmCopies& cp) {
    const u32 nj = (u32)cp.src.size();
    if (nj) {
        if (nj > 65535) throw F4Error{2, "too many pair-set copies"};
        std::vector<u64> pack;
        pack.insert(pack.end(), cp.src.begin(), cp.src.end());
        pack.insert(pack.end(), cp.dst.begin(), cp.dst.end());
        pack.insert(pack.end(), cp.words.begin(), cp.words.end());
        DBuf<u64> d(&c.pool, pack.size());
        upload(c, d.ptr, pack.data(), pack.size() * 8);
        u64 mx = 1;
        for (u64 w : cp.words) mx = std::max(mx, w);
        hipLaunchKernelGGL(k_gm_copies, dim3(std::min<u64>(64, (mx + 255) / 256), nj), dim3(256), 0, c.stream,
                           d.ptr, d.ptr + nj, d.ptr + 2 * nj, nj);
        F4_LAUNCH_CHECK();
    }
    cp = GmCopies();
}

static void gm_grow(Ctx& c, DevPairs& P, u64 need, GmCopies& cp) {
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
        cp.src.push_back((u64)(uintptr_t)P.lcm[P.cur].ptr);
        cp.dst.push_back((u64)(uintptr_t)Q.lcm[0].ptr);
        cp.words.push_back(2ull * P.count);
        cp.src.push_back((u64)(uintptr_t)P.ij[P.cur].ptr);
        cp.dst.push_back((u64)(uintptr_t)Q.ij[0].ptr);
        cp.words.push_back(2ull * P.count);
    }
    for (int b = 0; b < 2; ++b) {
        cp.keep64.push_back(std::move(P.lcm[b]));
        cp.keep32.push_back(std::move(P.ij[b]));
        P.lcm[b] = std::move(Q.lcm[b]);
        P.ij[b] = std::move(Q.ij[b]);
    }
    cp.keep32.push_back(std::move(P.born));
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
    u64 ntot = 0, ccap = 1, maxcnt = 1;
    u32 maxrho = 0, maxnp = 1;
    bool glob = false;
    GmCopies cp;
    for (const GmInsert& a : v) {
        DevPairs& P = *a.P;
        const u64 cand = (u64)P.nact + a.rho;
        const u64 room = (u64)P.count + (u64)a.rho * P.nact + (u64)a.rho * (a.rho ? a.rho - 1 : 0) / 2;
        gm_grow(c, P, std::max<u64>(room, 64), cp);
        const u64 np = (u64)a.h0 + a.rho;
        if (np > P.acap) {  // the active list (written whole by every update: nothing to copy)
            P.acap = std::max<u64>(np, 2 * P.acap);
            P.alist.reset(&c.pool, P.acap);
        }
        ntot += np;
        ccap = std::max<u64>(ccap, cand);
        maxcnt = std::max<u64>(maxcnt, room);
        maxrho = std::max(maxrho, a.rho);
        maxnp = std::max<u32>(maxnp, (u32)np);
        if (cand > GM_CAND_LDS) glob = true;
    }
    if (ntot >= (1ull << 31)) throw F4Error{2, "basis too large"};
    gm_copies_flush(c, cp);
    // the pairs of a system's new elements: grid of up to 256 workgroups per system
    const u32 gx = std::max<u32>(1, std::min<u32>(maxrho, glob ? 64u : 256u));
    // counters, histograms (both set by k_gm_ends) and summaries
    const u64 small_words = (u64)S * (4 + 256 + 8);
    DBuf<u32> se(&c.pool, 2 * ntot), small(&c.pool, small_words);
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
        g.qlcm = P.lcm[P.cur ^ 1].ptr;
        g.qij = P.ij[P.cur ^ 1].ptr;
        g.ctr = small.ptr + 4ull * i;
        g.hist = small.ptr + 4ull * S + 256ull * i;
        g.sum = small.ptr + 260ull * S + 8ull * i;
        if (glob) {
            const u64 o = (u64)i * gx * ccap;
            g.cE = cE.ptr + o;
            g.cI = cW.ptr + 3 * o;
            g.cInfo = g.cI + (u64)gx * ccap;
            g.cBig = g.cInfo + (u64)gx * ccap;
        }
        g.alist = P.alist.ptr;
        g.sel_out = a.sel_out;
        g.sel_halves = a.sel_halves;
        g.n = a.n;
        g.h0 = a.h0;
        g.rho = a.rho;
        g.p0 = P.count;
        g.cap = (u32)P.cap;
        g.ccap = glob ? (u32)ccap : GM_CAND_LDS;
    }
    DBuf<GmSeg> dsegs(&c.pool, S);
    upload(c, dsegs.ptr, segs.data(), S * sizeof(GmSeg));
    // workgroups per system: what the largest system needs, within a budget of
    // about 1024 for the batch (the kernels stride over what is left)
    const u32 per_sys = std::max<u32>(1, 1024 / S);
    const u32 bx = std::max<u32>(1, std::min<u32>(per_sys, ceil_div(maxnp, 4)));  // a wave per element
    hipLaunchKernelGGL(k_gm_ends, dim3(bx, S), dim3(256), 0, s, dsegs.ptr);
    F4_LAUNCH_CHECK();
    if (maxrho) {
        hipLaunchKernelGGL(k_gm_pairs, dim3(gx, S), dim3(GM_THREADS), 0, s, dsegs.ptr);
        F4_LAUNCH_CHECK();
    }
    // about 256 pairs per workgroup
    const u32 px = std::max<u32>(1, std::min<u32>(per_sys, ceil_div(maxcnt, 256)));
    hipLaunchKernelGGL(k_gm_prune, dim3(px, S), dim3(256), 0, s, dsegs.ptr);
    F4_LAUNCH_CHECK();
    std::vector<u32> sum(8ull * S);
    readback(c, sum.data(), small.ptr + 260ull * S, sum.size() * 4);
    for (u32 i = 0; i < S; ++i) {
        const u32* q = sum.data() + 8ull * i;
        if (q[5] & 8u) throw F4Error{5, "the selection disagreed with the pair set's summary"};
        if (q[5]) throw F4Error{5, "pair set overflowed its room"};
        DevPairs& P = *v[i].P;
        P.cur ^= 1;  // the survivors, compacted
        P.count = q[0];
        P.kept = q[1];
        P.dmin = q[2];
        P.nsel = q[3];
        P.nact = q[4];
    }
}

u32* gm_select_batch(Ctx& c, const std::vector<GmSelect>& v, u64* rows_t, u32* rows_k, DBuf<u64>& keep) {
    const u32 S = (u32)v.size();
    if (!S) return nullptr;
    hipStream_t s = c.stream;
    std::vector<GmSel> segs(S);
    u64 tab_tot = 0, maxcount = 1;
    std::vector<u32> tsz(S);
    for (u32 i = 0; i < S; ++i) {
        const DevPairs& P = *v[i].P;
        u32 t = 64;
        while (t < 4ull * P.nsel) t <<= 1;  // load factor at most 1/2
        tsz[i] = t;
        tab_tot += t;
        maxcount = std::max<u64>(maxcount, P.count);
    }
    // the hash sets and the output words in one block, cleared by one launch
    keep.reset(&c.pool, tab_tot + 2ull * S);
    fill_u64(keep.ptr, tab_tot + 2ull * S, 0, s);
    u64* const table = keep.ptr;
    u32* const outs = (u32*)(keep.ptr + tab_tot);
    u64 o = 0;
    for (u32 i = 0; i < S; ++i) {
        const GmSelect& a = v[i];
        DevPairs& P = *a.P;
        if (!P.nsel || P.dmin != a.d) throw F4Error{5, "selection of a degree without pairs"};
        GmSel& g = segs[i];
        std::memset(&g, 0, sizeof(g));
        g.plcm = P.lcm[P.cur].ptr;
        g.pij = P.ij[P.cur].ptr;
        g.lm = a.lm;
        g.binom = rank_table(c, a.n, a.d);
        g.tabn = (a.n + a.d + 2) * F4_BSTRIDE;
        g.table = table + o;
        g.tsize = tsz[i];
        o += tsz[i];
        g.room = 2 * P.nsel;
        g.count = P.count;
        g.n = a.n;
        g.d = a.d;
        g.kbits = std::max<u32>(1, gm_bitlen(a.npolys - 1));
        if (g.kbits + gm_bitlen(binom_host(a.n + a.d, a.n)) > 63) throw F4Error{2, "half key does not fit 64 bits"};
        g.row_base = a.row_base;
        g.out = outs + 4ull * i;
    }
    DBuf<GmSel> dsegs(&c.pool, S);
    upload(c, dsegs.ptr, segs.data(), S * sizeof(GmSel));
    const u32 bx = std::max<u32>(1, std::min<u32>(std::max<u32>(1, 1024 / S), ceil_div(maxcount, 256)));
    hipLaunchKernelGGL(k_gm_pick, dim3(bx, S), dim3(256), 0, s, dsegs.ptr, rows_t, rows_k);
    F4_LAUNCH_CHECK();
    for (u32 i = 0; i < S; ++i) {
        DevPairs& P = *v[i].P;
        P.kept -= P.nsel;  // marked removed in place; the next update compacts them away
        P.nsel = 0;
    }
    return outs;
}
