// Symbolic preprocessing SP : B -> (T, R, Pi) on gfx950 for a batch of
// independent systems (Definition "Symbolic preprocessing operator";
// Algorithm "FBSP"; section "FBSP: frontier-based symbolic preprocessing as
// bulk set algebra").  One launch of each kernel covers every system of the
// batch: per-system work uses a 2-D grid (blockIdx.y = system), flat work
// carries a system index per element.  A single system is the batch of one.
//
// Monomials of a step all have degree <= D, so the dictionary T lives inside
// Mon_{<=D}, which the dense grevlex rank maps order-isomorphically onto
// [0, N(n, D)).  Two dictionary paths share the closure:
//   * dense rank (default): the frontier multiset is setified into a bitmap
//     over ranks (a counting sort: sort + unique in one pass), the column of a
//     monomial is the popcount prefix of its rank, and the join of every row
//     term with the dictionary is a table lookup fused into the fill;
//   * radix sort (the pipeline as the algorithm states it): the fill
//     materialises a compact order key per row term, the keys are radix
//     sorted on their live bits, deduplicated, and every term is joined to its
//     dictionary position by binary search.
// The closure rounds (Remark "Truncation and why symbolic preprocessing
// matters", Definition "Support-closure for correctness") are bulk: frontier =
// (monomials seen) minus (monomials processed), one reducer per frontier
// monomial, new rows emit their supports, repeat until the frontier is empty.
#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "sig.hpp"
#include "sort_lds.hpp"

#define MB_THREADS 256
#define MB_WAVES (MB_THREADS / F4_WAVE)
#define RED_BUF 16      // reducer rows a wave buffers before one append
#define MK_THREADS 1024  // row marking: sixteen waves per workgroup share one LDS bitmap
#define MK_WAVES (MK_THREADS / F4_WAVE)

// ----------------------------------------------------------- rank tables
u64 binom_host(u32 x, u32 y) {
    if (y > x) return 0;
    u64 r = 1;
    for (u32 i = 1; i <= y; ++i) r = r * (x - y + i) / i;
    return r;
}

const u32* rank_table(Ctx& c, u32 n, u32 D) {
    auto key = std::make_pair(n, D);
    auto it = c.binom.find(key);
    if (it != c.binom.end()) return it->second.ptr;
    const u32 rows = n + D + 2;
    std::vector<u32> tab((size_t)rows * F4_BSTRIDE, 0);
    for (u32 x = 0; x < rows; ++x)
        for (u32 y = 0; y < F4_BSTRIDE; ++y) {
            u64 v = binom_host(x, y);
            tab[(size_t)x * F4_BSTRIDE + y] = v > 0xffffffffull ? 0xffffffffu : (u32)v;
        }
    DBuf<u32> buf(&c.pool, tab.size());
    upload(c, buf.ptr, tab.data(), tab.size() * 4);
    const u32* p = buf.ptr;
    c.binom.emplace(key, std::move(buf));
    return p;
}

__global__ void k_unrank_all(u64* out, u32 nmax, u32 n, u32 w, u32 D, const u32* B) {
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < nmax; q += gridDim.x * blockDim.x)
        out[q] = mono_unrank(q, n, w, D, B);
}

const u64* unrank_table(Ctx& c, u32 n, u32 D) {
    auto key = std::make_pair(n, D);
    auto it = c.montab.find(key);
    if (it != c.montab.end()) return it->second.ptr;
    const u32* B = rank_table(c, n, D);
    u32 nmax = (u32)binom_host(n + D, n);
    DBuf<u64> buf(&c.pool, nmax);
    hipLaunchKernelGGL(k_unrank_all, dim3(std::min<u32>(ceil_div(nmax, 256), 4096)), dim3(256), 0, c.stream, buf.ptr,
                       nmax, n, lane_bits(n), D, B);
    F4_LAUNCH_CHECK();
    const u64* p = buf.ptr;
    c.montab.emplace(key, std::move(buf));
    return p;
}

// ----------------------------------------------------- per-system descriptor
struct SegSP {
    const u64* mon;
    const u32* coeff;
    const u64* off;
    const u64* lm;
    const u32* len;
    const u32* binom;
    const u64* montab;
    u32 n, w, D, nmax;
    u32 wbase, nwords;   // bitmap words [wbase, wbase + nwords)
    u32 rbase, rcap;     // raw rows [rbase, rbase + rcap)
    u32 abase, nactive;  // active basis indices (descending)
    u32 tabn, npolys;
    u32 cmbase;          // colmap / dictionary capacity base
    u32 obase, r;        // ordered rows [obase, obase + r) (after the closure)
    u32 ibase, r0;       // initial rows in the packed upload (or the device rows: room)
    const u32* r0p;      // device rows: the actual count, on the device (else nullptr)
    const u32* actp;     // the system's own device active list (else nullptr: the batch's list at abase)
    const SigDev* sig;   // reducers restricted to admissible rows (else nullptr: any)
};

// counters per system: [0] row range begin, [1] row range end (= rows so
// far), [2] unused, [3] error (1 bad monomial, 2 row capacity, 4 signature
// overflow)
#define CTR 4

// ----------------------------------------------------------- row emission
// Rows of the current range of system blockIdx.y: record the rank of each
// row's leading monomial, mark it processed, and mark the rank of every term
// t * m of the row as seen.  One wave per row, lanes over terms; seen-bits are
// gathered in an LDS bitmap per workgroup, flushed with one atomic OR per
// nonzero word.
#define MK_UNROLL 4
__global__ __launch_bounds__(MK_THREADS) void k_mark_rows(const SegSP* segs, const u64* rows_t, const u32* rows_k,
                                                           u32* row_lmrank, u32* ctr, u32* present, u32* done,
                                                           u32* lead, int local_bitmap) {
    extern __shared__ u32 sm[];
    const SegSP S = segs[blockIdx.y];
    u32* C = ctr + CTR * blockIdx.y;
    const u32 rb = C[0], re = C[1];
    if (rb + blockIdx.x * MK_WAVES >= re) return;  // no row for this workgroup (uniform)
    u32* tab = sm;
    u32* lbits = sm + S.tabn;
    for (u32 i = threadIdx.x; i < S.tabn; i += MK_THREADS) tab[i] = S.binom[i];
    if (local_bitmap)
        for (u32 i = threadIdx.x; i < S.nwords; i += MK_THREADS) lbits[i] = 0;
    __syncthreads();
    u32* P = present + S.wbase;
    u32* Dn = done + S.wbase;
    u32* Ld = lead + S.wbase;
    const u32 n = S.n, w = S.w, D = S.D, lane = lane_id();
    const u32 nw_total = gridDim.x * MK_WAVES;
    for (u32 row = rb + blockIdx.x * MK_WAVES + threadIdx.x / F4_WAVE; row < re; row += nw_total) {
        const u64 t = rows_t[S.rbase + row];
        const u32 k = rows_k[S.rbase + row];
        if (lane == 0) {
            u32 q = mono_rank(t + S.lm[k], n, w, D, tab);
            if (q == F4_BAD_RANK) {
                C[3] = 1u;
                q = 0;
            }
            row_lmrank[S.rbase + row] = q;
            atomicOr(&Dn[q >> 5], 1u << (q & 31));
            atomicOr(&Ld[q >> 5], 1u << (q & 31));
        }
        const u64 off = S.off[k];
        const u32 len = S.len[k];
        // MK_UNROLL chunks of the row's terms are loaded before any is ranked:
        // one wait for memory per MK_UNROLL * 64 terms
        for (u32 j0 = 0; j0 < len; j0 += MK_UNROLL * F4_WAVE) {
            u64 mm[MK_UNROLL];
#pragma unroll
            for (u32 i = 0; i < MK_UNROLL; ++i) {
                const u32 j = j0 + i * F4_WAVE + lane;
                mm[i] = j < len ? S.mon[off + j] : 0;
            }
#pragma unroll
            for (u32 i = 0; i < MK_UNROLL; ++i) {
                if (j0 + i * F4_WAVE + lane >= len) continue;
                const u32 q = mono_rank(t + mm[i], n, w, D, tab);
                if (q == F4_BAD_RANK) {
                    C[3] = 1u;
                    continue;
                }
                if (local_bitmap)
                    atomicOr(&lbits[q >> 5], 1u << (q & 31));
                else
                    atomicOr(&P[q >> 5], 1u << (q & 31));
            }
        }
    }
    if (local_bitmap) {
        __syncthreads();
        for (u32 i = threadIdx.x; i < S.nwords; i += MK_THREADS) {
            const u32 v = lbits[i];
            if (v) atomicOr(&P[i], v);
        }
    }
}

// scatter the packed initial rows of every system into its row segment and
// clear the system's three bitmaps (W words apart) and its M counter
__global__ void k_init_rows(const SegSP* segs, const u64* t0, const u32* k0, u64* rows_t, u32* rows_k, u32* bitmaps,
                            u32 W, unsigned long long* M, u32* ctr) {
    const SegSP S = segs[blockIdx.y];
    const u32 r0 = S.r0p ? min(*S.r0p, S.r0) : S.r0;
    if (S.r0p && blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR * blockIdx.y + 1] = r0;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r0; i += gridDim.x * blockDim.x) {
        rows_t[S.rbase + i] = t0[S.ibase + i];
        rows_k[S.rbase + i] = k0[S.ibase + i];
    }
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < S.nwords; i += gridDim.x * blockDim.x) {
        bitmaps[S.wbase + i] = 0;
        bitmaps[W + S.wbase + i] = 0;
        bitmaps[2 * (u64)W + S.wbase + i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) M[blockIdx.y] = 0;
}

// frontier = seen and not processed (flat over all bitmap words)
__global__ void k_frontier_count(const u32* present, const u32* done, u32 nwords, u32* cnt) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x)
        cnt[i] = __popc(present[i] & ~done[i]);
}

// write the frontier ranks of system blockIdx.y (ascending), mark them
// processed, and open the system's next row range at its current row count
__global__ void k_frontier_write(const SegSP* segs, const u32* present, u32* done, const u32* off, u32* list_q,
                                 u32* list_s, u32* ctr) {
    const u32 s = blockIdx.y;
    const SegSP S = segs[s];
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < S.nwords; i += gridDim.x * blockDim.x) {
        const u32 wi = S.wbase + i;
        u32 f = present[wi] & ~done[wi];
        if (!f) continue;
        done[wi] |= f;
        u32 pos = off[wi];
        while (f) {
            const u32 b = __ffs(f) - 1;
            list_q[pos] = i * 32 + b;
            list_s[pos] = s;
            ++pos;
            f &= f - 1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR * s] = ctr[CTR * s + 1];
}

// Small bitmaps (W <= WORDS_SMALL words) in one workgroup: per word the count
// of its set bits (mode 2: present, and the leading-monomial bitmap into
// loff; modes 0, 1: present and not done), the exclusive offsets off[0..W]
// and, in mode 0, the frontier list in word and bit order with the words
// marked done - k_frontier_count + scan + k_frontier_write (or k_word_popc +
// scan) in one launch.
#define WORDS_SMALL 8192
__global__ __launch_bounds__(1024) void k_words_small(const SegSP* segs, u32 S, const u32* present, u32* done,
                                                      u32 W, int mode, u32* off, u32* list_q, u32* list_s,
                                                      u32* ctr, const u32* lead, u32* loff) {
    __shared__ u32 s_wave[33];
    const u32 tid = threadIdx.x;
    u32 carry = 0, lcarry = 0;
    for (u32 base = 0; base < W; base += 1024) {
        const u32 wi = base + tid;
        u32 f = 0;
        if (wi < W) f = mode == 2 ? present[wi] : (present[wi] & ~done[wi]);
        u32 tot;
        const u32 pre = block_exclusive_scan(__popc(f), s_wave, &tot);
        if (wi < W) off[wi] = carry + pre;
        if (mode == 2) {
            u32 ltot;
            const u32 lpre = block_exclusive_scan(wi < W ? __popc(lead[wi]) : 0u, s_wave, &ltot);
            if (wi < W) loff[wi] = lcarry + lpre;
            lcarry += ltot;
        }
        if (mode == 0 && f) {
            done[wi] |= f;
            u32 lo = 0, hi = S;  // system of the word: last s with wbase <= wi
            while (hi - lo > 1) {
                const u32 mid = (lo + hi) >> 1;
                if (segs[mid].wbase <= wi)
                    lo = mid;
                else
                    hi = mid;
            }
            const u32 i = wi - segs[lo].wbase;
            u32 pos = carry + pre;
            while (f) {
                const u32 b = __ffs(f) - 1;
                list_q[pos] = i * 32 + b;
                list_s[pos] = lo;
                ++pos;
                f &= f - 1;
            }
        }
        carry += tot;
    }
    if (tid == 0) {
        off[W] = carry;
        if (mode == 2) loff[W] = lcarry;
    }
    if (mode == 0)
        for (u32 sy = tid; sy < S; sy += 1024) ctr[CTR * sy] = ctr[CTR * sy + 1];
}

// One reducer per frontier monomial m: the active element with the largest
// index whose leading monomial divides m; the new row is (m / LM(g), g).
// With signatures, the largest such index whose row is admissible (the
// closure over the admissible reducers; m gets no row when there is none).
// Grid (blocks, systems): a system's frontier entries are contiguous in the
// list, and its active leading monomials are staged in LDS when they fit.
__global__ __launch_bounds__(MB_THREADS) void k_reducers(const SegSP* segs, const u32* list_q, const u32* fscan,
                                                          const u32* active, int lds_active, u64* rows_t,
                                                          u32* rows_k, u32* row_lmrank, u32* ctr) {
    extern __shared__ u64 slm[];
    const u32 s = blockIdx.y;
    const SegSP S = segs[s];
    const u32* act = S.actp ? S.actp : active + S.abase;
    if (lds_active) {
        for (u32 a = threadIdx.x; a < S.nactive; a += MB_THREADS) slm[a] = S.lm[act[a]];
        __syncthreads();
    }
    // lane-parallel divisibility (valid while every exponent is below 2^(w-1))
    const u32 n = S.n, w = S.w, lane = lane_id();
    u64 H = 0;
    for (u32 i = 0; i < n; ++i) H |= 1ull << (w * i + w - 1);
    const u64 lanes = (n * w >= 64) ? ~0ull : ((1ull << (n * w)) - 1);
    // one wave per frontier monomial, lanes over the active list (descending
    // index): the first divisor in list order is the reducer (largest index).
    // A wave keeps up to RED_BUF of its rows in LDS and appends them with one
    // atomic on the row counter (the rows' order in the list is immaterial:
    // the matrix orders its rows itself)
    __shared__ u64 s_bt[MB_WAVES][RED_BUF];
    __shared__ u32 s_bk[MB_WAVES][RED_BUF], s_bq[MB_WAVES][RED_BUF];
    const u32 wv = threadIdx.x / F4_WAVE;
    u32 nbuf = 0;  // rows buffered by this wave (the same in every lane)
    auto flush = [&]() {
        __builtin_amdgcn_wave_barrier();  // lane 0's buffer writes before the lanes' reads
        u32 base = 0;
        if (lane == 0) base = atomicAdd(&ctr[CTR * s + 1], nbuf);
        base = (u32)__shfl((int)base, 0);
        if (lane < nbuf) {
            const u32 slot = base + lane;
            if (slot >= S.rcap) {
                ctr[CTR * s + 3] = 2u;
            } else {
                rows_t[S.rbase + slot] = s_bt[wv][lane];
                rows_k[S.rbase + slot] = s_bk[wv][lane];
                row_lmrank[S.rbase + slot] = s_bq[wv][lane];
            }
        }
        nbuf = 0;
    };
    const u32 f0 = fscan[S.wbase], f1 = fscan[S.wbase + S.nwords];
    const u32 nwaves = gridDim.x * MB_WAVES;
    for (u32 i = f0 + blockIdx.x * MB_WAVES + wv; i < f1; i += nwaves) {
        const u32 q = list_q[i];
        const u64 m = S.montab[q];
        const bool mclean = (m & H) == 0;
        u32 found = 0xffffffffu;
        for (u32 a0 = 0; a0 < S.nactive; a0 += F4_WAVE) {
            const u32 a = a0 + lane;
            bool d = false;
            if (a < S.nactive) {
                const u64 l = lds_active ? slm[a] : S.lm[act[a]];
                d = (mclean && !(l & H)) ? (((((m & lanes) | H) - (l & lanes)) & H) == H) : mono_divides(l, m, n, w);
            }
            u64 hit = wave_ballot(d);
            while (hit) {  // candidates in list order (descending index)
                const u32 a = a0 + __ffsll((long long)hit) - 1;
                if (!S.sig) {
                    found = a;
                    break;
                }
                const u64 l = lds_active ? slm[a] : S.lm[act[a]];
                const u32 adm = sig_adm_wave(*S.sig, m - l, act[a]);
                if (adm == SIG_OK) {
                    found = a;
                    break;
                }
                if (adm == SIG_OVERFLOW && lane == 0) ctr[CTR * s + 3] = 4u;
                hit &= hit - 1;
            }
            if (found != 0xffffffffu) break;
        }
        if (found != 0xffffffffu) {  // the same in every lane (ballot results)
            if (lane == 0) {
                const u64 l = lds_active ? slm[found] : S.lm[act[found]];
                s_bt[wv][nbuf] = m - l;
                s_bk[wv][nbuf] = act[found];
                s_bq[wv][nbuf] = q;
            }
            if (++nbuf == RED_BUF) flush();
        }
    }
    if (nbuf) flush();
}

__global__ void k_word_popc(const u32* present, u32 nwords, u32* cnt) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x)
        cnt[i] = __popc(present[i]);
}

// Dictionary: column of rank q = number of seen ranks below q in the system;
// the columns are the seen monomials in descending grevlex order.
__global__ void k_dict(const SegSP* segs, const u32* present, const u32* off, u32* colmap, u64* dict_keys) {
    const SegSP S = segs[blockIdx.y];
    const u32 base0 = off[S.wbase];
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < S.nwords; i += gridDim.x * blockDim.x) {
        u32 f = present[S.wbase + i];
        u32 pos = off[S.wbase + i] - base0;
        while (f) {
            const u32 b = __ffs(f) - 1;
            const u32 q = i * 32 + b;
            colmap[S.cmbase + q] = pos;
            dict_keys[S.cmbase + pos] = S.montab[q];
            ++pos;
            f &= f - 1;
        }
    }
}

// per-system M = sum of row lengths (first pass of the two-pass plan)
__global__ void k_sum_len(const SegSP* segs, const u32* rows_k, const u32* ctr, unsigned long long* M) {
    const u32 s = blockIdx.y;
    const SegSP S = segs[s];
    const u32 r = ctr[CTR * s + 1];
    u32 acc = 0;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x)
        acc += S.len[rows_k[S.rbase + i]];
    for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, F4_WAVE);
    if (lane_id() == 0 && acc) atomicAdd(&M[s], (unsigned long long)acc);
}

// summary per system: rows, remaining frontier, error, N, M lo, M hi
__global__ void k_sp_summary(const SegSP* segs, u32 S, const u32* ctr, const u32* fscan, const u32* pscan,
                             const u32* lscan, const unsigned long long* M, u32* out) {
    for (u32 s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        const SegSP& G = segs[s];
        out[8 * s + 0] = ctr[CTR * s + 1];
        out[8 * s + 1] = fscan[G.wbase + G.nwords] - fscan[G.wbase];
        out[8 * s + 2] = ctr[CTR * s + 3];
        out[8 * s + 3] = pscan[G.wbase + G.nwords] - pscan[G.wbase];
        out[8 * s + 4] = (u32)M[s];
        out[8 * s + 5] = (u32)(M[s] >> 32);
        out[8 * s + 6] = lscan[G.wbase + G.nwords] - lscan[G.wbase];  // distinct leading monomials
    }
}

// End of the closure of a small batch in one workgroup: the frontier scan
// (convergence; empty without closure), the seen and leading-monomial scans
// (dictionary offsets, pivot counts), M per system and the summary -
// k_words_small modes 1 and 2, k_sum_len and k_sp_summary in one launch.
#define SUMMARY_SMALL_S 256
#define SUMMARY_SMALL_ROWS 65536
__global__ __launch_bounds__(1024) void k_summary_small(const SegSP* segs, u32 S, const u32* present,
                                                        const u32* done, const u32* lead, u32 W, int closure,
                                                        const u32* rows_k, const u32* ctr, u32* fcnt, u32* pcnt,
                                                        u32* lcnt, u32* out) {
    __shared__ u32 s_wave[33];
    __shared__ unsigned long long s_M[SUMMARY_SMALL_S];
    const u32 tid = threadIdx.x;
    for (u32 sy = tid; sy < S; sy += 1024) s_M[sy] = 0;
    u32 cf = 0, cp = 0, cl = 0;
    for (u32 base = 0; base < W; base += 1024) {
        const u32 wi = base + tid;
        const u32 pw = wi < W ? present[wi] : 0u;
        const u32 f = (wi < W && closure) ? (pw & ~done[wi]) : 0u;
        const u32 l = wi < W ? lead[wi] : 0u;
        u32 tf, tp, tl;
        const u32 pf = block_exclusive_scan(__popc(f), s_wave, &tf);
        const u32 pp = block_exclusive_scan(__popc(pw), s_wave, &tp);
        const u32 pl = block_exclusive_scan(__popc(l), s_wave, &tl);
        if (wi < W) {
            fcnt[wi] = cf + pf;
            pcnt[wi] = cp + pp;
            lcnt[wi] = cl + pl;
        }
        cf += tf;
        cp += tp;
        cl += tl;
    }
    if (tid == 0) {
        fcnt[W] = cf;
        pcnt[W] = cp;
        lcnt[W] = cl;
    }
    __syncthreads();
    // M = sum of the row lengths of each system
    for (u32 sy = 0; sy < S; ++sy) {
        const SegSP& G = segs[sy];
        const u32 r = ctr[CTR * sy + 1];
        u32 acc = 0;
        for (u32 i = tid; i < r; i += 1024) acc += G.len[rows_k[G.rbase + i]];
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, F4_WAVE);
        if (lane_id() == 0 && acc) atomicAdd(&s_M[sy], (unsigned long long)acc);
    }
    __syncthreads();
    for (u32 sy = tid; sy < S; sy += 1024) {
        const SegSP& G = segs[sy];
        const unsigned long long M = s_M[sy];
        out[8 * sy + 0] = ctr[CTR * sy + 1];
        out[8 * sy + 1] = fcnt[G.wbase + G.nwords] - fcnt[G.wbase];
        out[8 * sy + 2] = ctr[CTR * sy + 3];
        out[8 * sy + 3] = pcnt[G.wbase + G.nwords] - pcnt[G.wbase];
        out[8 * sy + 4] = (u32)M;
        out[8 * sy + 5] = (u32)(M >> 32);
        out[8 * sy + 6] = lcnt[G.wbase + G.nwords] - lcnt[G.wbase];
    }
}

// Row order of a small batch (at most SORT_SMALL_MAX rows) in one workgroup:
// the keys of k_row_keys sorted in LDS, then k_gather_rows and the scan of
// the row lengths (row_ptr) - four launches in one.
__global__ __launch_bounds__(1024) void k_rows_small(const SegSP* segs, u32 S, const u32* row_lmrank,
                                                     const u64* rows_t, const u32* rows_k, u32 R, u32 sshift,
                                                     u32 kbits, u32 hi_bit, u32 digit, u64* out_t, u32* out_k,
                                                     u32* row_ptr, u32* row_sys) {
    extern __shared__ u64 rs_mem[];
    u64* ka = rs_mem;
    u64* kb = ka + SORT_SMALL_MAX;
    u32* va = (u32*)(kb + SORT_SMALL_MAX);
    u32* vb = va + SORT_SMALL_MAX;
    __shared__ u32 run[256];
    __shared__ u32 wcnt[16 * 256];
    __shared__ u32 s_wave[33];
    const u32 tid = threadIdx.x;
    for (u32 sy = 0; sy < S; ++sy) {
        const SegSP& G = segs[sy];
        for (u32 i = tid; i < G.r; i += 1024) {
            const u32 src = G.rbase + i;
            ka[G.obase + i] = ((u64)sy << sshift) | ((u64)row_lmrank[src] << kbits) | rows_k[src];
            va[G.obase + i] = src;
        }
    }
    const bool sw = lds_radix_sort(ka, kb, va, vb, R, 0, hi_bit, digit, 1024, run, wcnt, s_wave);
    const u64* rk = sw ? kb : ka;
    const u32* rv = sw ? vb : va;
    __syncthreads();
    u32 carry = 0;
    for (u32 base = 0; base < R; base += 1024) {
        const u32 i = base + tid;
        u32 len = 0;
        if (i < R) {
            const u32 src = rv[i];
            const u32 sy = S > 1 ? (u32)(rk[i] >> sshift) : 0u;
            const u32 k = rows_k[src];
            out_t[i] = rows_t[src];
            out_k[i] = k;
            len = segs[sy].len[k];
            row_sys[i] = sy;
        }
        u32 tot;
        const u32 pre = block_exclusive_scan(len, s_wave, &tot);
        if (i < R) row_ptr[i] = carry + pre;
        carry += tot;
    }
    if (tid == 0) row_ptr[R] = carry;
}

// Row order: system, then leading monomial descending (= rank ascending), then
// basis index.
__global__ void k_row_keys(const SegSP* segs, const u32* row_lmrank, const u32* rows_k, u32 sshift, u32 kbits,
                           u64* keys, u32* vals) {
    const u32 s = blockIdx.y;
    const SegSP S = segs[s];
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < S.r; i += gridDim.x * blockDim.x) {
        const u32 src = S.rbase + i;
        keys[S.obase + i] = ((u64)s << sshift) | ((u64)row_lmrank[src] << kbits) | rows_k[src];
        vals[S.obase + i] = src;
    }
}

__global__ void k_gather_rows(const SegSP* segs, const u32* perm, const u64* keys, u32 sshift, const u64* rows_t,
                              const u32* rows_k, u32 R, u64* out_t, u32* out_k, u32* out_len, u32* row_sys) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < R; i += gridDim.x * blockDim.x) {
        const u32 src = perm[i];
        const u32 s = sshift >= 64 ? 0u : (u32)(keys[i] >> sshift);
        const u32 k = rows_k[src];
        out_t[i] = rows_t[src];
        out_k[i] = k;
        out_len[i] = segs[s].len[k];
        row_sys[i] = s;
    }
}

// Pass 2 of the two-pass plan fused with the dictionary join (dense rank):
// row i writes col_ind/val into its own segment [row_ptr[i], row_ptr[i+1]).
__global__ __launch_bounds__(MB_THREADS) void k_fill_rank(const SegSP* segs, const u64* row_t, const u32* row_k,
                                                           const u32* row_ptr, const u32* colmap, u32* col_ind,
                                                           u32* val) {
    extern __shared__ u32 sm[];
    const SegSP S = segs[blockIdx.y];
    for (u32 i = threadIdx.x; i < S.tabn; i += MB_THREADS) sm[i] = S.binom[i];
    __syncthreads();
    const u32 n = S.n, w = S.w, D = S.D, lane = lane_id();
    const u32 nw_total = gridDim.x * MB_WAVES;
    const u32* cm = colmap + S.cmbase;
    for (u32 ri = blockIdx.x * MB_WAVES + threadIdx.x / F4_WAVE; ri < S.r; ri += nw_total) {
        const u32 row = S.obase + ri;
        const u64 t = row_t[row];
        const u32 k = row_k[row];
        const u64 off = S.off[k];
        const u32 len = S.len[k];
        const u32 s0 = row_ptr[row];
        for (u32 j = lane; j < len; j += F4_WAVE) {
            const u32 q = mono_rank(t + S.mon[off + j], n, w, D, sm);
            col_ind[s0 + j] = q < S.nmax ? cm[q] : 0u;
            val[s0 + j] = S.coeff[off + j];
        }
    }
}

// ------------------------------------------------------- radix-sort path
// Compact order key of a monomial of degree <= D: (D - deg) on top, then the
// exponents a_n .. a_1 in fields of b = bitlength(D) bits.  Ascending keys are
// descending grevlex, and the key is injective on Mon_{<=D}.  The system index
// sits above the key so one sort serves the whole batch.
__device__ __forceinline__ u32 bitlen_d(u32 x) { return 32 - __clz(x); }
__device__ __forceinline__ u64 compact_key(u64 P, u32 n, u32 w, u32 b, u32 D) {
    u64 k = (u64)(D - mono_deg(P)) << (n * b);
    for (u32 i = 0; i < n; ++i) k |= (u64)mono_exp(P, i, w) << (b * i);
    return k;
}
__device__ __forceinline__ u64 compact_to_P(u64 k, u32 n, u32 w, u32 b) {
    u64 P = 0;
    u32 deg = 0;
    for (u32 i = 0; i < n; ++i) {
        const u32 a = (u32)((k >> (b * i)) & ((1u << b) - 1));
        P |= (u64)a << (w * i);
        deg += a;
    }
    return P | ((u64)deg << 56);
}

// Pass 2 of the two-pass plan as written: materialise row_key / row_val
__global__ __launch_bounds__(MB_THREADS) void k_fill_keys(const SegSP* segs, const u64* row_t, const u32* row_k,
                                                           const u32* row_ptr, u32 kshift, u64* row_key,
                                                           u32* row_val) {
    const u32 s = blockIdx.y;
    const SegSP S = segs[s];
    const u32 n = S.n, w = S.w, D = S.D, b = bitlen_d(S.D ? S.D : 1), lane = lane_id();
    const u64 sk = kshift >= 64 ? 0ull : ((u64)s << kshift);
    const u32 nw_total = gridDim.x * MB_WAVES;
    for (u32 ri = blockIdx.x * MB_WAVES + threadIdx.x / F4_WAVE; ri < S.r; ri += nw_total) {
        const u32 row = S.obase + ri;
        const u64 t = row_t[row];
        const u32 k = row_k[row];
        const u64 off = S.off[k];
        const u32 len = S.len[k];
        const u32 s0 = row_ptr[row];
        for (u32 j = lane; j < len; j += F4_WAVE) {
            row_key[s0 + j] = sk | compact_key(t + S.mon[off + j], n, w, b, D);
            row_val[s0 + j] = S.coeff[off + j];
        }
    }
}

// first position of each system's keys in the sorted unique key list
__global__ void k_seg_bounds(const u64* dict, const u32* N_ptr, u32 S, u32 kshift, u32* dstart) {
    const u32 N = *N_ptr;
    for (u32 s = blockIdx.x * blockDim.x + threadIdx.x; s <= S; s += gridDim.x * blockDim.x) {
        u32 lo = 0, hi = N;
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            const u32 ks = kshift >= 64 ? 0u : (u32)(dict[mid] >> kshift);
            if (ks < s)
                lo = mid + 1;
            else
                hi = mid;
        }
        dstart[s] = lo;
    }
}

// Join: position of every row key in its system's part of the sorted
// dictionary (binary search; in LDS when the batch has one system and fits).
// Every key is in the dictionary by construction; the system index and the
// position are still clamped into range so that no later kernel can index
// outside its arrays.
__global__ __launch_bounds__(MB_THREADS) void k_join(const u64* row_key, u64 M, const u64* dict, const u32* dstart,
                                                      u32 kshift, u32 S, int lds_dict, u32 Ncap, u32* col_ind) {
    extern __shared__ u64 sd[];
    if (lds_dict) {
        const u32 N = min(dstart[1] - dstart[0], Ncap);
        for (u32 i = threadIdx.x; i < N; i += MB_THREADS) sd[i] = dict[dstart[0] + i];
        __syncthreads();
    }
    for (u64 e = (u64)blockIdx.x * MB_THREADS + threadIdx.x; e < M; e += (u64)gridDim.x * MB_THREADS) {
        const u64 key = row_key[e];
        const u32 s = kshift >= 64 ? 0u : min((u32)(key >> kshift), S - 1);
        const u32 a = dstart[s], bnd = max(dstart[s + 1], a);
        const u64* Dd = lds_dict ? sd : dict + a;
        const u32 n = lds_dict ? min(bnd - a, Ncap) : bnd - a;
        u32 lo = 0, hi = n;
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (Dd[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        col_ind[e] = lo < n ? lo : (n ? n - 1 : 0);
    }
}

__global__ void k_dict_from_compact(const SegSP* segs, const u64* dictc, const u32* N_ptr, const u32* dstart,
                                    u32 kshift, u32 S, u64* dict_keys) {
    const u32 N = *N_ptr;
    const u64 kmask = kshift >= 64 ? ~0ull : ((1ull << kshift) - 1);
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const u32 s = kshift >= 64 ? 0u : (u32)(dictc[i] >> kshift);
        if (s >= S) continue;
        const SegSP& G = segs[s];
        const u32 col = i - dstart[s];
        if (col < G.nmax) dict_keys[G.cmbase + col] = compact_to_P(dictc[i] & kmask, G.n, G.w, bitlen_d(G.D ? G.D : 1));
    }
}

static u32 bitlen(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

static u32 grid_for(u64 items, u32 per_block, u32 cap) {
    u64 g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (u32)g;
}

// --------------------------------------------------------------- driver
void build_batch(Ctx& c, const std::vector<BuildArgs>& args, Matrix& out) {
    hipStream_t s = c.stream;
    const u32 S = (u32)args.size();
    if (S == 0) throw F4Error{1, "empty batch"};
    if (S > 65535) throw F4Error{2, "batch has more than 65535 systems"};
    hipEvent_t ev0 = stage_event(c);

    // ---- per-system layout (host)
    std::vector<SegSP> segs(S);
    std::vector<u32> actv;
    u64 W = 0, RC = 0, CM = 0, IB = 0, AB = 0;
    const bool dev_rows = args[0].rows_t_dev != nullptr;
    for (u32 i = 0; i < S; ++i) {
        // device rows and active lists: one buffer for the batch
        if (args[i].rows_t_dev != args[0].rows_t_dev || args[i].rows_k_dev != args[0].rows_k_dev ||
            (dev_rows && !args[i].rows_k_dev))
            throw F4Error{1, "device row lists are shared by the whole batch"};
        if (args[i].r0_dev && !dev_rows) throw F4Error{1, "a device row count without device rows"};
    }
    u32 max_tabn = 0, max_words = 0, max_nmax = 0, max_np = 1;
    for (u32 i = 0; i < S; ++i) {
        const BuildArgs& a = args[i];
        if (a.r0 == 0) throw F4Error{1, "empty row list"};
        const u32 n = a.G.n, D = a.D;
        const u64 nmax64 = binom_host(n + D, n);
        if (nmax64 > (1ull << 27)) throw F4Error{2, "N(n, D) too large for the dense-rank closure"};
        SegSP& g = segs[i];
        std::memset(&g, 0, sizeof(g));
        g.mon = a.G.mon;
        g.coeff = a.G.coeff;
        g.off = a.G.off;
        g.lm = a.G.lm;
        g.len = a.G.len;
        g.binom = rank_table(c, n, D);
        g.montab = unrank_table(c, n, D);
        g.n = n;
        g.w = a.G.w;
        g.D = D;
        g.nmax = (u32)nmax64;
        g.nwords = ceil_div(g.nmax, 32);
        g.wbase = (u32)W;
        g.rcap = a.r0 + (a.closure ? g.nmax : 0);
        g.rbase = (u32)RC;
        g.abase = (u32)AB;
        g.nactive = a.nactive;
        g.actp = a.active_dev;
        if (!a.active_dev) {
            AB += a.nactive;
            for (u32 k = 0; k < a.nactive; ++k) actv.push_back(a.active_host[k]);
        }
        g.tabn = (n + D + 2) * F4_BSTRIDE;
        g.npolys = a.G.npolys;
        g.cmbase = (u32)CM;
        g.ibase = (u32)IB;
        g.r0 = a.r0;
        g.r0p = a.r0_dev;
        g.sig = a.sig_dev;
        IB += a.r0;
        W += g.nwords;
        RC += g.rcap;
        CM += g.nmax;
        max_tabn = std::max(max_tabn, g.tabn);
        max_words = std::max(max_words, g.nwords);
        max_nmax = std::max(max_nmax, g.nmax);
        max_np = std::max(max_np, g.npolys);
    }
    if (W >= (1ull << 31) || RC >= (1ull << 31) || CM >= (1ull << 31)) throw F4Error{2, "batch too large"};
    const bool closure = args[0].closure;

    // descriptors, active lists, initial rows and counters: one upload
    if (AB >= (1ull << 31)) throw F4Error{2, "batch too large"};
    const u64 I = dev_rows ? 0 : IB;
    std::vector<u8> pack;
    auto put = [&](const void* src, size_t bytes) {
        const size_t off = (pack.size() + 255) & ~(size_t)255;
        pack.resize(off + std::max<size_t>(bytes, 1));
        if (bytes) std::memcpy(pack.data() + off, src, bytes);
        return off;
    };
    std::vector<u32> hc(CTR * S, 0);
    for (u32 i = 0; i < S; ++i) hc[CTR * i + 1] = args[i].r0;
    const size_t o_segs = put(segs.data(), S * sizeof(SegSP));
    const size_t o_act = put(actv.data(), actv.size() * 4);
    const size_t o_ctr = put(hc.data(), hc.size() * 4);
    const size_t o_t0 = put(nullptr, I * 8), o_k0 = put(nullptr, I * 4);
    for (u32 i = 0; i < S && !dev_rows; ++i) {
        const BuildArgs& a = args[i];
        std::memcpy(pack.data() + o_t0 + (size_t)segs[i].ibase * 8, a.rows_t_host, (size_t)a.r0 * 8);
        std::memcpy(pack.data() + o_k0 + (size_t)segs[i].ibase * 4, a.rows_k_host, (size_t)a.r0 * 4);
    }
    DBuf<u8> params(&c.pool, pack.size());
    upload(c, params.ptr, pack.data(), pack.size());
    SegSP* const dsegs = (SegSP*)(params.ptr + o_segs);
    const u32* const active = (const u32*)(params.ptr + o_act);
    u32* const ctr = (u32*)(params.ptr + o_ctr);  // counters live in the parameter block
    // present, done and leading-monomial bitmaps (cleared by k_init_rows)
    DBuf<u32> pd(&c.pool, 3 * W);
    u32* const present = pd.ptr;
    u32* const done = pd.ptr + W;
    u32* const leadmap = pd.ptr + 2 * W;
    DBuf<u64> rows_t(&c.pool, RC);
    DBuf<u32> rows_k(&c.pool, RC), row_lmrank(&c.pool, RC);
    DBuf<unsigned long long> Mdev(&c.pool, S);
    {
        u32 mr = 1;
        for (u32 i = 0; i < S; ++i) mr = std::max(mr, std::max(args[i].r0, segs[i].nwords));
        const u64* t0 = dev_rows ? args[0].rows_t_dev : (const u64*)(params.ptr + o_t0);
        const u32* k0 = dev_rows ? args[0].rows_k_dev : (const u32*)(params.ptr + o_k0);
        hipLaunchKernelGGL(k_init_rows, dim3(std::min<u32>(dev_rows ? 4096 : 64, ceil_div(mr, 256)), S), dim3(256), 0,
                           s, dsegs, t0, k0, rows_t.ptr, rows_k.ptr, pd.ptr, (u32)W, Mdev.ptr, ctr);
        F4_LAUNCH_CHECK();
    }

    const int local_bitmap = (max_tabn + max_words) * 4 <= 48 * 1024;
    const size_t mark_lds = (max_tabn + (local_bitmap ? max_words : 0)) * 4;
    // two workgroups per CU over the batch: the later closure rounds add rows
    // whose count the host does not see, and a workgroup past its system's
    // rows exits before its setup; rows are latency-bound (dependent rank
    // lookups), so the waves in flight set the rate
    u32 bx = std::max<u32>(1, std::min<u32>((u32)std::max(1, c.dev.cus), ceil_div(2048, S)));
    bx = std::max<u32>(bx, std::max<u32>(1, 2u * (u32)std::max(1, c.dev.cus) / S));
    auto mark = [&]() {
        hipLaunchKernelGGL(k_mark_rows, dim3(bx, S), dim3(MK_THREADS), mark_lds, s, dsegs, rows_t.ptr,
                           rows_k.ptr, row_lmrank.ptr, ctr, present, done, leadmap, local_bitmap);
        F4_LAUNCH_CHECK();
    };
    mark();

    DBuf<u32> fcnt(&c.pool, W + 1), pcnt(&c.pool, W + 1), lcnt(&c.pool, W + 1);
    DBuf<u32> list_q(&c.pool, closure ? CM : 1), list_s(&c.pool, closure ? CM : 1);
    DBuf<u32> summary(&c.pool, 8 * S);
    const u32 wgrid = grid_for(W, 256, 2048);
    const u32 wbx = std::max<u32>(1, std::min<u32>(64, ceil_div(max_words, 256)));
    u32 max_act = 0;
    for (u32 i = 0; i < S; ++i) max_act = std::max(max_act, segs[i].nactive);
    const int lds_active = (size_t)max_act * 8 <= 64 * 1024;
    // reducer search: a wave per frontier monomial, about four per wave at the
    // largest frontier, at most 4096 workgroups over the batch
    const u32 rbx_red = std::max<u32>(1, std::min<u32>(std::max<u32>(4, 4096 / std::max<u32>(S, 1)),
                                                       ceil_div(max_nmax, MB_WAVES * 4)));
    u32 rounds = 0;
    std::vector<u32> hs(8 * S);
    const bool small_words = W <= WORDS_SMALL;
    const bool fused_summary = small_words && S <= SUMMARY_SMALL_S && RC <= SUMMARY_SMALL_ROWS;
    u32 spec = 2;  // speculative rounds per host check
    for (;;) {
        if (closure) {
            // two speculative rounds at the first host check (dense systems
            // converge in two), then twice as many after each check that
            // finds a frontier left (a round past convergence only relaunches
            // three kernels on an empty frontier)
            for (u32 k = 0; k < spec; ++k) {
                if (small_words) {
                    hipLaunchKernelGGL(k_words_small, dim3(1), dim3(1024), 0, s, dsegs, S, present, done, (u32)W, 0,
                                       fcnt.ptr, list_q.ptr, list_s.ptr, ctr, leadmap, lcnt.ptr);
                    F4_LAUNCH_CHECK();
                } else {
                    hipLaunchKernelGGL(k_frontier_count, dim3(wgrid), dim3(256), 0, s, present, done, (u32)W,
                                       fcnt.ptr);
                    F4_LAUNCH_CHECK();
                    exclusive_scan_u32(fcnt.ptr, fcnt.ptr, W, c.pool, s);
                    hipLaunchKernelGGL(k_frontier_write, dim3(wbx, S), dim3(256), 0, s, dsegs, present, done,
                                       fcnt.ptr, list_q.ptr, list_s.ptr, ctr);
                    F4_LAUNCH_CHECK();
                }
                hipLaunchKernelGGL(k_reducers, dim3(rbx_red, S), dim3(MB_THREADS), lds_active ? max_act * 8 : 0, s,
                                   dsegs, list_q.ptr, fcnt.ptr, active, lds_active, rows_t.ptr, rows_k.ptr,
                                   row_lmrank.ptr, ctr);
                F4_LAUNCH_CHECK();
                mark();
                ++rounds;
            }
        }
        // dictionary sizes, pivot counts and M alongside the convergence check:
        // one readback (small batches: one launch)
        if (fused_summary) {
            hipLaunchKernelGGL(k_summary_small, dim3(1), dim3(1024), 0, s, dsegs, S, present, done, leadmap, (u32)W,
                               closure ? 1 : 0, rows_k.ptr, ctr, fcnt.ptr, pcnt.ptr, lcnt.ptr, summary.ptr);
            F4_LAUNCH_CHECK();
        } else {
            if (!closure) {
                fill_u32(fcnt.ptr, W + 1, 0, s);
            } else if (small_words) {
                hipLaunchKernelGGL(k_words_small, dim3(1), dim3(1024), 0, s, dsegs, S, present, done, (u32)W, 1,
                                   fcnt.ptr, list_q.ptr, list_s.ptr, ctr, leadmap, lcnt.ptr);
                F4_LAUNCH_CHECK();
            } else {
                hipLaunchKernelGGL(k_frontier_count, dim3(wgrid), dim3(256), 0, s, present, done, (u32)W,
                                   fcnt.ptr);
                F4_LAUNCH_CHECK();
                exclusive_scan_u32(fcnt.ptr, fcnt.ptr, W, c.pool, s);
            }
            if (small_words) {
                hipLaunchKernelGGL(k_words_small, dim3(1), dim3(1024), 0, s, dsegs, S, present, done, (u32)W, 2,
                                   pcnt.ptr, list_q.ptr, list_s.ptr, ctr, leadmap, lcnt.ptr);
                F4_LAUNCH_CHECK();
            } else {
                hipLaunchKernelGGL(k_word_popc, dim3(wgrid), dim3(256), 0, s, present, (u32)W, pcnt.ptr);
                F4_LAUNCH_CHECK();
                exclusive_scan_u32(pcnt.ptr, pcnt.ptr, W, c.pool, s);
                hipLaunchKernelGGL(k_word_popc, dim3(wgrid), dim3(256), 0, s, leadmap, (u32)W, lcnt.ptr);
                F4_LAUNCH_CHECK();
                exclusive_scan_u32(lcnt.ptr, lcnt.ptr, W, c.pool, s);
            }
            fill_u64((u64*)Mdev.ptr, S, 0, s);
            hipLaunchKernelGGL(k_sum_len, dim3(bx, S), dim3(256), 0, s, dsegs, rows_k.ptr, ctr, Mdev.ptr);
            F4_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_sp_summary, dim3(grid_for(S, 256, 64)), dim3(256), 0, s, dsegs, S, ctr, fcnt.ptr,
                               pcnt.ptr, lcnt.ptr, Mdev.ptr, summary.ptr);
            F4_LAUNCH_CHECK();
        }
        readback(c, hs.data(), summary.ptr, hs.size() * 4);
        bool more = false;
        for (u32 i = 0; i < S; ++i) {
            if (hs[8 * i + 2] == 4) throw F4Error{2, "a reducer's signature overflows an exponent lane"};
            if (hs[8 * i + 2])
                throw F4Error{1, hs[8 * i + 2] == 1 ? "a row term is not a monomial of degree <= D (unsorted or "
                                                      "inconsistent input terms)"
                                                    : "row capacity exceeded"};
            if (hs[8 * i + 1]) more = true;
        }
        if (!closure || !more) break;
        if (rounds > 4 * (max_nmax + 8)) throw F4Error{5, "closure did not converge"};
        spec = std::min<u32>(2 * spec, 8);
    }

    // ---- sizes and output layout
    out.S = S;
    out.sys.assign(S, SysPart());
    u64 R = 0, Mtot = 0;
    for (u32 i = 0; i < S; ++i) {
        SysPart& P = out.sys[i];
        P.n = segs[i].n;
        P.deg = segs[i].D;
        P.r = hs[8 * i + 0];
        P.N = hs[8 * i + 3];
        P.nnz = (u64)hs[8 * i + 4] | ((u64)hs[8 * i + 5] << 32);
        P.npiv = hs[8 * i + 6];
        P.row_base = (u32)R;
        P.nnz_base = Mtot;
        P.dict_base = segs[i].cmbase;
        segs[i].obase = (u32)R;
        segs[i].r = P.r;
        if (P.N >= (1u << 26)) throw F4Error{2, "dictionary has 2^26 or more columns"};
        R += P.r;
        Mtot += P.nnz;
    }
    if (Mtot >= (1ull << 32) || R >= (1ull << 31)) throw F4Error{2, "batch matrix has 2^32 or more entries"};
    upload(c, dsegs, segs.data(), S * sizeof(SegSP));
    hipEvent_t ev1 = stage_event(c);

    // dictionary (dense rank): popcount prefix of the seen bitmap
    DBuf<u32> colmap(&c.pool, CM);
    out.dict_keys.reset(&c.pool, CM);
    hipLaunchKernelGGL(k_dict, dim3(wbx, S), dim3(256), 0, s, dsegs, present, pcnt.ptr, colmap.ptr,
                       out.dict_keys.ptr);
    F4_LAUNCH_CHECK();

    // row order: sort by (system, rank of LM, basis index)
    const u32 kbits = std::max<u32>(1, bitlen(max_np - 1));
    const u32 rbits = std::max<u32>(1, bitlen(max_nmax - 1));
    const u32 sshift = rbits + kbits;
    const u32 sbits = S > 1 ? bitlen(S - 1) : 0;
    if (sshift + sbits > 64) throw F4Error{2, "row key does not fit 64 bits"};
    out.row_t.reset(&c.pool, R);
    out.row_k.reset(&c.pool, R);
    out.row_sys.reset(&c.pool, R);
    out.row_ptr.reset(&c.pool, R + 1);
    if (R <= SORT_SMALL_MAX) {
        const size_t lds = (size_t)SORT_SMALL_MAX * (2 * sizeof(u64) + 2 * sizeof(u32));
        const u32 digit = c.tune.force_digit ? c.tune.force_digit : 8u;
        hipLaunchKernelGGL(k_rows_small, dim3(1), dim3(1024), lds, s, dsegs, S, row_lmrank.ptr, rows_t.ptr,
                           rows_k.ptr, (u32)R, sshift, kbits, sshift + sbits, digit, out.row_t.ptr,
                           out.row_k.ptr, out.row_ptr.ptr, out.row_sys.ptr);
        F4_LAUNCH_CHECK();
    } else {
        DBuf<u64> keys(&c.pool, R);
        DBuf<u32> perm(&c.pool, R);
        const u32 rbx = std::max<u32>(1, std::min<u32>(64, ceil_div(ceil_div(R, S), 256)));
        hipLaunchKernelGGL(k_row_keys, dim3(rbx, S), dim3(256), 0, s, dsegs, row_lmrank.ptr, rows_k.ptr, sshift, kbits,
                           keys.ptr, perm.ptr);
        F4_LAUNCH_CHECK();
        tuned_sort(c, keys.ptr, perm.ptr, R, 0, sshift + sbits);
        hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(R, 256, 4096)), dim3(256), 0, s, dsegs, perm.ptr, keys.ptr,
                           S > 1 ? sshift : 64u, rows_t.ptr, rows_k.ptr, (u32)R, out.row_t.ptr, out.row_k.ptr,
                           out.row_ptr.ptr, out.row_sys.ptr);
        F4_LAUNCH_CHECK();
        exclusive_scan_u32(out.row_ptr.ptr, out.row_ptr.ptr, R, c.pool, s);
    }

    out.col_ind.reset(&c.pool, std::max<u64>(Mtot, 1));
    out.val.reset(&c.pool, std::max<u64>(Mtot, 1));
    int path = args[0].dict_path;
    if (path < 0) path = (c.flags & 4u) ? 1 : 0;  // F4_OPT_DICT_RADIX
    const u32 fbx =
        std::max<u32>(1, std::min<u32>(8 * (u32)std::max(1, c.dev.cus), ceil_div(ceil_div(R, S), MB_WAVES)));
    if (path == 0) {
        hipLaunchKernelGGL(k_fill_rank, dim3(fbx, S), dim3(MB_THREADS), max_tabn * 4, s, dsegs, out.row_t.ptr,
                           out.row_k.ptr, out.row_ptr.ptr, colmap.ptr, out.col_ind.ptr, out.val.ptr);
        F4_LAUNCH_CHECK();
    } else {
        u32 kb = 0;
        for (u32 i = 0; i < S; ++i) kb = std::max(kb, (segs[i].n + 1) * std::max<u32>(1, bitlen(segs[i].D)));
        if (kb + sbits > 64) throw F4Error{2, "compact key does not fit 64 bits"};
        const u32 kshift = S > 1 ? kb : 64u;
        DBuf<u64> row_key(&c.pool, std::max<u64>(Mtot, 1)), cand(&c.pool, std::max<u64>(Mtot, 1)),
            dictc(&c.pool, std::max<u64>(Mtot, 1));
        hipLaunchKernelGGL(k_fill_keys, dim3(fbx, S), dim3(MB_THREADS), 0, s, dsegs, out.row_t.ptr, out.row_k.ptr,
                           out.row_ptr.ptr, kshift, row_key.ptr, out.val.ptr);
        F4_LAUNCH_CHECK();
        F4_HIP_TRY(hipMemcpyAsync(cand.ptr, row_key.ptr, Mtot * 8, hipMemcpyDeviceToDevice, s));
        tuned_sort(c, cand.ptr, nullptr, Mtot, 0, kb + sbits);
        DBuf<u32> ncount(&c.pool, 1), dstart(&c.pool, S + 1);
        unique_sorted_u64(cand.ptr, Mtot, dictc.ptr, ncount.ptr, c.pool, s);
        hipLaunchKernelGGL(k_seg_bounds, dim3(grid_for(S + 1, 256, 64)), dim3(256), 0, s, dictc.ptr, ncount.ptr, S,
                           kshift, dstart.ptr);
        F4_LAUNCH_CHECK();
        const u32 N0 = out.sys[0].N;
        const int lds_dict = S == 1 && (u64)N0 * 8 <= c.dev.max_lds;
        hipLaunchKernelGGL(k_join, dim3(grid_for(Mtot, MB_THREADS, 16 * (u32)std::max(1, c.dev.cus))),
                           dim3(MB_THREADS), lds_dict ? (size_t)N0 * 8 : 0, s, row_key.ptr, Mtot, dictc.ptr,
                           dstart.ptr, kshift, S, lds_dict, N0, out.col_ind.ptr);
        F4_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_dict_from_compact, dim3(grid_for(Mtot, 256, 2048)), dim3(256), 0, s, dsegs,
                           dictc.ptr, ncount.ptr, dstart.ptr, kshift, S, out.dict_keys.ptr);
        F4_LAUNCH_CHECK();
    }
    hipEvent_t ev2 = stage_event(c);

    out.R = (u32)R;
    out.nnz = Mtot;
    out.closure_rounds = rounds;
    out.dict_path = (u32)path;
    out.ev[0] = ev0;
    out.ev[1] = ev1;
    out.ev[2] = ev2;
}
