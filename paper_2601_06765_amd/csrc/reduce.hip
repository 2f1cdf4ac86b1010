// Elimination mod p of the Macaulay matrices of a batch of systems (section
// "PSGE: panel-structured Gaussian elimination", two panels: pivot columns /
// non-pivot columns).  One launch per kernel covers the whole batch; each
// system has its own prime.
//
//  1. Split.  Pivot columns are the leading columns of the rows; each pivot
//     column keeps one pivot row (fewest entries, then lowest index); every
//     other row is a lower row.  Columns are renumbered pivot columns first.
//  2. Sparse triangular solve.  Each lower row is reduced by the monic pivot
//     rows on all pivot columns, left to right, in a dense LDS accumulator.
//     Pivot columns are taken in panels of 64: inside a panel the multipliers
//     come from a dense 64x64 unit upper-triangular solve done in registers by
//     one wave; the panel's pivot rows beyond the panel are then applied by the
//     whole workgroup with LDS atomic adds (no ordering needed inside a panel).
//     The result is the trailing block D' = D - C A^-1 B, one dense row each.
//  3. Echelon of D'.  Blocked Gauss-Jordan: each round one workgroup per
//     system computes, in place, the reduced row echelon form of the 32
//     remaining rows with the smallest leading columns; their leading columns
//     are pivot columns of the whole block, their nonzero rows become new
//     pivot rows, and those columns are removed from every other row
//     (remaining rows and earlier pivot rows) by a multi-workgroup update.
//  4. Emit the pivot rows of D' as CSR over the original columns, sorted by
//     leading column: the reduced row echelon form of the trailing block.
// All arithmetic is exact mod p with Barrett reduction (equation "mod-fma").
#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "sort_lds.hpp"

#define PANEL 64
#define TR_THREADS 1024
#define TR_UNROLL 4
#define ECH_B 32

// per-system elimination descriptor
struct SegR {
    Fp f;
    u32 small;     // p < 2^16 and npiv < 2^16: u32 lazy accumulators
    u32 N, cb;     // columns, base in the concatenated column space
    u32 rb, r;     // rows in the batch matrix
    u32 npiv, pb;  // pivot columns, base in the concatenated pivot space
    u32 L, lb;     // rows to reduce, base in the row list
    u32 c, nb;     // trailing columns N - npiv, base in the concatenated non-pivot space
    u32 tb;        // first 64x64 diagonal panel
    u32 cap, capb; // pivot-row store capacity min(L, c), base (rows)
    u32 ub;        // first block of the system in the echelon update grid
    u64 dpb;       // D' base (u32 entries, row stride c)
    u64 prb;       // pivot-row store base (u32 entries, row stride c)
    u32 db;        // dictionary base of the system in the matrix's dict_keys
    u32 pk;        // p = 2^31 - pk with 1 <= pk < 2^8 (and npiv < 2^24), else 0
};

// Triangular-solve arithmetic class of a system: 0 p < 2^16 (u32 lazy
// accumulators), 1 p = 2^31 - k with small k (u64 accumulators of folded
// products), 2 any other p (u64 accumulators of Barrett-reduced products).
__host__ __device__ inline int trsm_class(const SegR& g) { return g.small ? 0 : (g.pk ? 1 : 2); }

// ------------------------------------------------------------------ split
__global__ void k_lead_best(const SegR* segs, const u32* row_ptr, const u32* col_ind, const u32* row_sys, u32 R,
                            unsigned long long* best) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < R; i += gridDim.x * blockDim.x) {
        const u32 len = row_ptr[i + 1] - row_ptr[i];
        if (len) atomicMin(&best[segs[row_sys[i]].cb + col_ind[row_ptr[i]]], ((unsigned long long)len << 32) | i);
    }
}

__global__ void k_pivflag(const unsigned long long* best, u32 C, u32* flag) {
    for (u32 c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x)
        flag[c] = best[c] != ~0ull ? 1u : 0u;
}

// perm: column -> renumbered column (pivots first, then the rest, each in
// column order); prow: pivot -> its pivot row (batch row index)
__global__ void k_perm(const SegR* segs, const unsigned long long* best, const u32* ppos, u32* perm, u32* prow,
                       u32* pivot_cols, u32* nonpiv) {
    const SegR S = segs[blockIdx.y];
    const u32 p0 = ppos[S.cb];
    const u32 npiv = ppos[S.cb + S.N] - p0;
    for (u32 c = blockIdx.x * blockDim.x + threadIdx.x; c < S.N; c += gridDim.x * blockDim.x) {
        const u32 g = S.cb + c;
        const u32 q = ppos[g] - p0;
        if (best[g] != ~0ull) {
            perm[g] = q;
            prow[p0 + q] = (u32)(best[g] & 0xffffffffu);
            pivot_cols[p0 + q] = c;
        } else {
            perm[g] = npiv + (c - q);
            nonpiv[(S.cb - p0) + (c - q)] = c;
        }
    }
}

__global__ void k_lower_flags(const SegR* segs, const u32* row_ptr, const u32* col_ind, const u32* row_sys, u32 R,
                              const unsigned long long* best, u32* flag) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < R; i += gridDim.x * blockDim.x) {
        const u32 len = row_ptr[i + 1] - row_ptr[i];
        flag[i] = (len == 0 || (u32)(best[segs[row_sys[i]].cb + col_ind[row_ptr[i]]] & 0xffffffffu) != i) ? 1u : 0u;
    }
}

__global__ void k_compact_idx(const u32* flag, const u32* pos, u32 n, u32* out) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (flag[i]) out[pos[i]] = i;
}

__global__ void k_split_summary(const SegR* segs, u32 S, const u32* ppos, const u32* lpos, u32* out) {
    for (u32 s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        const SegR& G = segs[s];
        out[2 * s] = ppos[G.cb + G.N] - ppos[G.cb];
        out[2 * s + 1] = lpos[G.rb + G.r] - lpos[G.rb];
    }
}

// The whole split of a small batch in one workgroup (C <= SPLIT_SMALL_C
// columns): best row per leading column in LDS, the pivot-column scan, the
// column renumbering, the lower-row compaction and the per-system counts, with
// the results of k_lead_best ... k_split_summary.
#define SPLIT_SMALL_C 8192
#define SPLIT_SMALL_R 65536
__global__ __launch_bounds__(1024) void k_split_small(const SegR* segs, u32 S, const u32* row_ptr,
                                                      const u32* col_ind, const u32* row_sys, u32 R, u32 C,
                                                      u32* ppos, u32* lpos, u32* perm, u32* prow, u32* pivot_cols,
                                                      u32* nonpiv, u32* lower, u32* summ) {
    extern __shared__ unsigned long long sbest[];
    __shared__ u32 s_wave[33];
    const u32 tid = threadIdx.x;
    for (u32 c = tid; c < C; c += 1024) sbest[c] = ~0ull;
    __syncthreads();
    for (u32 i = tid; i < R; i += 1024) {
        const u32 len = row_ptr[i + 1] - row_ptr[i];
        if (len) atomicMin(&sbest[segs[row_sys[i]].cb + col_ind[row_ptr[i]]], ((unsigned long long)len << 32) | i);
    }
    __syncthreads();
    u32 carry = 0;
    for (u32 base = 0; base < C; base += 1024) {
        const u32 c = base + tid;
        u32 tot;
        const u32 pre = block_exclusive_scan(c < C && sbest[c] != ~0ull ? 1u : 0u, s_wave, &tot);
        if (c < C) ppos[c] = carry + pre;
        carry += tot;
    }
    if (tid == 0) ppos[C] = carry;
    __syncthreads();
    for (u32 sy = 0; sy < S; ++sy) {
        const SegR G = segs[sy];
        const u32 p0 = ppos[G.cb];
        const u32 npiv = ppos[G.cb + G.N] - p0;
        for (u32 c = tid; c < G.N; c += 1024) {
            const u32 g = G.cb + c;
            const u32 q = ppos[g] - p0;
            if (sbest[g] != ~0ull) {
                perm[g] = q;
                prow[p0 + q] = (u32)(sbest[g] & 0xffffffffu);
                pivot_cols[p0 + q] = c;
            } else {
                perm[g] = npiv + (c - q);
                nonpiv[(G.cb - p0) + (c - q)] = c;
            }
        }
    }
    carry = 0;
    for (u32 base = 0; base < R; base += 1024) {
        const u32 i = base + tid;
        bool fl = false;
        if (i < R) {
            const u32 len = row_ptr[i + 1] - row_ptr[i];
            fl = len == 0 || (u32)(sbest[segs[row_sys[i]].cb + col_ind[row_ptr[i]]] & 0xffffffffu) != i;
        }
        u32 tot;
        const u32 pre = block_exclusive_scan(fl ? 1u : 0u, s_wave, &tot);
        if (i < R) lpos[i] = carry + pre;
        if (fl) lower[carry + pre] = i;
        carry += tot;
    }
    if (tid == 0) lpos[R] = carry;
    __syncthreads();
    for (u32 sy = tid; sy < S; sy += 1024) {
        const SegR& G = segs[sy];
        summ[2 * sy] = ppos[G.cb + G.N] - ppos[G.cb];
        summ[2 * sy + 1] = lpos[G.rb + G.r] - lpos[G.rb];
    }
}

// Trailing-entry count of each pivot row (entries beyond its own panel).
// (also clears the system's dense panels T, filled by k_upper_fill)
__global__ void k_upper_count(const SegR* segs, const u32* row_ptr, const u32* col_ind, const u32* prow,
                              const u32* perm, u32* tcnt, u32* T) {
    const SegR S = segs[blockIdx.y];
    const u32 lane = lane_id();
    {
        u32* Ts = T + (u64)S.tb * PANEL * PANEL;
        const u64 nT = (u64)((S.npiv + PANEL - 1) / PANEL) * PANEL * PANEL;
        for (u64 x = (u64)blockIdx.x * blockDim.x + threadIdx.x; x < nT; x += (u64)gridDim.x * blockDim.x) Ts[x] = 0;
    }
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 q = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; q < S.npiv; q += nw) {
        const u32 i = prow[S.pb + q];
        const u32 pend = min((q / PANEL + 1) * PANEL, S.npiv);
        u32 cnt = 0;
        for (u32 e = row_ptr[i] + lane; e < row_ptr[i + 1]; e += F4_WAVE) cnt += perm[S.cb + col_ind[e]] >= pend;
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, F4_WAVE);
        if (lane == 0) tcnt[S.pb + q] = cnt;
    }
}

// Monic pivot rows: the part inside the row's panel goes to the dense 64x64
// block T[panel] (unit diagonal), the rest to the packed trailing list
// entry = val << 32 | (row within panel) << 26 | renumbered column.
__global__ void k_upper_fill(const SegR* segs, const u32* row_ptr, const u32* col_ind, const u32* val,
                             const u32* prow, const u32* perm, const u32* tptr, u64* tent, u32* T) {
    const SegR S = segs[blockIdx.y];
    const u32 lane = lane_id();
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    const u64 lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (u32 q = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; q < S.npiv; q += nw) {
        const u32 i = prow[S.pb + q];
        const u32 kp = q / PANEL, b = q % PANEL;
        const u32 pend = min((kp + 1) * PANEL, S.npiv);
        const u32 inv = fp_inv(S.f, val[row_ptr[i]]);
        u32* Tk = T + (u64)(S.tb + kp) * PANEL * PANEL + (u64)b * PANEL;
        u32 base = tptr[S.pb + q];
        for (u32 e0 = row_ptr[i]; e0 < row_ptr[i + 1]; e0 += F4_WAVE) {
            const u32 e = e0 + lane;
            const bool ok = e < row_ptr[i + 1];
            u32 pc = 0, v = 0;
            if (ok) {
                pc = perm[S.cb + col_ind[e]];
                v = fp_mul(S.f, val[e], inv);
            }
            const bool trail = ok && pc >= pend;
            const u64 m = wave_ballot(trail);
            if (trail)
                tent[base + __popcll(m & lt)] = ((u64)v << 32) | ((u64)b << 26) | pc;
            else if (ok)
                Tk[pc % PANEL] = v;
            base += __popcll(m);
        }
    }
}

// Inverse of every panel's diagonal block (unit upper triangular, the pivot
// rows are monic): row b of T^-1 is the x with x T = e_b, found by forward
// substitution, one wave per row (lanes are columns).  A row's panel solve is
// then x = l T^-1: independent products instead of a 64-step chain.
__global__ __launch_bounds__(256) void k_tinv(const SegR* segs, const u32* T, u32* Tinv) {
    const SegR S = segs[blockIdx.y];
    const Fp f = S.f;
    const u32 np = (S.npiv + PANEL - 1) / PANEL;
    const u32 lane = lane_id();
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 w = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; w < np * PANEL; w += nw) {
        const u32 kp = w / PANEL, b = w % PANEL;
        const u32* Tk = T + (u64)(S.tb + kp) * PANEL * PANEL;
        u32 tc[PANEL];
#pragma unroll
        for (int k = 0; k < PANEL; ++k) tc[k] = Tk[k * PANEL + lane];
        u32 v = lane == b ? 1u : 0u;
        if (S.small) {
#pragma unroll
            for (int k = 0; k < PANEL; ++k) {
                const u32 xk = __builtin_amdgcn_readlane(v, k);
                if (xk != 0 && (u32)k < lane) v = fp_fma_t<true>(f, v, f.p - xk, tc[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < PANEL; ++k) {
                const u32 xk = __builtin_amdgcn_readlane(v, k);
                if (xk != 0 && (u32)k < lane) v = fp_fma_t<false>(f, v, f.p - xk, tc[k]);
            }
        }
        Tinv[(u64)(S.tb + kp) * PANEL * PANEL + (u64)b * PANEL + lane] = v;
    }
}

// ------------------------------------------------------ triangular solve
// One workgroup per tile of up to TR_MAXR consecutive rows of one system
// (grid: tiles x systems), one dense accumulator per row.  Each pivot panel
// is solved for every row of the tile at once (wave r solves row r), then the
// panel's trailing entries are read once and applied to all rows of the tile,
// so the upper block is streamed once per tile rather than once per row.
// Arithmetic classes (MODE): 0, p < 2^16 and npiv < 2^16: each product
// reduced by the one-word Barrett step into a u32 accumulator (a column
// receives at most npiv additions of values below p); 1, p = 2^31 - k with
// k < 2^8 (the large prime of the workloads and the CRT primes): the product
// t < 2^62 is only folded, t = h 2^31 + l == k h + l (mod p), a value below
// 2^39 + 2^31 added to a u64 accumulator (at most 2^24 additions fit, so this
// class needs npiv < 2^24), which costs a multiply-add instead of a full
// reduction; 2, any other p: Barrett-reduced products into u64.  Systems of
// another class return at once.
#define TR_MAXR 4  // the multipliers of a panel column are one uint4 in LDS
template <int MODE>
struct AccOf {
    typedef u64 T;
};
template <>
struct AccOf<0> {
    typedef u32 T;
};

template <int MODE, bool LDS, int RR>
__global__ __launch_bounds__(TR_THREADS) void k_trsm(const SegR* segs, u32 sys_base, const u32* row_ptr,
                                                     const u32* col_ind, const u32* val, const u32* list,
                                                     int tail, u32 rr, u32 tile_base, int skip_lead,
                                                     const u32* perm, const u32* Tinv, const u32* tptr,
                                                     const u64* tent, typename AccOf<MODE>::T* gacc, u32* Dp,
                                                     u32* lead_out, u32* status, unsigned long long* ops) {
    constexpr bool SMALL = MODE == 0;
    typedef typename AccOf<MODE>::T AccT;
    extern __shared__ unsigned char smraw[];
    __shared__ uint4 s_x[PANEL];  // per panel column b: the multipliers -x_b of the tile's rows (0 past nr)
    __shared__ u64 s_xs[2][TR_MAXR][PANEL];  // partial sums of x = l T^-1 (double buffered)
    __shared__ u64 s_hit[TR_MAXR];
    __shared__ u32 s_lead[TR_MAXR];
    __shared__ u32 s_first_pc;
    const SegR S = segs[sys_base + blockIdx.y];
    if (trsm_class(S) != MODE || S.c == 0) return;
    const u32 cnt = tail ? S.r : S.L;  // rows of this system in the list
    const u32 t0 = (tile_base + blockIdx.x) * rr;
    if (t0 >= cnt) return;
    const u32 nr = min(min(rr, (u32)RR), cnt - t0);
    const u32 tid = threadIdx.x, lane = lane_id(), wave = tid / F4_WAVE;
    const Fp f = S.f;
    const u32 N = S.N, npiv = S.npiv;
    AccT* acc = LDS ? (AccT*)smraw : gacc + ((u64)blockIdx.y * gridDim.x + blockIdx.x) * TR_MAXR * (u64)N;
    for (u32 j = tid; j < nr * N; j += TR_THREADS) acc[j] = 0;
    if (tid < TR_MAXR) s_lead[tid] = 0xffffffffu;
    if (tid < PANEL) s_x[tid] = make_uint4(0u, 0u, 0u, 0u);
    if (tid == 0) s_first_pc = 0xffffffffu;
    __syncthreads();
    const u32* pm = perm + S.cb;
    // the tile's first pivot column with a nonzero entry: the panels before
    // it hold zeros in every row of the tile and receive nothing (updates
    // only flow to later columns), so the solve starts at its panel
    u32 mnpc = 0xffffffffu;
    for (u32 r = 0; r < nr; ++r) {
        const u32 i = list[S.lb + t0 + r];
        for (u32 e = row_ptr[i] + (skip_lead ? 1 : 0) + tid; e < row_ptr[i + 1]; e += TR_THREADS) {
            const u32 pc = pm[col_ind[e]];
            acc[r * N + pc] = val[e];
            mnpc = min(mnpc, pc);
        }
    }
    for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) mnpc = min(mnpc, (u32)__shfl_xor((int)mnpc, (int)d, F4_WAVE));
    if (lane == 0) atomicMin(&s_first_pc, mnpc);
    __syncthreads();
    const u32 npanels = (npiv + PANEL - 1) / PANEL;
    const u32 kp0 = s_first_pc < npiv ? s_first_pc / PANEL : npanels;  // npanels: no pivot column set
    // Per panel: (A) every wave w forms, for each row of the tile, the partial
    // products of rows 4w..4w+3 of T^-1 with the row's panel values and adds
    // them into s_xs; (B) the tile's waves finish x = l T^-1; (C) every
    // thread applies its trailing entries.  The next panel's T^-1 slice and
    // trailing entries are loaded during the current one (neither depends on
    // the accumulators), so memory latency stays off the critical path.
    constexpr u32 BW = PANEL / (TR_THREADS / F4_WAVE);  // T^-1 rows per wave
    static_assert(BW * (TR_THREADS / F4_WAVE) == PANEL, "panel split");
    u32 tin[BW];
    u64 t[TR_UNROLL];
    u32 ea = 0, eb = 0;
    u32 nops = 0;  // modular products of this thread (reported with the timing option)
    auto load_panel = [&](u32 kq, u32* tin_, u64* t_, u32& ea_, u32& eb_) {
        const u32* Tk = Tinv + (u64)(S.tb + kq) * PANEL * PANEL;
#pragma unroll
        for (u32 i = 0; i < BW; ++i) tin_[i] = Tk[(wave * BW + i) * PANEL + lane];
        const u32 qa = kq * PANEL, qb = min(npiv, qa + PANEL);
        ea_ = tptr[S.pb + qa];
        eb_ = tptr[S.pb + qb];
#pragma unroll
        for (int k = 0; k < TR_UNROLL; ++k) {
            const u32 e = ea_ + tid + k * TR_THREADS;
            t_[k] = e < eb_ ? tent[e] : 0ull;
        }
    };
    if (tid < 2 * TR_MAXR * PANEL) (&s_xs[0][0][0])[tid] = 0;
    if (kp0 < npanels) load_panel(kp0, tin, t, ea, eb);
    __syncthreads();
    for (u32 kp = kp0; kp < npanels; ++kp) {
        const u32 qa = kp * PANEL, wk = min((u32)PANEL, npiv - qa), buf = kp & 1;
        // (A) partial products: lane j reduces the row's panel value l_j once
        // (contiguous LDS reads), and the wave takes its BW values from those
        // lanes with readlane
        for (u32 r = 0; r < nr; ++r) {
            const AccT aj = lane < wk ? acc[r * N + qa + lane] : (AccT)0;
            const u32 lj = SMALL ? fp_reduce32(f, (u32)aj) : fp_reduce_any(f, (u64)aj);
            // BW raw products: below BW p^2 < 2^64 (BW = 4, p < 2^31), one
            // reduction (or fold) for the sum instead of one per product
            static_assert(BW <= 4, "lazy panel sums");
            u64 part = 0;
#pragma unroll
            for (u32 i = 0; i < BW; ++i) {
                const u32 lb = (u32)__builtin_amdgcn_readlane((int)lj, (int)(wave * BW + i));  // 0 past wk
                part += SMALL ? (u64)mul24(lb, tin[i]) : (u64)lb * tin[i];
                nops += lb != 0;
            }
            if (MODE == 1)  // p = 2^31 - k: 2^31 == k, a value below 2^41 + 2^31
                part = (u64)S.pk * (part >> 31) + (part & 0x7fffffffull);
            else if (MODE == 2)
                part = fp_reduce_any(f, part);
            if (part) atomicAdd((unsigned long long*)&s_xs[buf][r][lane], (unsigned long long)part);
        }
        // the next panel's loads go out now
        u32 tin2[BW] = {};
        u64 t2[TR_UNROLL] = {};
        u32 ea2 = 0, eb2 = 0;
        if (kp + 1 < npanels) load_panel(kp + 1, tin2, t2, ea2, eb2);
        __syncthreads();
        // (B) x of every row; the panel's pivot columns of the accumulators are done
        if (wave < nr) {
            const u32 r = wave;
            const u32 x = fp_reduce_any(f, s_xs[buf][r][lane]);
            s_xs[buf][r][lane] = 0;
            reinterpret_cast<u32*>(&s_x[lane])[r] = x ? f.p - x : 0u;  // -x as a residue (0: nothing to apply)
            // with the timing option: the trailing-entry products this row
            // gets in (C), from the pivot rows' entry counts
            if (ops && x && lane < wk) nops += tptr[S.pb + qa + lane + 1] - tptr[S.pb + qa + lane];
            const u64 hit = wave_ballot(x != 0);
            if (lane == 0) s_hit[r] = hit;
            if (lane < wk) acc[r * N + qa + lane] = 0;
        }
        __syncthreads();
        u64 anyhit = 0;
        for (u32 r = 0; r < nr; ++r) anyhit |= s_hit[r];
        // (C) apply every trailing entry to every row of the tile; for
        // p = 2^31 - 1 the folded product h + l stays below 2^32 and needs
        // no multiply by k
        auto apply = [&](auto mersenne) {
            constexpr bool MERS = decltype(mersenne)::value;
            for (u32 e0 = ea + tid;; e0 += TR_THREADS * TR_UNROLL) {
                // the multipliers of all TR_UNROLL entries are read from LDS
                // before any product (no branch between the reads), then
                // each product is added where both factors are nonzero
                // (slots past the panel's entries hold 0; stored values are
                // nonzero)
                u32 xs[TR_UNROLL][RR];
#pragma unroll
                for (int k = 0; k < TR_UNROLL; ++k) {
                    const u32 b = (u32)(t[k] >> 26) & (PANEL - 1);
                    if (RR == 1) {
                        xs[k][0] = reinterpret_cast<const u32*>(&s_x[b])[0];
                    } else if (RR == 2) {
                        const uint2 v = reinterpret_cast<const uint2*>(&s_x[b])[0];
                        xs[k][0] = v.x;
                        xs[k][RR - 1] = v.y;
                    } else {
                        const uint4 v = s_x[b];
                        const u32 w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int r = 0; r < RR; ++r) xs[k][r] = w[r];
                    }
                }
#pragma unroll
                for (int k = 0; k < TR_UNROLL; ++k) {
                    const u32 col = (u32)t[k] & 0x3ffffffu, tv = (u32)(t[k] >> 32);
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const u32 negx = xs[k][r];
                        AccT add;
                        if (MODE == 0) {
                            add = fp_mul32(f, negx, tv);
                        } else if (MODE == 1) {
                            const u64 t = (u64)negx * tv;  // < 2^62
                            if (MERS)
                                add = (u64)((u32)(t >> 31) + ((u32)t & 0x7fffffffu));
                            else
                                add = (u64)S.pk * (u32)(t >> 31) + ((u32)t & 0x7fffffffu);
                        } else {
                            add = fp_reduce(f, (u64)negx * tv);
                        }
                        if (tv && negx) atomicAdd(&acc[r * N + col], add);
                    }
                }
                const u32 e1 = e0 + TR_THREADS * TR_UNROLL;
                if (e1 - tid >= eb) break;  // no thread has entries left
#pragma unroll
                for (int k = 0; k < TR_UNROLL; ++k) {
                    const u32 e = e1 + k * TR_THREADS;
                    t[k] = e < eb ? tent[e] : 0ull;
                }
            }
        };
        if (anyhit) {
            if (MODE == 1 && S.pk == 1)
                apply(std::true_type{});
            else
                apply(std::false_type{});
        }
#pragma unroll
        for (u32 i = 0; i < BW; ++i) tin[i] = tin2[i];
#pragma unroll
        for (int k = 0; k < TR_UNROLL; ++k) t[k] = t2[k];
        ea = ea2;
        eb = eb2;
        __syncthreads();
    }
    // trailing block rows: non-pivot part of the accumulators
    const u32 c = S.c;
    for (u32 r = 0; r < nr; ++r) {
        u32* out = Dp + S.dpb + (u64)(t0 + r) * c;
        u32 first = 0xffffffffu;
        for (u32 j = tid; j < c; j += TR_THREADS) {
            const AccT a = acc[r * N + npiv + j];
            const u32 v = SMALL ? fp_reduce32(f, (u32)a) : fp_reduce_any(f, (u64)a);
            out[j] = v;
            if (v && j < first) first = j;
        }
        if (first != 0xffffffffu) atomicMin(&s_lead[r], first);
    }
    __syncthreads();
    if (tid < nr && lead_out) lead_out[S.lb + t0 + tid] = s_lead[tid];
    if (tid < nr && status) status[S.lb + t0 + tid] = 0;  // echelon row status: live
    if (ops) {
        u64 v = nops;
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, F4_WAVE);
        if (lane == 0 && v) atomicAdd(ops, (unsigned long long)v);
    }
}

// ---------------------------------------------------------------- echelon
// Round header per system: done flag, q (new pivots this round), npr (pivot
// rows stored so far), npr0 (npr before this round), smallest new pivot
// column, and the new pivot columns in the order of the new pivot rows.
struct EchRound {
    u32 done, q, npr, npr0, cmin, b;
    u32 pm;  // block rows (bits) that became pivot rows
    u32 cols[ECH_B];
    u32 rows[ECH_B];
    u32 Z[ECH_B * ECH_B];  // row t: coefficients of new pivot row t on the block rows
};

// One round of the blocked echelon, one workgroup per system.  The block is
// the ECH_B remaining rows with the smallest (leading column, index).  The
// workgroup finds the block's pivot columns by Gauss-Jordan elimination
// recorded in a b x b transform Z: the block's columns are visited in chunks
// of ECH_CH, each chunk is loaded and multiplied by Z, and the rows of
// [chunk | Z] (LDS, ECH_CH + ECH_B = 64 columns, one per lane) are eliminated
// by ECH_PW waves owning ECH_RPW rows each.  The first column where a non-pivot row is
// nonzero becomes the next pivot; every such column is the leading column of a
// vector of the row space, hence a pivot column of the RREF of the whole
// trailing block.  Row operations are fraction-free (row_k <- piv * row_k -
// row_k[jp] * row_kp), so no inverse is taken per pivot; each pivot row's value
// at its pivot column is formed at the end and divided out.  Scanning stops
// once every block row is a pivot or the columns are exhausted (the other rows
// are then zero), so all block rows are consumed; the new pivot rows
// Z * (block rows), formed by k_ech_update, are reduced on all pivot columns
// of the round.
#define ECH_CH 32
#define ECH_W (ECH_CH + ECH_B)  // row width of [chunk | Z]: one lane per column
#define ECH_RS (ECH_W + 1)      // LDS row stride: a column of the rows spans all banks

template <bool SMALL>
__device__ __forceinline__ u32 fp_mul_t(const Fp& f, u32 a, u32 b) {
    return SMALL ? fp_mul32(f, a, b) : fp_reduce(f, (u64)a * b);  // SMALL: p < 2^16
}

// (piv * a - fk * b) mod p
template <bool SMALL>
__device__ __forceinline__ u32 fp_ff(const Fp& f, u32 piv, u32 a, u32 fk, u32 b) {
    const u32 x = fp_mul_t<SMALL>(f, piv, a), y = fp_mul_t<SMALL>(f, fk, b);
    return x >= y ? x - y : x + f.p - y;
}
// p < 2^16: (piv * a mod p) + (p - fk) * b < p + (p - 1) p = p^2 < 2^32, so
// two one-word Barrett reductions finish it in 32-bit integer arithmetic
template <>
__device__ __forceinline__ u32 fp_ff<true>(const Fp& f, u32 piv, u32 a, u32 fk, u32 b) {
    return fp_reduce32(f, fp_mul32(f, piv, a) + (f.p - fk) * b);
}

// a^-1 mod p by Fermat's little theorem with the modular product of the class
template <bool SMALL>
__device__ __forceinline__ u32 fp_inv_t(const Fp& f, u32 a) {
    u32 e = f.p - 2, r = 1, x = a;
    while (e) {
        if (e & 1) r = fp_mul_t<SMALL>(f, r, x);
        x = fp_mul_t<SMALL>(f, x, x);
        e >>= 1;
    }
    return r;
}

// Pivot loop: ECH_PW working waves (two per SIMD) own ECH_RPW block rows each
// and keep them in registers; the LDS copy of [chunk | Z] is written through
// on every update, so the pivot row is read from it by the other waves.  Per
// column every working wave publishes the lowest of its non-pivot rows that is
// nonzero there, which gives the next pivot column and pivot row together, in
// one exchange and one block barrier per pivot.  The other waves only follow
// the loop control.  (Measured on the n = 10 workload: 4 waves of 8 rows and
// 16 waves of 2 rows were both slower; one wave per SIMD leaves the latency
// of the pivot chain exposed, four per SIMD issue the loop control 4 times.)
#define ECH_PW 8
#define ECH_RPW (ECH_B / ECH_PW)
#define ECH_EMPTY 2       // chunks in a row without a pivot that end a block's scan early ...
#define ECH_EMPTY_LEFT 8  // ... while more than this many chunks are left

template <bool SMALL>
__global__ __launch_bounds__(1024) void k_ech_block(const SegR* segs, u32* lead, u32* status, const u32* Dp,
                                                    u32* cnt_g, int cnt_lds, EchRound* rounds, u32* prlead,
                                                    u32* ndone, unsigned long long* ops) {
    extern __shared__ u32 scnt[];
    __shared__ u32 s_wave[33];
    __shared__ u32 s_rows[ECH_B];
    __shared__ u32 s_RZ[ECH_B * ECH_RS];
    __shared__ u32 s_B[ECH_B * ECH_CH];
    __shared__ u32 s_pcol[ECH_B], s_prow[ECH_B], s_pv[ECH_B], s_inv[ECH_B];
    __shared__ uint4 s_first[2][F4_WAVE][ECH_PW / 4];  // [buffer][column]: per working wave, its lowest live row there
    __shared__ u32 s_thr, s_need, s_cmin;
    EchRound* R = rounds + blockIdx.y;
    if (R->done) return;
    const SegR S = segs[blockIdx.y];
    if ((S.small != 0) != SMALL) return;  // the other class has its own launch
    const Fp f = S.f;
    const u32 L = S.L, c = S.c;
    const u32 tid = threadIdx.x;
    u32* ld = lead + S.lb;
    u32* st = status + S.lb;
    const u32* D = Dp + S.dpb;
    u32* cnt = cnt_lds ? scnt : cnt_g + S.nb;
    for (u32 j = tid; j < c; j += 1024) cnt[j] = 0;
    if (tid == 0) {
        s_thr = c;
        s_need = 0;
        s_cmin = c;
    }
    __syncthreads();
    for (u32 i = tid; i < L; i += 1024)
        if (st[i] == 0 && ld[i] < c) atomicAdd(&cnt[ld[i]], 1u);
    __syncthreads();
    // threshold column: the first column where the cumulative count reaches ECH_B
    u32 carry = 0;
    for (u32 base = 0; base < c; base += 1024) {
        const u32 j = base + tid;
        const u32 v = j < c ? cnt[j] : 0;
        u32 tot;
        const u32 pre = block_exclusive_scan(v, s_wave, &tot);
        if (j < c && carry + pre < ECH_B && carry + pre + v >= ECH_B) {
            s_thr = j;
            s_need = ECH_B - (carry + pre);
        }
        carry += tot;
        __syncthreads();
        if (s_thr != c) break;
    }
    const u32 thr = s_thr, need = s_need;
    // block rows in index order: lead < thr, then the first `need` rows with lead == thr
    u32 nb = 0, neq = 0;
    for (u32 base = 0; base < L; base += 1024) {
        const u32 i = base + tid;
        const bool live = i < L && st[i] == 0;
        const u32 li = live ? ld[i] : c;
        const bool eq = live && li == thr && thr < c;
        u32 teq;
        const u32 peq = block_exclusive_scan(eq ? 1u : 0u, s_wave, &teq);
        const bool sel = (live && li < thr) || (eq && neq + peq < need);
        u32 tsel;
        const u32 psel = block_exclusive_scan(sel ? 1u : 0u, s_wave, &tsel);
        if (sel && nb + psel < ECH_B) {
            s_rows[nb + psel] = i;
            atomicMin(&s_cmin, li);
        }
        nb += tsel;
        neq += teq;
    }
    const u32 b = __builtin_amdgcn_readfirstlane(nb < ECH_B ? nb : ECH_B);  // uniform: lets row tests branch on scalars
    if (b == 0) {
        if (tid == 0) {
            R->done = 1;
            atomicAdd(ndone, 1u);
        }
        return;
    }
    static_assert(ECH_W == F4_WAVE && ECH_B * ECH_CH == 1024 && ECH_PW % 4 == 0 && ECH_RPW * ECH_PW == ECH_B,
                  "echelon block layout");
    for (u32 x = tid; x < ECH_B * ECH_W; x += 1024) {
        const u32 k = x / ECH_W, j = x % ECH_W;  // element (k, j) lives at k * ECH_RS + j
        s_RZ[k * ECH_RS + j] = (j >= ECH_CH && j - ECH_CH == k) ? 1u : 0u;
    }
    __syncthreads();
    const u32 lane = tid % F4_WAVE, wave = __builtin_amdgcn_readfirstlane(tid / F4_WAVE);
    const bool worker = wave < ECH_PW;
    const u32 rw = ECH_RPW * wave;  // block rows rw .. rw + ECH_RPW - 1 of a working wave
    u32 q = 0, pmask = 0, it = 0;
    u64 nops = 0;  // modular products (counted by lane 0 of each wave; timing option)
    u32 nupd = 0;  // row updates of this working wave in the pivot loop (2 ECH_W products each)
    const bool count_ops = ops != nullptr;
    // chunks of ECH_CH columns from the smallest leading column of the block;
    // each thread holds one entry of the next chunk in a register (its load is
    // in flight while the current chunk is eliminated)
    const u32 kB = tid / ECH_CH, jB = tid % ECH_CH;
    const u64 boff = kB < b ? (u64)s_rows[kB] * c : 0;
    auto load_b = [&](u32 j0) -> u32 { return (kB < b && j0 + jB < c) ? D[boff + j0 + jB] : 0u; };
    const u32 cmin0 = s_cmin;
    u32 bnext = load_b(cmin0);
    // the scan stops early after ECH_EMPTY chunks in a row without a new
    // pivot: the block rows that are not pivots then go back to the remaining
    // rows (they are zero on the scanned columns after the elimination, and
    // the round's update reduces them like any other row, to zero when they
    // are dependent), instead of being followed to the last column
    u32 empty = 0;
    bool early = false;
    for (u32 j0 = cmin0; j0 < c && q < b; j0 += ECH_CH) {
        const u32 q_before = q;
        const u32 w = min((u32)ECH_CH, c - j0);
        s_B[tid] = bnext;
        bnext = load_b(j0 + ECH_CH);
        __syncthreads();
        // chunk part of the rows: Z * B_chunk (B itself while Z is the identity)
        {
            const u32 k = tid / ECH_CH, j = tid % ECH_CH;
            u32 v = s_B[tid];
            if (q && k < b) {
                u64 acc = 0;
                if (SMALL) {
                    for (u32 u = 0; u < b; ++u) acc += (u64)mul24(s_RZ[k * ECH_RS + ECH_CH + u], s_B[u * ECH_CH + j]);
                } else {
                    // four raw products (below 4 p^2 < 2^64) per reduction
                    for (u32 u0 = 0; u0 < b; u0 += 4) {
                        u64 part = 0;
#pragma unroll
                        for (u32 du = 0; du < 4; ++du) {
                            const u32 u = u0 + du;
                            if (u < b) part += (u64)s_RZ[k * ECH_RS + ECH_CH + u] * s_B[u * ECH_CH + j];
                        }
                        acc += fp_reduce_any(f, part);
                    }
                }
                v = fp_reduce_any(f, acc);
                if (j == 0) nops += (u64)b * ECH_CH;  // the row's products, counted once
            }
            s_RZ[k * ECH_RS + j] = v;
        }
        __syncthreads();
        // working waves: own rows into registers, and the first publication
        u32 rv[ECH_RPW];
        if (worker) {
#pragma unroll
            for (u32 h = 0; h < ECH_RPW; ++h) rv[h] = s_RZ[(rw + h) * ECH_RS + lane];
            u32 fr = ECH_B;
#pragma unroll
            for (int h = ECH_RPW - 1; h >= 0; --h) {
                const u32 r = rw + h;
                if (r < b && !((pmask >> r) & 1u) && rv[h] != 0) fr = r;
            }
            reinterpret_cast<u32*>(&s_first[it & 1][lane][0])[wave] = fr;
        }
        __syncthreads();
        while (q < b) {
            // next pivot column: the first column of the chunk where a live
            // (not yet pivot) row is nonzero; pivot row: the lowest such row
            u32 fmin = ECH_B;
#pragma unroll
            for (u32 g = 0; g < ECH_PW / 4; ++g) {
                const uint4 fw = s_first[it & 1][lane][g];
                fmin = min(fmin, min(min(fw.x, fw.y), min(fw.z, fw.w)));
            }
            const u64 all = wave_ballot(fmin < ECH_B && lane < w);
            if (!all) break;
            const u32 jp = __ffsll((long long)all) - 1;
            const u32 kp = (u32)__builtin_amdgcn_readlane((int)fmin, (int)jp);
            if (worker) {
                const u32 prow = s_RZ[kp * ECH_RS + lane];
                const u32 piv = (u32)__builtin_amdgcn_readlane((int)prow, (int)jp);
                const u32 pm2 = pmask | (1u << kp);
#pragma unroll
                for (u32 h = 0; h < ECH_RPW; ++h) {
                    const u32 r = rw + h;
                    const u32 fk = (u32)__builtin_amdgcn_readlane((int)rv[h], (int)jp);
                    if (r < b && r != kp && fk) {
                        rv[h] = fp_ff<SMALL>(f, piv, rv[h], fk, prow);
                        s_RZ[r * ECH_RS + lane] = rv[h];
                        ++nupd;
                    }
                }
                u32 fr = ECH_B;
#pragma unroll
                for (int h = ECH_RPW - 1; h >= 0; --h) {
                    const u32 r = rw + h;
                    if (r < b && !((pm2 >> r) & 1u) && rv[h] != 0) fr = r;
                }
                reinterpret_cast<u32*>(&s_first[(it + 1) & 1][lane][0])[wave] = fr;
                if (tid == 0) {
                    s_pcol[q] = j0 + jp;
                    s_prow[q] = kp;
                }
                pmask = pm2;
            }
            ++q;
            ++it;
            __syncthreads();
        }
        empty = q == q_before ? empty + 1 : 0;
        if (empty >= ECH_EMPTY && q < b && c - j0 > ECH_EMPTY_LEFT * ECH_CH) {
            early = true;
            break;
        }
    }
    if (count_ops && lane == 0) nops += (u64)nupd * 2 * ECH_W;
    // each pivot row is its value at its own pivot column times its normalised
    // form; that value is (Z B) at the column (the rows stay Z B throughout),
    // formed here once instead of being tracked through the pivot steps
    {
        const u32 t = tid / ECH_B, u = tid % ECH_B;  // a half-wave per pivot
        u64 acc = 0;
        if (t < q && u < b)
            acc = fp_mul_t<SMALL>(f, s_RZ[s_prow[t] * ECH_RS + ECH_CH + u], D[(u64)s_rows[u] * c + s_pcol[t]]);
        for (u32 d = ECH_B / 2; d > 0; d >>= 1) acc += (u64)__shfl_xor((unsigned long long)acc, d, F4_WAVE);
        if (u == 0 && t < q) s_pv[t] = fp_reduce_any(f, acc);
    }
    __syncthreads();
    if (tid < q) s_inv[tid] = fp_inv_t<SMALL>(f, s_pv[tid]);
    __syncthreads();
    const u32 npr = R->npr;
    // round record: pivot columns, block rows and normalised Z rows of the pivots
    if (tid < q) {
        R->cols[tid] = s_pcol[tid];
        prlead[S.capb + npr + tid] = s_pcol[tid];
    }
    for (u32 x = tid; x < q * ECH_B; x += 1024) {
        const u32 t = x / ECH_B, u = x % ECH_B;
        R->Z[t * ECH_B + u] = u < b ? fp_mul_t<SMALL>(f, s_RZ[s_prow[t] * ECH_RS + ECH_CH + u], s_inv[t]) : 0u;
    }
    u32 pmk = 0;  // block rows that became pivot rows
    for (u32 t = 0; t < q; ++t) pmk |= 1u << s_prow[t];
    if (tid < b) {
        R->rows[tid] = s_rows[tid];
        // consumed: pivot rows, and after a complete scan the other block rows
        // too (they are zero)
        st[s_rows[tid]] = (!early || ((pmk >> tid) & 1u)) ? 1u : 0u;
    }
    if (ops && nops) atomicAdd(ops, (unsigned long long)nops);
    __syncthreads();
    if (tid == 0) {
        R->q = q;
        R->b = b;
        R->pm = pmk;
        R->npr0 = npr;
        R->npr = npr + q;
        ndone[1 + blockIdx.y] = npr + q;  // pivot rows so far, read back with the done count
        R->cmin = q ? s_pcol[0] : c;
    }
}

// Exact modular dot products in double precision.  A double holds every
// integer below 2^53, and a fused multiply-add whose exact result is an
// integer below 2^53 in magnitude returns it exactly, so a sum of products of
// residues costs one full-rate FMA per product and a single reduction:
//   p < 2^16: 32 products below 2^32 sum to less than 2^37;
//   otherwise the left factor w is split as w_hi 2^16 + w_lo (w_hi < 2^15,
//   w_lo < 2^16), giving sums below 2^51 and 2^52 that recombine as
//   (S_hi mod p) 2^16 + S_lo < 2^53.
// x mod p for an integer-valued double with |x| < 2^53: the estimate
// floor(x / p) from the rounded reciprocal has relative error below 2^-52 and
// |x| / p < 2^52, so it is off by at most one, and x - q p, an integer of
// magnitude below 2p, is formed exactly by the fused multiply-add.
__device__ __forceinline__ double dmod(double x, double pd, double pinv) {
    const double q = floor(x * pinv);
    double r = fma(-q, pd, x);
    r = r < 0.0 ? r + pd : r;
    return r >= pd ? r - pd : r;
}

// One round's update of a tile of ECH_RT row slots x ECH_CT columns, per
// prime class.  Row slots of a system: its L
// remaining rows of D', then its pivot-row store.  Store slots npr0 ..
// npr0+q-1 become this round's new pivot rows NP_t = sum_u Z[t][u] (block row
// u); every other live row r (remaining rows, earlier pivot rows) loses its
// entries on the round's pivot columns: with coef_t = r[col_t],
// r - sum_t coef_t NP_t = r + sum_u w_u (block row u), w = -coef Z.  This is a
// product of the tile's weights (ECH_RT x 32) with the block rows (32 x
// ECH_CT), formed with the exact double-precision sums above.  Only block
// rows that became pivot rows are read (the others have weight zero in every
// row and may be updated in the same launch).  The round's pivot columns of
// the updated rows are left as they are - other tiles read them as the
// coefficients - and are cleared by k_ech_lead afterwards.  Columns left of
// the round's first pivot column are unchanged (the block rows are zero
// there), except in new pivot rows, which are written whole.
#define ECH_RT 32
#define ECH_CT 256
typedef double ech_d4 __attribute__((ext_vector_type(4)));
#define ECH_SPAN_MAX 1024  // most columns of one tile (passes of ECH_CT columns)
#define ECH_SHORT 1024     // rows of at most this many trailing columns use the per-row update forms
template <bool SMALL>
__global__ __launch_bounds__(ECH_CT) void k_ech_gemm(const SegR* segs, u32 S, const u32* tbase, u32* Dp,
                                                     const u32* status, u32* lead, const EchRound* rounds, u32* PR,
                                                     u32 span) {
    __shared__ double2 s_w[ECH_RT][ECH_B];  // weights: (high half, low half); SMALL: (weight, 0)
    __shared__ u32 s_coef[ECH_RT][ECH_B];
    __shared__ u32 s_Z[ECH_B][ECH_B + 1];
    __shared__ u32 s_cols[ECH_B], s_rows[ECH_B];
    __shared__ u32 s_kind[ECH_RT], s_any[ECH_RT];
    __shared__ u32 s_pc[ECH_SPAN_MAX / 32];  // the round's pivot columns inside this column tile
    __shared__ u32 s_lead[ECH_RT];     // whole-row tiles: new leading column of each remaining row
    const u32 tile = blockIdx.x;
    u32 lo = 0, hi = S;  // system: last s with tbase[s] <= tile
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (tbase[mid] <= tile)
            lo = mid;
        else
            hi = mid;
    }
    const u32 s = lo;
    const EchRound* R = rounds + s;
    if (R->done) return;
    const SegR G = segs[s];
    if ((G.small != 0) != SMALL) return;
    const u32 c = G.c, j0 = blockIdx.y * span;
    if (j0 >= c) return;
    const Fp f = G.f;
    const u32 q = R->q, b = R->b, npr0 = R->npr0, cmin = R->cmin, pm = R->pm;
    const u32 l0 = (tile - tbase[s]) * ECH_RT;
    const u32 tid = threadIdx.x;
    const bool left = j0 + span <= cmin;  // only new pivot rows have work left of cmin
    auto row_of = [&](u32 local) -> u32* {
        return local < G.L ? Dp + G.dpb + (u64)local * c : PR + G.prb + (u64)(local - G.L) * c;
    };
    // kinds: 0 no work, 1 update (live remaining row or earlier pivot row),
    // 2 + t new pivot row t
    if (tid < ECH_RT) {
        const u32 local = l0 + tid;
        u32 kind = 0;
        if (local < G.L) {
            if (!left && status[G.lb + local] == 0 && lead[G.lb + local] < c) kind = 1;
        } else if (local - G.L < npr0) {
            if (!left) kind = 1;
        } else if (local - G.L < npr0 + q) {
            kind = 2 + (local - G.L - npr0);
        }
        s_kind[tid] = kind;
        s_any[tid] = 0;
        s_lead[tid] = 0xffffffffu;
    }
    if (tid < ECH_B) {
        s_cols[tid] = tid < q ? R->cols[tid] : 0u;
        s_rows[tid] = tid < b ? R->rows[tid] : 0u;
    }
    if (tid < ECH_SPAN_MAX / 32) s_pc[tid] = 0;
    for (u32 x = tid; x < q * ECH_B; x += ECH_CT) s_Z[x / ECH_B][x % ECH_B] = R->Z[x];
    __syncthreads();
    const u32 lane = tid % F4_WAVE, wv = tid / F4_WAVE;
    const u32 li = lane % 16, lk = lane / 16;
    const u32* D = Dp + G.dpb;
    const u32 jend = min(c, j0 + span);
    u32 xn[ECH_B / 4];  // block-row entries of a wave's next column block (lane: column li, rows 4 kk + lk)
    auto load_x = [&](u32 jb) {
        const u32 j = jb + li;
#pragma unroll
        for (u32 kk = 0; kk < ECH_B / 4; ++kk) {
            const u32 u = 4 * kk + lk;
            xn[kk] = (((pm >> u) & 1u) && j < jend) ? D[(u64)s_rows[u] * c + j] : 0u;
        }
    };
    if (j0 + 16 * wv < jend) load_x(j0 + 16 * wv);
    if (tid < q && s_cols[tid] >= j0 && s_cols[tid] < j0 + span)
        atomicOr(&s_pc[(s_cols[tid] - j0) / 32], 1u << ((s_cols[tid] - j0) % 32));
    // coefficients of the update rows on the round's pivot columns
    for (u32 x = tid; x < ECH_RT * ECH_B; x += ECH_CT) {
        const u32 r = x / ECH_B, t = x % ECH_B;
        u32 v = 0;
        if (s_kind[r] == 1 && t < q) v = row_of(l0 + r)[s_cols[t]];
        s_coef[r][t] = v;
        if (v) s_any[r] = 1;
    }
    __syncthreads();
    const double pd = (double)f.p, pinv = 1.0 / pd;
    // weights w_u = -(sum_t coef_t Z[t][u]) of update rows, Z[t][u] of new pivot row t
    for (u32 x = tid; x < ECH_RT * ECH_B; x += ECH_CT) {
        const u32 r = x / ECH_B, u = x % ECH_B, kind = s_kind[r];
        u32 w = 0;
        if (kind >= 2) {
            w = u < b ? s_Z[kind - 2][u] : 0u;
        } else if (kind == 1 && s_any[r] && u < b) {
            double sh = 0.0, sl = 0.0;
            for (u32 t = 0; t < q; ++t) {
                const u32 cf = s_coef[r][t];
                const double z = (double)s_Z[t][u];
                if (SMALL) {
                    sh = fma((double)cf, z, sh);
                } else {
                    sh = fma((double)(cf >> 16), z, sh);
                    sl = fma((double)(cf & 0xffffu), z, sl);
                }
            }
            const double v = SMALL ? dmod(sh, pd, pinv) : dmod(fma(dmod(sh, pd, pinv), 65536.0, sl), pd, pinv);
            w = fp_neg(f, (u32)v);
        }
        s_w[r][u] = SMALL ? make_double2((double)w, 0.0) : make_double2((double)(w >> 16), (double)(w & 0xffffu));
    }
    // no row of the tile has work (tiles left of the round's first pivot
    // column without new pivot rows, rows without coefficients)
    const bool mine = tid < ECH_RT && (s_kind[tid] >= 2 || (s_kind[tid] == 1 && s_any[tid]));
    if (!__syncthreads_or(mine)) return;
    // a row that fits in one tile has its coefficients read by this workgroup
    // only, so it clears the pivot columns and finds the new leading columns
    // itself (k_ech_lead then finds nothing left to do)
    const bool whole = j0 == 0 && c <= span;
    // The product on the double-precision matrix cores: per wave, blocks of 16
    // columns; a 16 x 16 x 4 product takes A = weights (row i = lane % 16,
    // block-row index k = lane / 16) and B = block rows (k = lane / 16,
    // column lane % 16), and leaves rows lane / 16 + 4 v, v < 4, of column
    // lane % 16.  Every partial sum is an integer below 2^53, so the products
    // are exact in any summation order.
    double ah[ECH_RT / 16][ECH_B / 4], al[ECH_RT / 16][ECH_B / 4];
#pragma unroll
    for (u32 m = 0; m < ECH_RT / 16; ++m)
#pragma unroll
        for (u32 kk = 0; kk < ECH_B / 4; ++kk) {
            const double2 w = s_w[16 * m + li][4 * kk + lk];
            ah[m][kk] = w.x;
            al[m][kk] = w.y;
        }
    // software pipeline over a wave's column blocks: the block rows of the
    // next block and the current entries of this block's updated rows are
    // requested before this block's products, so their latency overlaps them
    // (the first block's block rows were requested before the weights)
    for (u32 jb = j0 + 16 * wv; jb < jend; jb += 16 * (ECH_CT / F4_WAVE)) {
        const u32 j = jb + li;
        double xb[ECH_B / 4];
#pragma unroll
        for (u32 kk = 0; kk < ECH_B / 4; ++kk) xb[kk] = (double)xn[kk];
        const bool pcol = j < jend && ((s_pc[(j - j0) / 32] >> ((j - j0) % 32)) & 1u);
        u32 ov[ECH_RT / 16][4];
#pragma unroll
        for (u32 m = 0; m < ECH_RT / 16; ++m)
#pragma unroll
            for (u32 v = 0; v < 4; ++v) {
                const u32 r = 16 * m + lk + 4 * v;
                ov[m][v] = (s_kind[r] == 1 && s_any[r] && j >= cmin && j < jend && !pcol) ? row_of(l0 + r)[j] : 0u;
            }
        if (jb + 16 * (ECH_CT / F4_WAVE) < jend) load_x(jb + 16 * (ECH_CT / F4_WAVE));
        ech_d4 sh[ECH_RT / 16], sl[ECH_RT / 16];
#pragma unroll
        for (u32 m = 0; m < ECH_RT / 16; ++m) {
            sh[m] = ech_d4{0.0, 0.0, 0.0, 0.0};
            sl[m] = ech_d4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (u32 kk = 0; kk < ECH_B / 4; ++kk)
#pragma unroll
            for (u32 m = 0; m < ECH_RT / 16; ++m) {
                sh[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ah[m][kk], xb[kk], sh[m], 0, 0, 0);
                if (!SMALL) sl[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(al[m][kk], xb[kk], sl[m], 0, 0, 0);
            }
        if (j >= jend) continue;
#pragma unroll
        for (u32 m = 0; m < ECH_RT / 16; ++m)
#pragma unroll
            for (u32 v = 0; v < 4; ++v) {
                const u32 r = 16 * m + lk + 4 * v;
                const u32 kind = s_kind[r];
                if (kind == 0 || (kind == 1 && !s_any[r])) continue;
                if (kind == 1 && j < cmin) continue;
                u32* row = row_of(l0 + r);
                if (kind == 1 && pcol) {
                    if (whole) row[j] = 0;
                    continue;
                }
                const u32 val = (u32)(SMALL ? dmod(sh[m][v], pd, pinv)
                                            : dmod(fma(dmod(sh[m][v], pd, pinv), 65536.0, sl[m][v]), pd, pinv));
                if (kind >= 2) {
                    row[j] = val;
                } else {
                    u32 nv = ov[m][v] + val;  // both below p < 2^31
                    nv = nv >= f.p ? nv - f.p : nv;
                    row[j] = nv;
                    if (whole && nv && l0 + r < G.L) atomicMin(&s_lead[r], j);
                }
            }
    }
    if (whole) {
        __syncthreads();
        if (tid < ECH_RT && s_kind[tid] == 1 && s_any[tid] && l0 + tid < G.L) lead[G.lb + l0 + tid] = s_lead[tid];
    }
}

// After a round's update, one wave per row slot: an updated row (one with a
// nonzero coefficient on the round's pivot columns) gets zeros on those
// columns (exact: the update subtracts coef_t times a row that is 1 at col_t
// and 0 at the other pivot columns), and an updated remaining row gets its
// new leading column (none: the row is zero and leaves the elimination).
#define ECH_LW 4
__global__ __launch_bounds__(64 * ECH_LW) void k_ech_lead(const SegR* segs, u32 S, const u32* ubase, u32* Dp,
                                                          const u32* status, u32* lead, const EchRound* rounds,
                                                          u32* PR) {
    const u32 lane = lane_id();
    const u32 u = blockIdx.x * ECH_LW + threadIdx.x / F4_WAVE;
    if (u >= ubase[S]) return;
    u32 lo = 0, hi = S;  // system: last s with ubase[s] <= u
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (ubase[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    const EchRound* R = rounds + lo;
    if (R->done) return;
    const SegR G = segs[lo];
    const u32 c = G.c, q = R->q, npr0 = R->npr0;
    const u32 local = u - G.ub;
    u32* row;
    bool rem;
    if (local < G.L) {
        if (status[G.lb + local] != 0 || lead[G.lb + local] >= c) return;
        row = Dp + G.dpb + (u64)local * c;
        rem = true;
    } else {
        if (local - G.L >= npr0) return;
        row = PR + G.prb + (u64)(local - G.L) * c;
        rem = false;
    }
    const u32 col = lane < q ? R->cols[lane] : 0u;
    const u32 coef = lane < q ? row[col] : 0u;
    if (!wave_ballot(coef != 0)) return;  // not touched by the update
    if (coef) row[col] = 0;
    if (!rem) return;
    // first nonzero at or after cmin that is not one of the round's pivot
    // columns (the zeros just written are not read back)
    u32 first = 0xffffffffu;
    for (u32 j0 = R->cmin; j0 < c; j0 += F4_WAVE) {
        const u32 j = j0 + lane;
        bool nz = j < c && row[j] != 0;
        for (u32 t = 0; t < q; ++t) nz = nz && j != (u32)__builtin_amdgcn_readlane((int)col, (int)t);
        const u64 m = wave_ballot(nz);
        if (m) {
            first = j0 + (u32)__ffsll((long long)m) - 1;
            break;
        }
    }
    if (lane == 0) lead[G.lb + local] = first;
}


// Update forms for short rows (at most ECH_SHORT trailing columns), where
// per-row parallelism matters more than operand reuse.  Only block rows that
// became pivot rows are read (the others have weight zero in every row and
// may be updated by the same launch).
// The same update for many rows (large batches): one wave per row slot of a
// system (remaining rows of D': the first L slots; the pivot-row store: the
// next cap slots), ECH_UPW slots per workgroup.  Store slots npr0 ..
// npr0+q-1 form this round's new pivot rows NP_t = sum_u Z[t][u] * (block row
// u).  Every other live row r loses its entries on the round's pivot columns:
// with coef_t = r[col_t], r - sum_t coef_t NP_t = r - sum_u w_u (block row u),
// w = coef * Z, so the update reads the block rows directly and does not wait
// for NP.  Lane u of the wave holds block row u and its weight w_u (read
// across the wave with shuffles), and the 32 block-row entries of a column
// are loaded together; no LDS and no workgroup barrier.
#define ECH_UPW 4
__global__ __launch_bounds__(64 * ECH_UPW) void k_ech_update_wave(const SegR* segs, u32 S, const u32* ubase, u32* Dp,
                                                             u32* status, u32* lead, const EchRound* rounds,
                                                             u32* PR) {
    const u32 lane = lane_id();
    const u32 u = blockIdx.x * ECH_UPW + threadIdx.x / F4_WAVE;
    if (u >= ubase[S]) return;
    u32 lo = 0, hi = S;  // system: last s with ubase[s] <= u
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (ubase[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    const u32 s = lo;
    const EchRound* R = rounds + s;
    if (R->done) return;
    const SegR G = segs[s];
    const Fp f = G.f;
    const bool small = G.small != 0;
    const u32 c = G.c, q = R->q, b = R->b, npr0 = R->npr0;
    const u32 local = u - G.ub;
    const u32* D = Dp + G.dpb;
    u32* row;
    bool is_rem, form = false;
    u32 t = 0;
    if (local < G.L) {
        if (status[G.lb + local] != 0 || lead[G.lb + local] >= c) return;
        row = Dp + G.dpb + (u64)local * c;
        is_rem = true;
    } else {
        const u32 k = local - G.L;
        if (k >= npr0 + q) return;
        row = PR + G.prb + (u64)k * c;
        is_rem = false;
        if (k >= npr0) {
            form = true;
            t = k - npr0;
        }
    }
    // block rows and weights of lanes 0 .. b-1 broadcast to every lane once,
    // while the whole wave is active (the column loops below may not be)
    const u32 brow = lane < b ? R->rows[lane] : 0u;
    const u32 pm = R->pm;
    u64 rbase[ECH_B];
#pragma unroll
    for (u32 v = 0; v < ECH_B; ++v) rbase[v] = (u64)(u32)__shfl((int)brow, (int)v, F4_WAVE) * c;
    u32 wv[ECH_B];
    auto spread = [&](u32 w) {
#pragma unroll
        for (u32 v = 0; v < ECH_B; ++v) wv[v] = (u32)__shfl((int)w, (int)v, F4_WAVE);
    };
    // sum_v w_v * (block row v)[j] (w is zero past b)
    auto combo = [&](u32 j) -> u32 {
        u32 x[ECH_B];
#pragma unroll
        for (u32 v = 0; v < ECH_B; ++v) x[v] = ((pm >> v) & 1u) ? D[rbase[v] + j] : 0u;
        u64 acc = 0;
#pragma unroll
        for (u32 v = 0; v < ECH_B; ++v) acc += small ? (u64)mul24(wv[v], x[v]) : (u64)fp_mul(f, wv[v], x[v]);
        return fp_reduce_any(f, acc);
    };
    if (form) {
        spread(lane < b ? R->Z[t * ECH_B + lane] : 0u);
        for (u32 j = lane; j < c; j += F4_WAVE) row[j] = combo(j);
        return;
    }
    const u32 coef = lane < q ? row[R->cols[lane]] : 0u;  // coef_t in lane t
    if (!wave_ballot(coef != 0)) return;
    u64 acc = 0;
    for (u32 t2 = 0; t2 < q; ++t2) {
        const u32 cf = (u32)__shfl((int)coef, (int)t2, F4_WAVE);
        const u32 z = lane < b ? R->Z[t2 * ECH_B + lane] : 0u;
        acc += small ? (u64)mul24(cf, z) : (u64)fp_mul(f, cf, z);
    }
    spread(lane < b ? fp_reduce_any(f, acc) : 0u);
    const u32 cmin = R->cmin;
    u32 first = 0xffffffffu;
    for (u32 j = cmin + lane; j < c; j += F4_WAVE) {
        const u32 sub = combo(j);
        const u32 old = row[j];
        const u32 nv = old >= sub ? old - sub : old + f.p - sub;
        row[j] = nv;
        if (nv && j < first) first = j;
    }
    if (is_rem) {
        // columns below cmin are zero for remaining rows (their lead is >= cmin)
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) first = min(first, (u32)__shfl_xor((int)first, (int)d, F4_WAVE));
        if (lane == 0) lead[G.lb + local] = first;
    }
}


// End of a batch of rounds: a system none of whose remaining rows is live
// (every row a pivot row or zero) is done now, as the next round's block
// step would find, so the batch's readback can end the elimination without
// another batch of rounds.
__global__ __launch_bounds__(256) void k_ech_check(const SegR* segs, const u32* lead, const u32* status,
                                                   EchRound* rounds, u32* ndone) {
    __shared__ u32 s_live;
    EchRound* R = rounds + blockIdx.y;
    if (R->done) return;
    const SegR S = segs[blockIdx.y];
    if (threadIdx.x == 0) s_live = 0;
    __syncthreads();
    for (u32 i = threadIdx.x; i < S.L; i += blockDim.x)
        if (status[S.lb + i] == 0 && lead[S.lb + i] < S.c) s_live = 1;  // every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0 && !s_live) {
        R->done = 1;
        atomicAdd(ndone, 1u);
    }
}

// One kernel per round after the block step (the form for few rows: a
// workgroup per row slot spreads each row over 256 threads), one workgroup per row slot of a
// system (remaining rows of D': the first L slots; the pivot-row store: the
// next cap slots).  Store slots npr0 .. npr0+q-1 form this round's new pivot
// rows NP_t = sum_u Z[t][u] * (block row u).  Every other live row r loses its
// entries on the round's pivot columns: with coef_t = r[col_t],
// r - sum_t coef_t NP_t = r - sum_u w_u (block row u), w = coef * Z, so the
// update reads the block rows directly and does not wait for NP.  The round's
// Z goes to LDS in one cooperative load, and each column's block-row entries
// are loaded together (no load waits behind another).
__global__ __launch_bounds__(256) void k_ech_update_row(const SegR* segs, u32 S, const u32* ubase, u32* Dp, u32* status,
                                                    u32* lead, const EchRound* rounds, u32* PR) {
    __shared__ u32 s_Z[ECH_B * ECH_B];
    __shared__ u32 s_coef[ECH_B], s_w[ECH_B], s_rows[ECH_B];
    __shared__ u32 s_any, s_lead;
    const u32 u = blockIdx.x;
    u32 lo = 0, hi = S;  // system: last s with ubase[s] <= u
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (ubase[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    const u32 s = lo;
    const EchRound* R = rounds + s;
    if (R->done) return;
    const SegR G = segs[s];
    const Fp f = G.f;
    const bool small = G.small != 0;
    const u32 c = G.c, q = R->q, b = R->b, npr0 = R->npr0, pm = R->pm;
    const u32 local = u - G.ub;
    const u32 tid = threadIdx.x;
    const u32* D = Dp + G.dpb;
    u32* row;
    bool is_rem, form = false;
    u32 t = 0;
    if (local < G.L) {
        if (status[G.lb + local] != 0 || lead[G.lb + local] >= c) return;
        row = Dp + G.dpb + (u64)local * c;
        is_rem = true;
    } else {
        const u32 k = local - G.L;
        if (k >= npr0 + q) return;
        row = PR + G.prb + (u64)k * c;
        is_rem = false;
        if (k >= npr0) {
            form = true;
            t = k - npr0;
        }
    }
    // sum_v s_w[v] * (block row v)[j]; s_w is zero past b
    auto combo = [&](u32 j) -> u32 {
        u32 x[ECH_B];
#pragma unroll
        for (u32 v = 0; v < ECH_B; ++v) x[v] = ((pm >> v) & 1u) ? D[(u64)s_rows[v] * c + j] : 0u;
        u64 acc = 0;
#pragma unroll
        for (u32 v = 0; v < ECH_B; ++v) acc += small ? (u64)mul24(s_w[v], x[v]) : (u64)fp_mul(f, s_w[v], x[v]);
        return fp_reduce_any(f, acc);
    };
    if (tid < b) s_rows[tid] = R->rows[tid];
    if (form) {
        if (tid < ECH_B) s_w[tid] = tid < b ? R->Z[t * ECH_B + tid] : 0u;
        __syncthreads();
        for (u32 j = tid; j < c; j += 256) row[j] = combo(j);
        return;
    }
    if (tid == 0) {
        s_any = 0;
        s_lead = 0xffffffffu;
    }
    for (u32 x = tid; x < q * ECH_B; x += 256) s_Z[x] = R->Z[x];
    if (tid < q) {
        const u32 v = row[R->cols[tid]];
        s_coef[tid] = v;
        if (v) atomicOr(&s_any, 1u);
    }
    __syncthreads();
    if (!s_any) return;
    if (tid < ECH_B) {
        u64 acc = 0;
        if (tid < b)
            for (u32 t2 = 0; t2 < q; ++t2) {
                const u32 cf = s_coef[t2], z = s_Z[t2 * ECH_B + tid];
                acc += small ? (u64)mul24(cf, z) : (u64)fp_mul(f, cf, z);
            }
        s_w[tid] = fp_reduce_any(f, acc);
    }
    __syncthreads();
    const u32 cmin = R->cmin;
    u32 first = 0xffffffffu;
    for (u32 j = cmin + tid; j < c; j += 256) {
        const u32 sub = combo(j);
        const u32 old = row[j];
        const u32 nv = old >= sub ? old - sub : old + f.p - sub;
        row[j] = nv;
        if (nv && j < first) first = j;
    }
    if (is_rem) {
        // columns below cmin are zero for remaining rows (their lead is >= cmin)
        if (first != 0xffffffffu) atomicMin(&s_lead, first);
        __syncthreads();
        if (tid == 0) lead[G.lb + local] = s_lead;
    }
}


// ------------------------------------------------------------------- emit
// keys of the pivot-row store slots: (system, leading column) for the system's
// first npr[s] slots, `sent` (sorts after every real key) for the rest; value:
// store row index
__global__ void k_emit_keys(const SegR* segs, const u32* npr, const u32* prlead, u32 cbits, u64 sent, u64* keys,
                            u32* vals) {
    const u32 s = blockIdx.y;
    const SegR G = segs[s];
    const u32 n = npr[s];
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < G.cap; t += gridDim.x * blockDim.x) {
        keys[G.capb + t] = t < n ? (((u64)s << cbits) | prlead[G.capb + t]) : sent;
        vals[G.capb + t] = G.capb + t;
    }
}

// k_emit_keys and their sort for at most SORT_SMALL_MAX store slots in one
// workgroup (keys and values in LDS).
__global__ __launch_bounds__(1024) void k_emit_keys_small(const SegR* segs, u32 S, const u32* npr, const u32* prlead,
                                                          u32 cbits, u64 sent, u32 n, u32 hi_bit, u32 digit,
                                                          u64* keys, u32* vals) {
    extern __shared__ u64 ek_mem[];
    u64* ka = ek_mem;
    u64* kb = ka + SORT_SMALL_MAX;
    u32* va = (u32*)(kb + SORT_SMALL_MAX);
    u32* vb = va + SORT_SMALL_MAX;
    __shared__ u32 run[256];
    __shared__ u32 wcnt[16 * 256];
    __shared__ u32 s_wave[33];
    const u32 tid = threadIdx.x;
    for (u32 sy = 0; sy < S; ++sy) {
        const SegR& G = segs[sy];
        const u32 m = npr[sy];
        for (u32 t = tid; t < G.cap; t += 1024) {
            ka[G.capb + t] = t < m ? (((u64)sy << cbits) | prlead[G.capb + t]) : sent;
            va[G.capb + t] = G.capb + t;
        }
    }
    const bool sw = lds_radix_sort(ka, kb, va, vb, n, 0, hi_bit, digit, 1024, run, wcnt, s_wave);
    const u64* rk = sw ? kb : ka;
    const u32* rv = sw ? vb : va;
    __syncthreads();
    for (u32 i = tid; i < n; i += 1024) {
        keys[i] = rk[i];
        vals[i] = rv[i];
    }
}

// Leading monomial of every sorted pivot-row slot: the dictionary key of its
// leading column (0 for unused slots, or when the matrix has no dictionary).
__device__ __forceinline__ u64 emit_lm(const SegR* segs, const u64* keys, u32 i, u32 kc, u64 sent, const u32* nonpiv,
                                       const u64* dict_keys) {
    const u64 key = keys[i];
    if (key == sent || !dict_keys) return 0;
    const u32 s = kc >= 64 ? 0u : (u32)(key >> kc);
    const u32 lead = kc >= 64 ? (u32)key : (u32)(key & ((1ull << kc) - 1));
    const SegR& G = segs[s];
    return dict_keys[G.db + nonpiv[G.nb + lead]];
}
__global__ void k_emit_lms(const SegR* segs, const u64* keys, u32 n, u32 kc, u64 sent, const u32* nonpiv,
                           const u64* dict_keys, u64* lm) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        lm[i] = emit_lm(segs, keys, i, kc, sent, nonpiv, dict_keys);
}

// Exclusive scan of the per-row counts (pos[0..n]) and the per-system totals
// of k_emit_totals, in one workgroup (n up to a few tens of thousands), and
// the leading monomials of k_emit_lms.
__global__ __launch_bounds__(1024) void k_emit_scan_totals(const u32* cnt, u32 n, const u32* npr, u32 S, u32* pos,
                                                           u32* tot, const SegR* segs, const u64* keys, u32 kc,
                                                           u64 sent, const u32* nonpiv, const u64* dict_keys,
                                                           u64* lm) {
    __shared__ u32 s_wave[33];
    const u32 tid = threadIdx.x;
    u32 carry = 0;
    for (u32 base = 0; base < n; base += 1024) {
        const u32 i = base + tid;
        const u32 v = i < n ? cnt[i] : 0u;
        u32 t;
        const u32 pre = block_exclusive_scan(v, s_wave, &t);
        if (i < n) pos[i] = carry + pre;
        carry += t;
    }
    if (tid == 0) pos[n] = carry;
    __syncthreads();
    u32 ecarry = 0;
    for (u32 base = 0; base < S; base += 1024) {
        const u32 i = base + tid;
        const u32 v = i < S ? npr[i] : 0u;
        u32 t;
        const u32 pre = block_exclusive_scan(v, s_wave, &t);
        if (i < S) tot[i] = pos[ecarry + pre + v] - pos[ecarry + pre];
        ecarry += t;
    }
    for (u32 i = tid; i < n; i += 1024) lm[i] = emit_lm(segs, keys, i, kc, sent, nonpiv, dict_keys);
}

// Row offsets of the emitted rows end where the real rows end: system s owns
// sorted rows [eb[s], eb[s] + npr[s]) with eb the exclusive scan of npr, and
// emits pos[eb[s] + npr[s]] - pos[eb[s]] nonzeros.  One workgroup.
__global__ __launch_bounds__(1024) void k_emit_totals(const u32* npr, u32 S, const u32* pos, u32* tot) {
    __shared__ u32 s_wave[33];
    u32 carry = 0;
    for (u32 base = 0; base < S; base += 1024) {
        const u32 i = base + threadIdx.x;
        const u32 v = i < S ? npr[i] : 0u;
        u32 t;
        const u32 pre = block_exclusive_scan(v, s_wave, &t);
        if (i < S) tot[i] = pos[carry + pre + v] - pos[carry + pre];
        carry += t;
    }
}

// nonzero count of each listed row (wave per row); row `id` of system s lives
// at base + (id - idbase) * c
__global__ void k_count_nz(const SegR* segs, const u64* keys, u32 cbits, u64 sent, const u32* ids, u32 n,
                           int from_pr, const u32* Dp, const u32* PR, u32* cnt) {
    const u32 lane = lane_id();
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 t = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; t < n; t += nw) {
        if (keys[t] == sent) {  // unused store slot
            if (lane == 0) cnt[t] = 0;
            continue;
        }
        const u32 s = cbits >= 64 ? 0u : (u32)(keys[t] >> cbits);
        const SegR G = segs[s];
        const u32* row = from_pr ? PR + G.prb + (u64)(ids[t] - G.capb) * G.c : Dp + G.dpb + (u64)(ids[t] - G.lb) * G.c;
        u32 k = 0;
        for (u32 j = lane; j < G.c; j += F4_WAVE) k += row[j] != 0;
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) k += __shfl_xor(k, d, F4_WAVE);
        if (lane == 0) cnt[t] = k;
    }
}

// row t of the listed rows -> CSR row t over the system's original columns
__global__ void k_emit(const SegR* segs, const u64* keys, u32 cbits, u64 sent, const u32* ids, u32 n, int from_pr,
                       const u32* Dp, const u32* PR, const u32* nonpiv, const u32* optr, u32* ocol, u32* oval) {
    const u32 lane = lane_id();
    const u64 lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 t = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; t < n; t += nw) {
        if (keys[t] == sent) continue;
        const u32 s = cbits >= 64 ? 0u : (u32)(keys[t] >> cbits);
        const SegR G = segs[s];
        const u32* row = from_pr ? PR + G.prb + (u64)(ids[t] - G.capb) * G.c : Dp + G.dpb + (u64)(ids[t] - G.lb) * G.c;
        u32 base = optr[t];
        for (u32 j0 = 0; j0 < G.c; j0 += F4_WAVE) {
            const u32 j = j0 + lane;
            const u32 v = j < G.c ? row[j] : 0;
            const u64 m = wave_ballot(v != 0);
            if (v) {
                const u32 pos = base + __popcll(m & lt);
                ocol[pos] = nonpiv[G.nb + j];
                oval[pos] = v;
            }
            base += __popcll(m);
        }
    }
}

__global__ void k_gather_u32(const u32* in, const u32* idx, u32 n, u32* out) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = in[idx[i]];
}

__global__ void k_row_sys_keys(const u32* row_sys, u32 n, u64* keys) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        keys[i] = (u64)row_sys[i] << 32;
}

__global__ void k_iota(u32* out, u32 n) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = i;
}

static u32 grid_of(u64 items, u32 per, u32 cap) {
    u64 g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (u32)g;
}

static u32 bitlen(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// ------------------------------------------------------------ host side
struct SplitState {
    u32 S = 0;
    std::vector<SegR> segs;
    DBuf<SegR> dsegs;
    DBuf<u32> perm, prow, pivot_cols, nonpiv, lower, tptr;
    DBuf<u64> tent;
    DBuf<u32> T, Tinv;
    u32 P = 0, Ltot = 0, C = 0;
    bool known = false;  // layout from the build's pivot counts (split summary checked later)
};

// Elimination layout of every system from its pivot count: lower rows,
// trailing columns, pivot-row store capacity and the offsets of each
// system's slices in the batched buffers.
static void split_layout(SplitState& X, const std::vector<u32>& p, const std::vector<u32>& npiv,
                         const std::vector<u32>& L) {
    u32 P = 0, Lb = 0, nbase = 0, tb = 0, capb = 0, ub = 0;
    u64 dpb = 0, prb = 0;
    for (u32 i = 0; i < X.S; ++i) {
        SegR& g = X.segs[i];
        g.npiv = npiv[i];
        g.L = L[i];
        g.small = (p[i] < 65536 && g.npiv < 65536) ? 1u : 0u;
        g.pk = (!g.small && p[i] > (1u << 31) - 256 && g.npiv < (1u << 24)) ? (1u << 31) - p[i] : 0u;
        g.pb = P;
        g.lb = Lb;
        g.c = g.N - g.npiv;
        g.nb = nbase;
        g.tb = tb;
        g.cap = std::min(g.L, g.c);
        g.capb = capb;
        g.ub = ub;
        g.dpb = dpb;
        g.prb = prb;
        P += g.npiv;
        Lb += g.L;
        nbase += g.c;
        tb += (g.npiv + PANEL - 1) / PANEL;
        capb += g.cap;
        ub += g.L + g.cap;
        dpb += (u64)g.L * g.c;
        prb += (u64)g.cap * g.c;
    }
    X.P = P;
    X.Ltot = Lb;
}

// The pivot / non-pivot split.  With `summ_out` (2 words per system, device)
// and pivot counts known from the build, the layout is fixed before the split
// kernels run and their own counts are left in summ_out for the caller to
// check with a later readback; otherwise the counts are read back here.
static void do_split(Ctx& c, const std::vector<u32>& p, const Matrix& A, SplitState& X, u32* summ_out = nullptr) {
    hipStream_t s = c.stream;
    const u32 S = A.S, R = A.R;
    X.S = S;
    X.segs.assign(S, SegR());
    u64 C = 0;
    for (u32 i = 0; i < S; ++i) {
        SegR& g = X.segs[i];
        std::memset(&g, 0, sizeof(g));
        g.f = make_fp(p[i]);
        g.N = A.sys[i].N;
        g.cb = (u32)C;
        g.rb = A.sys[i].row_base;
        g.db = A.sys[i].dict_base;
        g.r = A.sys[i].r;
        C += g.N;
    }
    if (C >= (1ull << 31)) throw F4Error{2, "batch has too many columns"};
    X.C = (u32)C;
    X.known = summ_out != nullptr;
    for (u32 i = 0; i < S; ++i)
        if (A.sys[i].npiv > A.sys[i].r || A.sys[i].npiv > A.sys[i].N) X.known = false;
    if (X.known) {
        std::vector<u32> np(S), L(S);
        for (u32 i = 0; i < S; ++i) {
            np[i] = A.sys[i].npiv;
            L[i] = A.sys[i].r - np[i];
        }
        split_layout(X, p, np, L);
    }
    X.dsegs.reset(&c.pool, S);
    upload(c, X.dsegs.ptr, X.segs.data(), S * sizeof(SegR));
    DBuf<u32> ppos(&c.pool, C + 1);
    X.perm.reset(&c.pool, std::max<u64>(C, 1));
    X.prow.reset(&c.pool, std::max<u64>(C, 1));
    X.pivot_cols.reset(&c.pool, std::max<u64>(C, 1));
    X.nonpiv.reset(&c.pool, std::max<u64>(C, 1));
    DBuf<u32> lf(&c.pool, (u64)R + 1), lpos(&c.pool, (u64)R + 1);
    X.lower.reset(&c.pool, std::max<u32>(R, 1));
    DBuf<u32> summ_own;
    if (!X.known) summ_own.reset(&c.pool, 2 * S);
    u32* const summ = X.known ? summ_out : summ_own.ptr;
    if (C <= SPLIT_SMALL_C && R <= SPLIT_SMALL_R) {
        hipLaunchKernelGGL(k_split_small, dim3(1), dim3(1024), (size_t)std::max<u64>(C, 1) * 8, s, X.dsegs.ptr, S,
                           A.row_ptr.ptr, A.col_ind.ptr, A.row_sys.ptr, R, (u32)C, ppos.ptr, lpos.ptr, X.perm.ptr,
                           X.prow.ptr, X.pivot_cols.ptr, X.nonpiv.ptr, X.lower.ptr, summ);
        F4_LAUNCH_CHECK();
    } else {
        DBuf<unsigned long long> best(&c.pool, std::max<u64>(C, 1));
        fill_u64((u64*)best.ptr, C, ~0ull, s);
        if (R) {
            hipLaunchKernelGGL(k_lead_best, dim3(grid_of(R, 256, 4096)), dim3(256), 0, s, X.dsegs.ptr, A.row_ptr.ptr,
                               A.col_ind.ptr, A.row_sys.ptr, R, best.ptr);
            F4_LAUNCH_CHECK();
        }
        if (C) {
            hipLaunchKernelGGL(k_pivflag, dim3(grid_of(C, 256, 4096)), dim3(256), 0, s, best.ptr, (u32)C, ppos.ptr);
            F4_LAUNCH_CHECK();
        }
        exclusive_scan_u32(ppos.ptr, ppos.ptr, C, c.pool, s);
        u32 maxN = 1;
        for (auto& g : X.segs) maxN = std::max(maxN, g.N);
        hipLaunchKernelGGL(k_perm, dim3(std::min<u32>(64, ceil_div(maxN, 256)), S), dim3(256), 0, s, X.dsegs.ptr,
                           best.ptr, ppos.ptr, X.perm.ptr, X.prow.ptr, X.pivot_cols.ptr, X.nonpiv.ptr);
        F4_LAUNCH_CHECK();
        if (R) {
            hipLaunchKernelGGL(k_lower_flags, dim3(grid_of(R, 256, 4096)), dim3(256), 0, s, X.dsegs.ptr,
                               A.row_ptr.ptr, A.col_ind.ptr, A.row_sys.ptr, R, best.ptr, lf.ptr);
            F4_LAUNCH_CHECK();
        }
        exclusive_scan_u32(lf.ptr, lpos.ptr, R, c.pool, s);
        if (R) {
            hipLaunchKernelGGL(k_compact_idx, dim3(grid_of(R, 256, 4096)), dim3(256), 0, s, lf.ptr, lpos.ptr, R,
                               X.lower.ptr);
            F4_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_split_summary, dim3(grid_of(S, 256, 64)), dim3(256), 0, s, X.dsegs.ptr, S, ppos.ptr,
                           lpos.ptr, summ);
        F4_LAUNCH_CHECK();
    }
    if (!X.known) {
        std::vector<u32> hs(2 * S);
        readback(c, hs.data(), summ, hs.size() * 4);
        std::vector<u32> np(S), L(S);
        for (u32 i = 0; i < S; ++i) {
            np[i] = hs[2 * i];
            L[i] = hs[2 * i + 1];
        }
        split_layout(X, p, np, L);
        upload(c, X.dsegs.ptr, X.segs.data(), S * sizeof(SegR));
    }
    u32 tb = 0;
    for (const SegR& g : X.segs) tb += (g.npiv + PANEL - 1) / PANEL;
    const u32 P = X.P;
    X.tptr.reset(&c.pool, (u64)P + 1);
    X.T.reset(&c.pool, (u64)std::max<u32>(tb, 1) * PANEL * PANEL);
    u32 maxP = 1;
    for (auto& g : X.segs) maxP = std::max(maxP, g.npiv);
    if (P) {
        hipLaunchKernelGGL(k_upper_count, dim3(std::min<u32>(4096, ceil_div(maxP, 4)), S), dim3(256), 0, s,
                           X.dsegs.ptr, A.row_ptr.ptr, A.col_ind.ptr, X.prow.ptr, X.perm.ptr, X.tptr.ptr, X.T.ptr);
        F4_LAUNCH_CHECK();
    }
    exclusive_scan_u32(X.tptr.ptr, X.tptr.ptr, P, c.pool, s);
    X.tent.reset(&c.pool, std::max<u64>(A.nnz, 1));
    if (P) {
        hipLaunchKernelGGL(k_upper_fill, dim3(std::min<u32>(4096, ceil_div(maxP, 4)), S), dim3(256), 0, s,
                           X.dsegs.ptr, A.row_ptr.ptr, A.col_ind.ptr, A.val.ptr, X.prow.ptr, X.perm.ptr, X.tptr.ptr,
                           X.tent.ptr, X.T.ptr);
        F4_LAUNCH_CHECK();
    }
    X.Tinv.reset(&c.pool, (u64)std::max<u32>(tb, 1) * PANEL * PANEL);
    if (tb) {
        u32 maxpan = 1;
        for (auto& g : X.segs) maxpan = std::max(maxpan, (g.npiv + PANEL - 1) / PANEL);
        hipLaunchKernelGGL(k_tinv, dim3(std::min<u32>(1024, ceil_div((u64)maxpan * PANEL, 4)), S), dim3(256), 0, s,
                           X.dsegs.ptr, X.T.ptr, X.Tinv.ptr);
        F4_LAUNCH_CHECK();
    }
}

// Reduce the listed rows of every system by its pivot rows: list[lb ..
// lb + cnt) are the system's rows (cnt = L, or r for the tail reduction);
// dense trailing rows go to Dp at segs[s].dpb + local * c.
static void run_trsm(Ctx& c, const Matrix& A, const SplitState& X, const u32* list, int tail, int skip_lead, u32* Dp,
                     u32* lead_out, u32* status, Reduced* kt) {
    unsigned long long* ops = kt && kt->ops.ptr ? (unsigned long long*)kt->ops.ptr : nullptr;
    hipStream_t s = c.stream;
    const u32 S = X.S;
    for (int cls = 0; cls < 3; ++cls) {
        const bool small = cls == 0;
        const size_t accb = small ? 4 : 8;
        u32 nmax = 0, cmax = 0;
        for (const SegR& g : X.segs)
            if (g.c && trsm_class(g) == cls) {
                nmax = std::max(nmax, g.N);
                cmax = std::max(cmax, tail ? g.r : g.L);
            }
        if (!cmax) continue;
        const size_t row_bytes = (size_t)nmax * accb;
        // the kernel's static LDS (panel vectors, partial sums) is below 8 KB
        const size_t budget = c.dev.max_lds > 8192 ? c.dev.max_lds - 8192 : 0;
        if (row_bytes <= budget) {
            // rows per tile: as many as the LDS holds (at most TR_MAXR), unless
            // forced or tuned; fewer rows per tile give more, smaller tiles
            const u32 rmax = (u32)std::min<size_t>(TR_MAXR, budget / row_bytes);
            auto launch = [&](u32 rr, unsigned long long* op) {
                const u32 tiles = ceil_div(cmax, rr);
                auto go = [&](auto mode, auto rows) {
                    constexpr int MODE = decltype(mode)::value, RR = decltype(rows)::value;
                    typedef typename AccOf<MODE>::T AccT;
                    hipLaunchKernelGGL((k_trsm<MODE, true, RR>), dim3(tiles, S), dim3(TR_THREADS), rr * row_bytes, s,
                                       X.dsegs.ptr, 0u, A.row_ptr.ptr, A.col_ind.ptr, A.val.ptr, list, tail, rr, 0u,
                                       skip_lead, X.perm.ptr, X.Tinv.ptr, X.tptr.ptr, X.tent.ptr, (AccT*)nullptr, Dp,
                                       lead_out, status, op);
                };
                auto by_rows = [&](auto mode) {
                    if (rr == 1)
                        go(mode, std::integral_constant<int, 1>{});
                    else if (rr == 2)
                        go(mode, std::integral_constant<int, 2>{});
                    else if (rr == 3)
                        go(mode, std::integral_constant<int, 3>{});
                    else
                        go(mode, std::integral_constant<int, 4>{});
                };
                if (cls == 0)
                    by_rows(std::integral_constant<int, 0>{});
                else if (cls == 1)
                    by_rows(std::integral_constant<int, 1>{});
                else
                    by_rows(std::integral_constant<int, 2>{});
                F4_LAUNCH_CHECK();
            };
            u32 rr = rmax;
            if (c.tune.force_rr) {
                rr = std::min(rmax, c.tune.force_rr);
            } else if (c.tune.on && rmax > 1) {
                // the solve rewrites its outputs completely, so candidates can
                // run on the live data
                u64 rows = 0;
                for (const SegR& g : X.segs)
                    if (g.c && trsm_class(g) == cls) rows += tail ? g.r : g.L;
                std::vector<u32> cands;
                for (u32 v = 1; v <= rmax; ++v) cands.push_back(v);
                rr = tune_pick(c, tune_key(TUNE_TRSM, small ? 1 : 0, tune_lg(rows), tune_lg(nmax)), cands,
                               [](u32) {}, [&](u32 v) { launch(v, nullptr); });
            }
            hipEvent_t ka = kt ? kernel_event(c) : nullptr;
            launch(rr, ops);
            if (ka) kt->ev_trsm.push_back({ka, kernel_event(c)});
            continue;
        }
        // accumulators in global memory (one row per tile), one system and a
        // bounded number of tiles per launch
        const size_t slot = (size_t)TR_MAXR * row_bytes;
        const u32 batch = (u32)std::max<size_t>(1, std::min<size_t>(cmax, ((size_t)1 << 30) / slot));
        DBuf<u8> gacc(&c.pool, (u64)batch * slot);
        for (u32 sy = 0; sy < S; ++sy) {
            const SegR& g = X.segs[sy];
            const u32 cnt = tail ? g.r : g.L;
            if (!g.c || trsm_class(g) != cls || !cnt) continue;
            for (u32 b0 = 0; b0 < cnt; b0 += batch) {
                const u32 nb = std::min(batch, cnt - b0);
                if (cls == 0)
                    hipLaunchKernelGGL((k_trsm<0, false, 1>), dim3(nb, 1), dim3(TR_THREADS), 0, s, X.dsegs.ptr, sy,
                                       A.row_ptr.ptr, A.col_ind.ptr, A.val.ptr, list, tail, 1u, b0, skip_lead,
                                       X.perm.ptr, X.Tinv.ptr, X.tptr.ptr, X.tent.ptr, (u32*)gacc.ptr, Dp, lead_out,
                                       status, ops);
                else if (cls == 1)
                    hipLaunchKernelGGL((k_trsm<1, false, 1>), dim3(nb, 1), dim3(TR_THREADS), 0, s, X.dsegs.ptr, sy,
                                       A.row_ptr.ptr, A.col_ind.ptr, A.val.ptr, list, tail, 1u, b0, skip_lead,
                                       X.perm.ptr, X.Tinv.ptr, X.tptr.ptr, X.tent.ptr, (u64*)gacc.ptr, Dp, lead_out,
                                       status, ops);
                else
                    hipLaunchKernelGGL((k_trsm<2, false, 1>), dim3(nb, 1), dim3(TR_THREADS), 0, s, X.dsegs.ptr, sy,
                                       A.row_ptr.ptr, A.col_ind.ptr, A.val.ptr, list, tail, 1u, b0, skip_lead,
                                       X.perm.ptr, X.Tinv.ptr, X.tptr.ptr, X.tent.ptr, (u64*)gacc.ptr, Dp, lead_out,
                                       status, ops);
                F4_LAUNCH_CHECK();
            }
        }
    }
}

void reduce_batch(Ctx& c, const std::vector<u32>& p, const Matrix& A, Reduced& out) {
    hipStream_t s = c.stream;
    for (const SysPart& P : A.sys)
        if (P.N >= (1u << 26)) throw F4Error{2, "matrix has 2^26 or more columns"};
    hipEvent_t e0 = stage_event(c);
    // one parameter block: round records, update-grid bases and the done
    // counter (uploaded), followed by what the host reads back in one copy
    // per echelon batch: the done count, pivot rows per system, the split's
    // own counts (2 per system, written by the split kernels) and the emitted
    // nonzeros per system
    const u32 S = A.S;
    const size_t rbytes = ((size_t)S * sizeof(EchRound) + 255) & ~(size_t)255;
    const size_t o_nd = (rbytes + 2 * ((size_t)S + 1) * 4 + 255) & ~(size_t)255;
    const size_t nback = (size_t)(S + 1) + 2 * (size_t)S + S;  // words read back, then the leading monomials
    u32 CAP0 = 0;  // pivot-row store slots: sum of min(L, c) <= sum of min(r, N)
    for (const SysPart& P : A.sys) CAP0 += std::min(P.r, P.N);
    const size_t o_lm = (o_nd + nback * 4 + 7) & ~(size_t)7;
    DBuf<u8> eparams(&c.pool, o_lm + (size_t)CAP0 * 8);
    EchRound* const rounds = (EchRound*)eparams.ptr;
    u32* const ubp = (u32*)(eparams.ptr + rbytes);  // row-slot bases, then update-tile bases (S + 1 each)
    u32* const ndone = (u32*)(eparams.ptr + o_nd);  // [0] done count, [1 + s] pivot rows of system s
    u32* const dsumm = ndone + S + 1;               // split counts: pivots, lower rows
    u32* const dtot = dsumm + 2 * S;                // emitted nonzeros per system
    u64* const dlm = (u64*)(eparams.ptr + o_lm);    // leading monomial per sorted pivot-row slot
    SplitState X;
    do_split(c, p, A, X, dsumm);
    hipEvent_t e1 = stage_event(c);
    u64 Dtot = 0, PRtot = 0;
    u32 CAP = 0, UB = 0, maxc = 0, maxcap = 1;
    for (const SegR& g : X.segs) {
        Dtot += (u64)g.L * g.c;
        PRtot += (u64)g.cap * g.c;
        CAP += g.cap;
        UB += g.L + g.cap;
        maxc = std::max(maxc, g.c);
        maxcap = std::max(maxcap, g.cap);
    }
    DBuf<u32> Dp(&c.pool, std::max<u64>(Dtot, 1)), lead(&c.pool, std::max<u32>(X.Ltot, 1));
    DBuf<u32> status(&c.pool, std::max<u32>(X.Ltot, 1));  // cleared by the solve
    if (kernel_timing_on(c)) {
        out.ops.reset(&c.pool, 2);
        fill_u64(out.ops.ptr, 2, 0, s);
    }
    run_trsm(c, A, X, X.lower.ptr, 0, 0, Dp.ptr, lead.ptr, status.ptr, &out);
    hipEvent_t e2 = stage_event(c);

    // echelon of every system's D' (L x c)
    DBuf<u32> PR(&c.pool, std::max<u64>(PRtot, 1)), prlead(&c.pool, std::max<u32>(CAP, 1));
    std::vector<u32> npr(S, 0), rnnz(S, 0);
    u32 active = 0, TT = 0;
    for (const SegR& g : X.segs) active += (g.L && g.c) ? 1 : 0;
    // systems with nothing to eliminate are done from the start
    {
        std::vector<u8> pack(o_nd + (size_t)(S + 1) * 4, 0);
        EchRound* init = (EchRound*)pack.data();
        for (u32 i = 0; i < S; ++i) init[i].done = (X.segs[i].L && X.segs[i].c) ? 0u : 1u;
        u32* hub = (u32*)(pack.data() + rbytes);
        for (u32 i = 0; i < S; ++i) hub[i] = X.segs[i].ub;
        hub[S] = UB;
        u32 tt = 0;
        for (u32 i = 0; i < S; ++i) {
            hub[S + 1 + i] = tt;
            tt += ceil_div((u64)X.segs[i].L + X.segs[i].cap, ECH_RT);
        }
        hub[2 * S + 1] = tt;
        TT = tt;
        upload(c, eparams.ptr, pack.data(), pack.size());
    }
    out.S = S;
    out.sys.assign(S, RedPart());
    // emit plan, speculative: after each echelon batch the pivot-row keys
    // (system, leading column) of every store slot (slots past a system's
    // pivot-row count get a key that sorts last), their sort, the nonzero
    // count of each row, the row offsets and the per-system totals - so one
    // readback tells whether every system is done and how large the output is
    const u32 cbits = std::max<u32>(1, bitlen(std::max<u32>(maxc, 1)));
    const u32 sbits = S > 1 ? bitlen(S - 1) : 0;
    const u32 kc = S > 1 ? cbits : 64u;
    const u64 sent = (cbits + sbits >= 64) ? ~0ull : ((1ull << (cbits + sbits)) - 1);
    out.row_ptr.reset(&c.pool, (u64)CAP + 1);
    DBuf<u64> keys(&c.pool, std::max<u32>(CAP, 1));
    DBuf<u32> ids(&c.pool, std::max<u32>(CAP, 1)), cnt(&c.pool, (u64)CAP + 1);
    hipEvent_t e3 = nullptr;
    std::vector<u32> hb((o_lm - o_nd) / 4 + 2 * (size_t)CAP0, 0);
    if (active) {
        const int cnt_lds = (size_t)maxc * 4 + 32768 <= c.dev.max_lds;
        DBuf<u32> ccnt(&c.pool, cnt_lds ? 1 : std::max<u64>(X.C, 1));
        // rounds per readback: the first batch from min(L, c) (each round yields
        // up to ECH_B pivots), later ones four at a time
        u32 maxlc = 0;
        for (const SegR& g : X.segs) maxlc = std::max(maxlc, std::min(g.L, g.c));
        u32 batch = std::min<u32>(8, std::max<u32>(2, ceil_div(maxlc, ECH_B) + 1));
        // the block step is compiled per prime class; a mixed batch runs both
        bool any_small = false, any_large = false;
        for (const SegR& g : X.segs)
            if (g.L && g.c) (g.small ? any_small : any_large) = true;
        u32 r = 0;
        bool first = true;
        for (;;) {
            for (u32 k = 0; k < batch; ++k) {
                hipEvent_t ka = kernel_event(c);
                unsigned long long* bops = out.ops.ptr ? (unsigned long long*)out.ops.ptr + 1 : nullptr;
                const size_t blds = cnt_lds ? (size_t)maxc * 4 : 0;
                if (any_small)
                    hipLaunchKernelGGL(k_ech_block<true>, dim3(1, S), dim3(1024), blds, s, X.dsegs.ptr, lead.ptr,
                                       status.ptr, Dp.ptr, ccnt.ptr, cnt_lds, rounds, prlead.ptr, ndone, bops);
                if (any_large)
                    hipLaunchKernelGGL(k_ech_block<false>, dim3(1, S), dim3(1024), blds, s, X.dsegs.ptr, lead.ptr,
                                       status.ptr, Dp.ptr, ccnt.ptr, cnt_lds, rounds, prlead.ptr, ndone, bops);
                F4_LAUNCH_CHECK();
                if (ka) out.ev_block.push_back({ka, kernel_event(c)});
                if (maxc <= ECH_SHORT) {
                    // short rows: a workgroup per row while rows are few (each
                    // row spread over 256 threads and the rows over the CUs), a
                    // wave per row for a few thousand rows and more
                    if (UB >= 2048)
                        hipLaunchKernelGGL(k_ech_update_wave, dim3(ceil_div(UB, ECH_UPW)), dim3(64 * ECH_UPW), 0, s,
                                           X.dsegs.ptr, S, ubp, Dp.ptr, status.ptr, lead.ptr, rounds, PR.ptr);
                    else
                        hipLaunchKernelGGL(k_ech_update_row, dim3(std::max<u32>(UB, 1)), dim3(256), 0, s,
                                           X.dsegs.ptr, S, ubp, Dp.ptr, status.ptr, lead.ptr, rounds, PR.ptr);
                    F4_LAUNCH_CHECK();
                } else {
                    // long rows: tiles of row slots x ECH_CT columns (block-row
                    // operands reused across the tile's rows), then the cleared
                    // pivot columns and the new leading columns
                    const dim3 ug(std::max<u32>(TT, 1), ceil_div(maxc, ECH_CT));
                    if (any_small)
                        hipLaunchKernelGGL(k_ech_gemm<true>, ug, dim3(ECH_CT), 0, s, X.dsegs.ptr, S, ubp + S + 1,
                                           Dp.ptr, status.ptr, lead.ptr, rounds, PR.ptr, (u32)ECH_CT);
                    if (any_large)
                        hipLaunchKernelGGL(k_ech_gemm<false>, ug, dim3(ECH_CT), 0, s, X.dsegs.ptr, S, ubp + S + 1,
                                           Dp.ptr, status.ptr, lead.ptr, rounds, PR.ptr, (u32)ECH_CT);
                    F4_LAUNCH_CHECK();
                    hipLaunchKernelGGL(k_ech_lead, dim3(std::max<u32>(ceil_div(UB, ECH_LW), 1)), dim3(64 * ECH_LW), 0,
                                       s, X.dsegs.ptr, S, ubp, Dp.ptr, status.ptr, lead.ptr, rounds, PR.ptr);
                    F4_LAUNCH_CHECK();
                }
                ++r;
            }
            batch = 4;
            hipLaunchKernelGGL(k_ech_check, dim3(1, S), dim3(256), 0, s, X.dsegs.ptr, lead.ptr, status.ptr, rounds,
                               ndone);
            F4_LAUNCH_CHECK();
            e3 = stage_event(c);
            if (CAP <= SORT_SMALL_MAX) {
                const size_t lds = (size_t)SORT_SMALL_MAX * (2 * sizeof(u64) + 2 * sizeof(u32));
                const u32 digit = c.tune.force_digit ? c.tune.force_digit : 8u;
                hipLaunchKernelGGL(k_emit_keys_small, dim3(1), dim3(1024), lds, s, X.dsegs.ptr, S, ndone + 1,
                                   prlead.ptr, cbits, sent, CAP, cbits + sbits, digit, keys.ptr, ids.ptr);
                F4_LAUNCH_CHECK();
            } else {
                hipLaunchKernelGGL(k_emit_keys, dim3(std::min<u32>(16, ceil_div(maxcap, 256)), S), dim3(256), 0, s,
                                   X.dsegs.ptr, ndone + 1, prlead.ptr, cbits, sent, keys.ptr, ids.ptr);
                F4_LAUNCH_CHECK();
                tuned_sort(c, keys.ptr, ids.ptr, CAP, 0, cbits + sbits);
            }
            hipLaunchKernelGGL(k_count_nz, dim3(grid_of(CAP, 4, 4096)), dim3(256), 0, s, X.dsegs.ptr, keys.ptr, kc,
                               sent, ids.ptr, CAP, 1, Dp.ptr, PR.ptr, cnt.ptr);
            F4_LAUNCH_CHECK();
            if (CAP <= 65536) {
                hipLaunchKernelGGL(k_emit_scan_totals, dim3(1), dim3(1024), 0, s, cnt.ptr, CAP, ndone + 1, S,
                                   out.row_ptr.ptr, dtot, X.dsegs.ptr, keys.ptr, kc, sent, X.nonpiv.ptr,
                                   A.dict_keys.ptr, dlm);
                F4_LAUNCH_CHECK();
            } else {
                exclusive_scan_u32(cnt.ptr, out.row_ptr.ptr, CAP, c.pool, s);
                hipLaunchKernelGGL(k_emit_totals, dim3(1), dim3(1024), 0, s, ndone + 1, S, out.row_ptr.ptr, dtot);
                F4_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_emit_lms, dim3(grid_of(CAP, 256, 4096)), dim3(256), 0, s, X.dsegs.ptr,
                                   keys.ptr, CAP, kc, sent, X.nonpiv.ptr, A.dict_keys.ptr, dlm);
                F4_LAUNCH_CHECK();
            }
            // counts and the leading monomials of the sorted slots, one copy
            readback(c, hb.data(), ndone, o_lm + (size_t)CAP * 8 - o_nd);
            if (first && X.known)
                for (u32 i = 0; i < S; ++i)
                    if (hb[S + 1 + 2 * i] != X.segs[i].npiv || hb[S + 2 + 2 * i] != X.segs[i].L)
                        throw F4Error{5, "pivot split disagrees with the symbolic preprocessing"};
            first = false;
            if (hb[0] >= active) break;
            if (r > CAP + 8 + 4 * (X.Ltot / ECH_B + 1)) throw F4Error{5, "echelon did not converge"};
        }
        u32 etot = 0;
        for (u32 i = 0; i < S; ++i) {
            npr[i] = hb[1 + i];
            rnnz[i] = hb[1 + 3 * S + i];
            etot += npr[i];
        }
        // leading monomials of the emitted rows, in row order
        const u64* hl = (const u64*)(hb.data() + (o_lm - o_nd) / 4);
        out.newlm.assign(hl, hl + etot);
    } else {
        if (X.known) {
            readback(c, hb.data(), ndone, nback * 4);
            for (u32 i = 0; i < S; ++i)
                if (hb[S + 1 + 2 * i] != X.segs[i].npiv || hb[S + 2 + 2 * i] != X.segs[i].L)
                    throw F4Error{5, "pivot split disagrees with the symbolic preprocessing"};
        }
        fill_u32(out.row_ptr.ptr, 1, 0, s);
    }
    if (!e3) e3 = stage_event(c);

    // emit RREF(D') over the original columns, rows by (system, leading column):
    // the sorted keys put the E real pivot rows first
    std::vector<u32> eb(S + 1, 0);
    for (u32 i = 0; i < S; ++i) eb[i + 1] = eb[i] + npr[i];
    const u32 E = eb[S];
    u64 nnz = 0;
    for (u32 v : rnnz) nnz += v;
    out.col_ind.reset(&c.pool, std::max<u64>(nnz, 1));
    out.val.reset(&c.pool, std::max<u64>(nnz, 1));
    if (E) {
        hipLaunchKernelGGL(k_emit, dim3(grid_of(E, 4, 4096)), dim3(256), 0, s, X.dsegs.ptr, keys.ptr, kc, sent,
                           ids.ptr, E, 1, Dp.ptr, PR.ptr, X.nonpiv.ptr, out.row_ptr.ptr, out.col_ind.ptr,
                           out.val.ptr);
        F4_LAUNCH_CHECK();
    }
    u64 nb = 0;
    for (u32 i = 0; i < S; ++i) {
        RedPart& P = out.sys[i];
        P.N = X.segs[i].N;
        P.npivot = X.segs[i].npiv;
        P.lower = X.segs[i].L;
        P.rho = npr[i];
        P.rank = P.npivot + P.rho;
        P.nnz = rnnz[i];
        P.row_base = eb[i];
        P.nnz_base = nb;
        P.piv_base = X.segs[i].pb;
        nb += rnnz[i];
    }
    out.pivot_cols = std::move(X.pivot_cols);
    hipEvent_t e4 = stage_event(c);
    out.ev[0] = e0;
    out.ev[1] = e1;
    out.ev[2] = e2;
    out.ev[3] = e3;
    out.ev[4] = e4;
}

void tail_reduce_batch(Ctx& c, const std::vector<u32>& p, const Matrix& A, DBuf<u32>& tptr, DBuf<u32>& tcol,
                       DBuf<u32>& tval) {
    hipStream_t s = c.stream;
    SplitState X;
    do_split(c, p, A, X);
    if (X.Ltot != 0) throw F4Error{6, "inter-reduction matrix has repeated leading monomials"};
    const u32 S = X.S, R = A.R;
    // every row is reduced: the row list is all rows, D' rows follow the row order
    u64 dpb = 0;
    for (u32 i = 0; i < S; ++i) {
        SegR& g = X.segs[i];
        g.lb = g.rb;
        g.dpb = dpb;
        dpb += (u64)g.r * g.c;
    }
    upload(c, X.dsegs.ptr, X.segs.data(), S * sizeof(SegR));
    DBuf<u32> rows(&c.pool, std::max<u32>(R, 1)), Dp(&c.pool, std::max<u64>(dpb, 1)), cnt(&c.pool, (u64)R + 1);
    DBuf<u64> keys(&c.pool, std::max<u32>(R, 1));
    hipLaunchKernelGGL(k_iota, dim3(grid_of(R, 256, 1024)), dim3(256), 0, s, rows.ptr, R);
    F4_LAUNCH_CHECK();
    // system of each row as a key (for the wave kernels below)
    hipLaunchKernelGGL(k_row_sys_keys, dim3(grid_of(R, 256, 1024)), dim3(256), 0, s, A.row_sys.ptr, R, keys.ptr);
    F4_LAUNCH_CHECK();
    run_trsm(c, A, X, rows.ptr, 1, 1, Dp.ptr, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_count_nz, dim3(grid_of(R, 4, 4096)), dim3(256), 0, s, X.dsegs.ptr, keys.ptr, 32u, ~0ull,
                       rows.ptr, R, 0, Dp.ptr, Dp.ptr, cnt.ptr);
    F4_LAUNCH_CHECK();
    tptr.reset(&c.pool, (u64)R + 1);
    exclusive_scan_u32(cnt.ptr, tptr.ptr, R, c.pool, s);
    u32 nnz = 0;
    readback(c, &nnz, tptr.ptr + R, 4);
    tcol.reset(&c.pool, std::max<u32>(nnz, 1));
    tval.reset(&c.pool, std::max<u32>(nnz, 1));
    hipLaunchKernelGGL(k_emit, dim3(grid_of(R, 4, 4096)), dim3(256), 0, s, X.dsegs.ptr, keys.ptr, 32u, ~0ull,
                       rows.ptr, R, 0, Dp.ptr, Dp.ptr, X.nonpiv.ptr, tptr.ptr, tcol.ptr, tval.ptr);
    F4_LAUNCH_CHECK();
}
