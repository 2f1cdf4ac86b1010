// Elimination mod p of the Macaulay matrix (section "PSGE: panel-structured
// Gaussian elimination", two panels: pivot columns / non-pivot columns).
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
//  3. Echelon of D'.  Blocked Gauss-Jordan by lead selection: each round
//     takes up to 32 remaining rows with distinct smallest leading columns
//     (independent by their echelon shape), inverts their 32x32 upper
//     triangular block at those columns, forms the new pivot rows and removes
//     those columns from every other row (remaining rows and earlier pivots).
//  4. Emit the pivot rows of D' as CSR over the original columns, sorted by
//     leading column: the reduced row echelon form of the trailing block.
// All arithmetic is exact mod p with Barrett reduction (equation "mod-fma").
#include <algorithm>
#include <cstring>

#include "internal.hpp"

#define PANEL 64
#define TR_THREADS 256
#define ECH_Q 32

// ------------------------------------------------------------------ split
__global__ void k_lead_best(const u32* row_ptr, const u32* col_ind, u32 r, unsigned long long* best) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        u32 len = row_ptr[i + 1] - row_ptr[i];
        if (len) atomicMin(&best[col_ind[row_ptr[i]]], ((unsigned long long)len << 32) | i);
    }
}

__global__ void k_pivflag(const unsigned long long* best, u32 N, u32* flag) {
    for (u32 c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x)
        flag[c] = best[c] != ~0ull ? 1u : 0u;
}

// perm: original column -> renumbered column (pivots first, then the rest,
// each in original order); prow: pivot index -> its pivot row
__global__ void k_perm(const unsigned long long* best, const u32* ppos, u32 N, u32* perm, u32* prow, u32* pivot_cols,
                       u32* nonpiv) {
    const u32 npiv = ppos[N];
    for (u32 c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        u32 q = ppos[c];
        if (best[c] != ~0ull) {
            perm[c] = q;
            prow[q] = (u32)(best[c] & 0xffffffffu);
            pivot_cols[q] = c;
        } else {
            perm[c] = npiv + (c - q);
            nonpiv[c - q] = c;
        }
    }
}

__global__ void k_lower_flags(const u32* row_ptr, const u32* col_ind, u32 r, const unsigned long long* best,
                              u32* flag) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        u32 len = row_ptr[i + 1] - row_ptr[i];
        flag[i] = (len == 0 || (u32)(best[col_ind[row_ptr[i]]] & 0xffffffffu) != i) ? 1u : 0u;
    }
}

__global__ void k_compact_idx(const u32* flag, const u32* pos, u32 n, u32* out) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (flag[i]) out[pos[i]] = i;
}

// Trailing-entry count of each pivot row (entries beyond its own panel).
__global__ void k_upper_count(const u32* row_ptr, const u32* col_ind, const u32* prow, const u32* perm, u32 npiv,
                              u32* tcnt) {
    const u32 lane = lane_id();
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 q = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; q < npiv; q += nw) {
        const u32 i = prow[q];
        const u32 pend = min((q / PANEL + 1) * PANEL, npiv);  // end of the row's panel among pivots
        u32 cnt = 0;
        for (u32 e = row_ptr[i] + lane; e < row_ptr[i + 1]; e += F4_WAVE) cnt += perm[col_ind[e]] >= pend;
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, F4_WAVE);
        if (lane == 0) tcnt[q] = cnt;
    }
}

// Monic pivot rows: the part inside the row's panel goes to the dense 64x64
// block T[panel] (unit diagonal), the rest to the packed trailing list
// entry = val << 32 | (row within panel) << 26 | renumbered column.
__global__ void k_upper_fill(const u32* row_ptr, const u32* col_ind, const u32* val, const u32* prow, const u32* perm,
                             u32 npiv, Fp f, const u32* tptr, u64* tent, u32* T) {
    const u32 lane = lane_id();
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    const u64 lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (u32 q = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; q < npiv; q += nw) {
        const u32 i = prow[q];
        const u32 kp = q / PANEL, b = q % PANEL;
        const u32 pend = min((kp + 1) * PANEL, npiv);
        const u32 inv = fp_inv(f, val[row_ptr[i]]);
        u32* Tk = T + (u64)kp * PANEL * PANEL + (u64)b * PANEL;
        u32 base = tptr[q];
        for (u32 e0 = row_ptr[i]; e0 < row_ptr[i + 1]; e0 += F4_WAVE) {
            const u32 e = e0 + lane;
            const bool ok = e < row_ptr[i + 1];
            u32 pc = 0, v = 0;
            if (ok) {
                pc = perm[col_ind[e]];
                v = fp_mul(f, val[e], inv);
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

// ------------------------------------------------------ triangular solve
// One workgroup per row to reduce.  SMALL: p < 2^16 (u32 lazy accumulator:
// every column receives at most npiv additions of values < p).
template <bool SMALL>
struct AccOf {
    typedef u64 T;
};
template <>
struct AccOf<true> {
    typedef u32 T;
};

template <bool SMALL, bool LDS>
__global__ __launch_bounds__(TR_THREADS) void k_trsm(const u32* row_ptr, const u32* col_ind, const u32* val,
                                                     const u32* src_rows, u32 row_base, u32 nrows, int skip_lead,
                                                     const u32* perm, u32 N, u32 npiv, Fp f, const u32* T,
                                                     const u32* tptr, const u64* tent,
                                                     typename AccOf<SMALL>::T* gacc, u32* Dp, u64 ldd, u32* lead_out) {
    typedef typename AccOf<SMALL>::T AccT;
    extern __shared__ unsigned char smraw[];
    __shared__ u32 s_x[PANEL];
    __shared__ u64 s_hit;
    __shared__ u32 s_lead;
    const u32 tid = threadIdx.x;
    const u32 ridx = row_base + blockIdx.x;
    if (ridx >= nrows) return;
    AccT* acc = LDS ? (AccT*)smraw : gacc + (u64)blockIdx.x * N;
    for (u32 j = tid; j < N; j += TR_THREADS) acc[j] = 0;
    if (tid == 0) s_lead = 0xffffffffu;
    __syncthreads();
    const u32 i = src_rows[ridx];
    for (u32 e = row_ptr[i] + (skip_lead ? 1 : 0) + tid; e < row_ptr[i + 1]; e += TR_THREADS)
        acc[perm[col_ind[e]]] = val[e];
    __syncthreads();
    const u32 npanels = (npiv + PANEL - 1) / PANEL;
    const u32 lane = lane_id();
    for (u32 kp = 0; kp < npanels; ++kp) {
        if (tid < F4_WAVE) {
            const u32 c0 = kp * PANEL + lane;
            u32 v = 0;
            if (c0 < npiv) v = SMALL ? fp_reduce32(f, (u32)acc[c0]) : fp_reduce_any(f, (u64)acc[c0]);
            const u64 any = wave_ballot(v != 0);
            if (any) {
                const u32* Tk = T + (u64)kp * PANEL * PANEL;
                u32 tc[PANEL];
#pragma unroll
                for (int b = 0; b < PANEL; ++b) tc[b] = Tk[b * PANEL + lane];
#pragma unroll
                for (int b = 0; b < PANEL; ++b) {
                    const u32 xb = __builtin_amdgcn_readlane(v, b);
                    if (xb != 0 && (u32)b < lane) v = fp_fma_t<SMALL>(f, v, f.p - xb, tc[b]);
                }
                if (c0 < npiv) acc[c0] = 0;
            }
            s_x[lane] = v;
            const u64 hit = wave_ballot(v != 0);
            if (lane == 0) s_hit = hit;
        }
        __syncthreads();
        if (s_hit) {
            const u32 qa = kp * PANEL, qb = min(npiv, qa + PANEL);
            const u32 ea = tptr[qa], eb = tptr[qb];
            for (u32 e = ea + tid; e < eb; e += TR_THREADS) {
                const u64 t = tent[e];
                const u32 xb = s_x[(t >> 26) & (PANEL - 1)];
                if (xb) {
                    const u32 add = SMALL ? fp_reduce32(f, (f.p - xb) * (u32)(t >> 32))
                                          : fp_reduce(f, (u64)(f.p - xb) * (u32)(t >> 32));
                    atomicAdd(&acc[(u32)t & 0x3ffffffu], (AccT)add);
                }
            }
        }
        __syncthreads();
    }
    // trailing block row: non-pivot part of the accumulator
    const u32 c = N - npiv;
    u32 first = 0xffffffffu;
    u32* out = Dp + (u64)ridx * ldd;
    for (u32 j = tid; j < c; j += TR_THREADS) {
        const AccT a = acc[npiv + j];
        const u32 v = SMALL ? fp_reduce32(f, (u32)a) : fp_reduce_any(f, (u64)a);
        out[j] = v;
        if (v && j < first) first = j;
    }
    if (first != 0xffffffffu) atomicMin(&s_lead, first);
    __syncthreads();
    if (tid == 0 && lead_out) lead_out[ridx] = s_lead;
}

// ---------------------------------------------------------------- echelon
// Round header (device): [0] done flag, [1] q of this round, [2] npr (pivot
// rows stored so far), [3] npr before this round, [4] smallest chosen column
struct EchRound {
    u32 done, q, npr, npr0, cmin;
    u32 cols[ECH_Q];
    u32 rows[ECH_Q];
    u32 Z[ECH_Q * ECH_Q];  // inverse of the chosen rows' block at the chosen columns
};

__global__ __launch_bounds__(1024) void k_ech_select(u32 L, u32 c, const u32* lead, u32* status, const u32* Dp,
                                                     u64 ldd, u32* cand_g, Fp f, EchRound* R, u32* prlead,
                                                     int cand_lds) {
    extern __shared__ u32 scand[];
    __shared__ u32 s_wave[33];
    __shared__ u32 s_cols[ECH_Q], s_rows[ECH_Q];
    __shared__ u32 s_K[ECH_Q * ECH_Q];
    __shared__ u32 s_Z[ECH_Q * ECH_Q];
    __shared__ u32 s_inv[ECH_Q];
    if (R->done) return;
    u32* cand = cand_lds ? scand : cand_g;
    const u32 tid = threadIdx.x;
    for (u32 j = tid; j < c; j += 1024) cand[j] = 0xffffffffu;
    __syncthreads();
    for (u32 i = tid; i < L; i += 1024)
        if (status[i] == 0 && lead[i] < c) atomicMin(&cand[lead[i]], i);
    __syncthreads();
    // first ECH_Q columns that lead some remaining row
    u32 carry = 0;
    for (u32 base = 0; base < c && carry < ECH_Q; base += 1024) {
        const u32 j = base + tid;
        const u32 fl = (j < c && cand[j] != 0xffffffffu) ? 1u : 0u;
        u32 tot;
        const u32 pre = block_exclusive_scan(fl, s_wave, &tot);
        if (fl && carry + pre < ECH_Q) {
            s_cols[carry + pre] = j;
            s_rows[carry + pre] = cand[j];
        }
        carry += tot;
        __syncthreads();
    }
    const u32 q = carry < ECH_Q ? carry : ECH_Q;
    if (q == 0) {
        if (tid == 0) R->done = 1;
        return;
    }
    // block K[u][t] = D'[row_u][col_t] (upper triangular, nonzero diagonal)
    for (u32 x = tid; x < q * q; x += 1024) {
        const u32 u = x / q, t = x % q;
        s_K[u * ECH_Q + t] = Dp[(u64)s_rows[u] * ldd + s_cols[t]];
    }
    __syncthreads();
    // Z = K^-1 (upper triangular): lane j solves K z = e_j by back substitution
    if (tid < q) s_inv[tid] = fp_inv(f, s_K[tid * ECH_Q + tid]);
    __syncthreads();
    if (tid < q) {
        const u32 j = tid;
        for (int u = (int)q - 1; u >= 0; --u) {
            u64 acc = (u32)u == j ? 1u : 0u;
            for (u32 t = u + 1; t < q; ++t) acc += (u64)(f.p - fp_mul(f, s_K[u * ECH_Q + t], s_Z[t * ECH_Q + j]));
            s_Z[u * ECH_Q + j] = fp_mul(f, fp_reduce_any(f, acc), s_inv[u]);
        }
    }
    __syncthreads();
    for (u32 x = tid; x < q * q; x += 1024) R->Z[(x / q) * ECH_Q + (x % q)] = s_Z[(x / q) * ECH_Q + (x % q)];
    if (tid < q) {
        R->cols[tid] = s_cols[tid];
        R->rows[tid] = s_rows[tid];
        status[s_rows[tid]] = 1;
        prlead[R->npr + tid] = s_cols[tid];
    }
    __syncthreads();
    if (tid == 0) {
        R->q = q;
        R->npr0 = R->npr;
        R->npr = R->npr + q;
        R->cmin = s_cols[0];
    }
}

// New pivot rows NP = Z * (chosen rows), written to the pivot-row store.
__global__ void k_ech_np(u32 c, const u32* Dp, u64 ldd, const EchRound* R, u32* PR, Fp f) {
    if (R->done) return;
    const u32 q = R->q, npr0 = R->npr0;
    const u64 total = (u64)q * c;
    for (u64 x = (u64)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (u64)gridDim.x * blockDim.x) {
        const u32 t = (u32)(x / c), j = (u32)(x % c);
        u32 v = 0;
        if (j >= R->cmin) {
            u64 s = 0;
            for (u32 u = t; u < q; ++u) {
                const u32 z = R->Z[t * ECH_Q + u];
                if (z) s += fp_mul(f, z, Dp[(u64)R->rows[u] * ldd + j]);
            }
            v = fp_reduce_any(f, s);
        }
        PR[(u64)(npr0 + t) * ldd + j] = v;
    }
}

// Remove the chosen columns from every other row: remaining rows of D' (grid
// part 1) and the pivot rows stored in earlier rounds (grid part 2).
template <bool SMALL>
__global__ __launch_bounds__(256) void k_ech_update(u32 L, u32 c, u32* Dp, u64 ldd, u32* status, u32* lead,
                                                    const EchRound* R, u32* PR, Fp f) {
    __shared__ u32 s_coef[ECH_Q];
    __shared__ u32 s_any, s_lead;
    if (R->done) return;
    const u32 q = R->q, npr0 = R->npr0;
    const u32 b = blockIdx.x;
    u32* row;
    bool is_rem;
    if (b < L) {
        if (status[b] != 0 || lead[b] >= c) return;
        row = Dp + (u64)b * ldd;
        is_rem = true;
    } else {
        if (b - L >= npr0) return;
        row = PR + (u64)(b - L) * ldd;
        is_rem = false;
    }
    const u32 tid = threadIdx.x;
    if (tid == 0) {
        s_any = 0;
        s_lead = 0xffffffffu;
    }
    __syncthreads();
    if (tid < q) {
        const u32 v = row[R->cols[tid]];
        s_coef[tid] = v;
        if (v) atomicOr(&s_any, 1u);
    }
    __syncthreads();
    if (!s_any) return;
    const u32 cmin = R->cmin;
    const u32* NP = PR + (u64)npr0 * ldd;
    u32 first = 0xffffffffu;
    for (u32 j = cmin + tid; j < c; j += 256) {
        u64 s = 0;
        for (u32 t = 0; t < q; ++t) {
            const u32 cf = s_coef[t];
            if (cf) {
                const u32 np = NP[(u64)t * ldd + j];
                if (SMALL)
                    s += (u64)cf * np;
                else
                    s += fp_mul(f, cf, np);
            }
        }
        const u32 sub = fp_reduce_any(f, s);
        const u32 old = row[j];
        const u32 nv = old >= sub ? old - sub : old + f.p - sub;
        row[j] = nv;
        if (nv && j < first) first = j;
    }
    if (is_rem) {
        // columns below cmin are zero for remaining rows (their lead is >= cmin)
        if (first != 0xffffffffu) atomicMin(&s_lead, first);
        __syncthreads();
        if (tid == 0) lead[b] = s_lead;
    }
}

// ------------------------------------------------------------------- emit
__global__ void k_count_nz(const u32* rows, u32 nrows, u32 c, u64 ldd, u32* cnt) {
    const u32 lane = lane_id();
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 t = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; t < nrows; t += nw) {
        const u32* row = rows + (u64)t * ldd;
        u32 k = 0;
        for (u32 j = lane; j < c; j += F4_WAVE) k += row[j] != 0;
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) k += __shfl_xor(k, d, F4_WAVE);
        if (lane == 0) cnt[t] = k;
    }
}

// Row t of `rows` (source order `order[t]`) -> CSR row t over original columns.
__global__ void k_emit(const u32* rows, const u32* order, u32 nrows, u32 c, u64 ldd, const u32* nonpiv,
                       const u32* optr, u32* ocol, u32* oval, const u32* lead_col_orig, int with_lead) {
    const u32 lane = lane_id();
    const u64 lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const u32 nw = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 t = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; t < nrows; t += nw) {
        const u32 src = order ? order[t] : t;
        const u32* row = rows + (u64)src * ldd;
        u32 base = optr[t];
        if (with_lead) {
            if (lane == 0) {
                ocol[base] = lead_col_orig[src];
                oval[base] = 1;
            }
            base += 1;
        }
        for (u32 j0 = 0; j0 < c; j0 += F4_WAVE) {
            const u32 j = j0 + lane;
            const u32 v = j < c ? row[j] : 0;
            const u64 m = wave_ballot(v != 0);
            if (v) {
                const u32 pos = base + __popcll(m & lt);
                ocol[pos] = nonpiv[j];
                oval[pos] = v;
            }
            base += __popcll(m);
        }
    }
}

__global__ void k_gather_u32(const u32* in, const u32* idx, u32 n, u32* out) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = in[idx[i]];
}

__global__ void k_iota(u32* out, u32 n) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = i;
}

__global__ void k_lead_keys(const u32* prlead, u32 n, u64* keys, u32* vals) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        keys[i] = prlead[i];
        vals[i] = i;
    }
}

__global__ void k_add_one(u32* cnt, u32 n) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) cnt[i] += 1;
}

static u32 grid_of(u64 items, u32 per, u32 cap) {
    u64 g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (u32)g;
}

// ------------------------------------------------------------ host side
struct SplitState {
    u32 npiv = 0, L = 0;
    DBuf<u32> perm, prow, pivot_cols, nonpiv, lower, tptr;
    DBuf<u64> tent;
    DBuf<u32> T;
};

static void do_split(Ctx& c, const Matrix& A, SplitState& S) {
    hipStream_t s = c.stream;
    const u32 r = A.r, N = A.N;
    DBuf<unsigned long long> best(&c.pool, N);
    fill_u64((u64*)best.ptr, N, ~0ull, s);
    hipLaunchKernelGGL(k_lead_best, dim3(grid_of(r, 256, 4096)), dim3(256), 0, s, A.row_ptr.ptr, A.col_ind.ptr, r,
                       best.ptr);
    F4_LAUNCH_CHECK();
    DBuf<u32> ppos(&c.pool, (u64)N + 1);
    hipLaunchKernelGGL(k_pivflag, dim3(grid_of(N, 256, 4096)), dim3(256), 0, s, best.ptr, N, ppos.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(ppos.ptr, ppos.ptr, N, c.pool, s);
    S.perm.reset(&c.pool, N);
    S.prow.reset(&c.pool, N);
    S.pivot_cols.reset(&c.pool, N);
    S.nonpiv.reset(&c.pool, N);
    hipLaunchKernelGGL(k_perm, dim3(grid_of(N, 256, 4096)), dim3(256), 0, s, best.ptr, ppos.ptr, N, S.perm.ptr,
                       S.prow.ptr, S.pivot_cols.ptr, S.nonpiv.ptr);
    F4_LAUNCH_CHECK();
    DBuf<u32> lf(&c.pool, (u64)r + 1), lpos(&c.pool, (u64)r + 1);
    hipLaunchKernelGGL(k_lower_flags, dim3(grid_of(r, 256, 4096)), dim3(256), 0, s, A.row_ptr.ptr, A.col_ind.ptr, r,
                       best.ptr, lf.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(lf.ptr, lpos.ptr, r, c.pool, s);
    S.lower.reset(&c.pool, r);
    hipLaunchKernelGGL(k_compact_idx, dim3(grid_of(r, 256, 4096)), dim3(256), 0, s, lf.ptr, lpos.ptr, r,
                       S.lower.ptr);
    F4_LAUNCH_CHECK();
    u32 h[2];
    {
        u8* st = staging(c, 8);
        F4_HIP_TRY(hipMemcpyAsync(st, ppos.ptr + N, 4, hipMemcpyDeviceToHost, s));
        F4_HIP_TRY(hipMemcpyAsync(st + 4, lpos.ptr + r, 4, hipMemcpyDeviceToHost, s));
        F4_HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(h, st, 8);
    }
    S.npiv = h[0];
    S.L = h[1];
    // pivot rows: dense diagonal panels + trailing entries
    const u32 npiv = S.npiv;
    const u32 npanels = (npiv + PANEL - 1) / PANEL;
    S.tptr.reset(&c.pool, (u64)npiv + 1);
    S.T.reset(&c.pool, (u64)std::max<u32>(npanels, 1) * PANEL * PANEL);
    fill_u32(S.T.ptr, (u64)npanels * PANEL * PANEL, 0, s);
    if (npiv) {
        hipLaunchKernelGGL(k_upper_count, dim3(grid_of(npiv, 4, 8192)), dim3(256), 0, s, A.row_ptr.ptr,
                           A.col_ind.ptr, S.prow.ptr, S.perm.ptr, npiv, S.tptr.ptr);
        F4_LAUNCH_CHECK();
    }
    exclusive_scan_u32(S.tptr.ptr, S.tptr.ptr, npiv, c.pool, s);
    S.tent.reset(&c.pool, std::max<u64>(A.nnz, 1));
}

static void fill_upper(Ctx& c, u32 p, const Matrix& A, SplitState& S) {
    if (!S.npiv) return;
    Fp f = make_fp(p);
    hipLaunchKernelGGL(k_upper_fill, dim3(grid_of(S.npiv, 4, 8192)), dim3(256), 0, c.stream, A.row_ptr.ptr,
                       A.col_ind.ptr, A.val.ptr, S.prow.ptr, S.perm.ptr, S.npiv, f, S.tptr.ptr, S.tent.ptr, S.T.ptr);
    F4_LAUNCH_CHECK();
}

// Reduce rows src_rows[0..nrows) by the pivot rows: dense trailing rows into Dp.
static void run_trsm(Ctx& c, u32 p, const Matrix& A, const SplitState& S, const u32* src_rows, u32 nrows,
                     int skip_lead, u32* Dp, u64 ldd, u32* lead_out) {
    if (!nrows) return;
    hipStream_t s = c.stream;
    Fp f = make_fp(p);
    const u32 N = A.N;
    const bool small = p < 65536 && S.npiv < 65536;
    const size_t acc_bytes = (size_t)N * (small ? 4 : 8);
    const bool lds = acc_bytes + 1024 <= c.dev.max_lds;
    if (lds) {
        if (small)
            hipLaunchKernelGGL((k_trsm<true, true>), dim3(nrows), dim3(TR_THREADS), acc_bytes, s, A.row_ptr.ptr,
                               A.col_ind.ptr, A.val.ptr, src_rows, 0u, nrows, skip_lead, S.perm.ptr, N, S.npiv, f,
                               S.T.ptr, S.tptr.ptr, S.tent.ptr, (u32*)nullptr, Dp, ldd, lead_out);
        else
            hipLaunchKernelGGL((k_trsm<false, true>), dim3(nrows), dim3(TR_THREADS), acc_bytes, s, A.row_ptr.ptr,
                               A.col_ind.ptr, A.val.ptr, src_rows, 0u, nrows, skip_lead, S.perm.ptr, N, S.npiv, f,
                               S.T.ptr, S.tptr.ptr, S.tent.ptr, (u64*)nullptr, Dp, ldd, lead_out);
        F4_LAUNCH_CHECK();
        return;
    }
    // accumulators in global memory, rows in batches
    const u32 batch = (u32)std::max<u64>(1, std::min<u64>(nrows, (u64)(1u << 30) / acc_bytes));
    DBuf<u8> gacc(&c.pool, (u64)batch * acc_bytes);
    for (u32 b0 = 0; b0 < nrows; b0 += batch) {
        const u32 nb = std::min(batch, nrows - b0);
        if (small)
            hipLaunchKernelGGL((k_trsm<true, false>), dim3(nb), dim3(TR_THREADS), 0, s, A.row_ptr.ptr, A.col_ind.ptr,
                               A.val.ptr, src_rows, b0, nrows, skip_lead, S.perm.ptr, N, S.npiv, f, S.T.ptr,
                               S.tptr.ptr, S.tent.ptr, (u32*)gacc.ptr, Dp, ldd, lead_out);
        else
            hipLaunchKernelGGL((k_trsm<false, false>), dim3(nb), dim3(TR_THREADS), 0, s, A.row_ptr.ptr,
                               A.col_ind.ptr, A.val.ptr, src_rows, b0, nrows, skip_lead, S.perm.ptr, N, S.npiv, f,
                               S.T.ptr, S.tptr.ptr, S.tent.ptr, (u64*)gacc.ptr, Dp, ldd, lead_out);
        F4_LAUNCH_CHECK();
    }
}

void reduce_matrix(Ctx& c, u32 p, const Matrix& A, Reduced& out) {
    hipStream_t s = c.stream;
    if (A.N >= (1u << 26)) throw F4Error{2, "matrix has 2^26 or more columns"};
    Fp f = make_fp(p);
    hipEvent_t e0 = stage_event(c);
    SplitState S;
    do_split(c, A, S);
    fill_upper(c, p, A, S);
    const u32 N = A.N, npiv = S.npiv, L = S.L, cc = N - npiv;
    hipEvent_t e1 = stage_event(c);
    out.N = N;
    out.npivot = npiv;
    out.lower = L;
    out.pivot_cols = std::move(S.pivot_cols);
    const u64 ldd = cc;
    DBuf<u32> Dp(&c.pool, std::max<u64>((u64)L * ldd, 1)), lead(&c.pool, std::max<u32>(L, 1));
    if (cc) run_trsm(c, p, A, S, S.lower.ptr, L, 0, Dp.ptr, ldd, lead.ptr);
    hipEvent_t e2 = stage_event(c);

    // echelon of D' (L x cc)
    u32 rho = 0;
    const u32 cap = std::min(L, cc);
    DBuf<u32> PR(&c.pool, std::max<u64>((u64)cap * ldd, 1)), prlead(&c.pool, std::max<u32>(cap, 1));
    if (L && cc) {
        DBuf<u32> status(&c.pool, L);
        fill_u32(status.ptr, L, 0, s);
        DBuf<EchRound> R(&c.pool, 1);
        fill_u32((u32*)R.ptr, sizeof(EchRound) / 4, 0, s);
        const int cand_lds = (size_t)cc * 4 + 12288 <= c.dev.max_lds;
        DBuf<u32> cand(&c.pool, cand_lds ? 1 : cc);
        const bool small = p < 65536;
        const u32 npgrid = grid_of((u64)ECH_Q * cc, 256, 4096);
        u32 done = 0;
        u32 rounds = 0;
        while (!done) {
            for (int k = 0; k < 4; ++k) {
                hipLaunchKernelGGL(k_ech_select, dim3(1), dim3(1024), cand_lds ? (size_t)cc * 4 : 0, s, L, cc,
                                   lead.ptr, status.ptr, Dp.ptr, ldd, cand.ptr, f, R.ptr, prlead.ptr, cand_lds);
                F4_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_ech_np, dim3(npgrid), dim3(256), 0, s, cc, Dp.ptr, ldd, R.ptr, PR.ptr, f);
                F4_LAUNCH_CHECK();
                if (small)
                    hipLaunchKernelGGL(k_ech_update<true>, dim3(L + cap), dim3(256), 0, s, L, cc, Dp.ptr, ldd,
                                       status.ptr, lead.ptr, R.ptr, PR.ptr, f);
                else
                    hipLaunchKernelGGL(k_ech_update<false>, dim3(L + cap), dim3(256), 0, s, L, cc, Dp.ptr, ldd,
                                       status.ptr, lead.ptr, R.ptr, PR.ptr, f);
                F4_LAUNCH_CHECK();
                ++rounds;
            }
            u32 h[3];
            readback(c, h, R.ptr, 12);
            done = h[0];
            rho = h[2];
            if (rounds > cap + 8) throw F4Error{5, "echelon did not converge"};
        }
    }
    hipEvent_t e3 = stage_event(c);

    // emit RREF(D') over the original columns, rows by leading column
    out.rho = rho;
    out.rank = npiv + rho;
    out.row_ptr.reset(&c.pool, (u64)rho + 1);
    if (rho) {
        DBuf<u64> keys(&c.pool, rho);
        DBuf<u32> order(&c.pool, rho);
        hipLaunchKernelGGL(k_lead_keys, dim3(grid_of(rho, 256, 1024)), dim3(256), 0, s, prlead.ptr, rho, keys.ptr,
                           order.ptr);
        F4_LAUNCH_CHECK();
        u32 bits = 1;
        while ((1ull << bits) < cc) ++bits;
        radix_sort_pairs(keys.ptr, order.ptr, rho, 0, bits, c.pool, s);
        DBuf<u32> cnt(&c.pool, (u64)rho + 1);
        DBuf<u32> sorted_cnt(&c.pool, (u64)rho + 1);
        hipLaunchKernelGGL(k_count_nz, dim3(grid_of(rho, 4, 4096)), dim3(256), 0, s, PR.ptr, rho, cc, ldd, cnt.ptr);
        F4_LAUNCH_CHECK();
        // counts in output order
        hipLaunchKernelGGL(k_gather_u32, dim3(grid_of(rho, 256, 1024)), dim3(256), 0, s, cnt.ptr, order.ptr, rho,
                           sorted_cnt.ptr);
        F4_LAUNCH_CHECK();
        exclusive_scan_u32(sorted_cnt.ptr, out.row_ptr.ptr, rho, c.pool, s);
        u32 nnz = 0;
        readback(c, &nnz, out.row_ptr.ptr + rho, 4);
        out.nnz = nnz;
        out.col_ind.reset(&c.pool, std::max<u32>(nnz, 1));
        out.val.reset(&c.pool, std::max<u32>(nnz, 1));
        hipLaunchKernelGGL(k_emit, dim3(grid_of(rho, 4, 4096)), dim3(256), 0, s, PR.ptr, order.ptr, rho, cc, ldd,
                           S.nonpiv.ptr, out.row_ptr.ptr, out.col_ind.ptr, out.val.ptr, (const u32*)nullptr, 0);
        F4_LAUNCH_CHECK();
    } else {
        fill_u32(out.row_ptr.ptr, 1, 0, s);
        out.nnz = 0;
        out.col_ind.reset(&c.pool, 1);
        out.val.reset(&c.pool, 1);
    }
    hipEvent_t e4 = stage_event(c);
    if (e0) {
        F4_HIP_TRY(hipEventSynchronize(e4));
        out.t_split = event_ms(e0, e1);
        out.t_trsm = event_ms(e1, e2);
        out.t_echelon = event_ms(e2, e3);
        out.t_emit = event_ms(e3, e4);
    }
}

void tail_reduce_matrix(Ctx& c, u32 p, const Matrix& A, DBuf<u32>& tptr, DBuf<u32>& tcol, DBuf<u32>& tval) {
    hipStream_t s = c.stream;
    SplitState S;
    do_split(c, A, S);
    if (S.L != 0) throw F4Error{6, "inter-reduction matrix has repeated leading monomials"};
    fill_upper(c, p, A, S);
    const u32 r = A.r, cc = A.N - S.npiv;
    const u64 ldd = std::max<u32>(cc, 1);
    DBuf<u32> rows(&c.pool, r), Dp(&c.pool, (u64)r * ldd), cnt(&c.pool, (u64)r + 1);
    hipLaunchKernelGGL(k_iota, dim3(grid_of(r, 256, 1024)), dim3(256), 0, s, rows.ptr, r);
    F4_LAUNCH_CHECK();
    if (cc) run_trsm(c, p, A, S, rows.ptr, r, 1, Dp.ptr, ldd, nullptr);
    hipLaunchKernelGGL(k_count_nz, dim3(grid_of(r, 4, 4096)), dim3(256), 0, s, Dp.ptr, r, cc, ldd, cnt.ptr);
    F4_LAUNCH_CHECK();
    tptr.reset(&c.pool, (u64)r + 1);
    exclusive_scan_u32(cnt.ptr, tptr.ptr, r, c.pool, s);
    u32 nnz = 0;
    readback(c, &nnz, tptr.ptr + r, 4);
    tcol.reset(&c.pool, std::max<u32>(nnz, 1));
    tval.reset(&c.pool, std::max<u32>(nnz, 1));
    hipLaunchKernelGGL(k_emit, dim3(grid_of(r, 4, 4096)), dim3(256), 0, s, Dp.ptr, (const u32*)nullptr, r, cc, ldd,
                       S.nonpiv.ptr, tptr.ptr, tcol.ptr, tval.ptr, (const u32*)nullptr, 0);
    F4_LAUNCH_CHECK();
}
