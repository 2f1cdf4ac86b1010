// Block Wiedemann over F_p for left-kernel vectors of a Macaulay matrix
// (section "Block Wiedemann and Block Lanczos": kernel vectors by black-box
// linear algebra; Remark "Syzygies, revisited": v^T A = 0 is a syzygy among
// the shifted reducers by Proposition "Kernel equals syzygies under
// dictionary closure").  The square operator is B = A D A^T (D a diagonal of
// nonzero elements); every step below runs on the device:
//   1. the projected block Krylov sequence S_t = X^T B^t (B Y): two block
//      operator applications (k_spmm on A^T with D folded into its values,
//      then on A) and a projection per term;
//   2. the generator: an M-Basis sigma-basis of [S(x)^T ; -I_b] (residual of
//      every row at the current order, one wave's fraction-free elimination in
//      the order of (shift, index), the row operations and the multiplication
//      of pivot rows by x applied to all coefficients), one order per pass;
//   3. kernel vectors: u = sum_m B^m Y f_m by Horner for every generator
//      column at once, then B applied until each column vanishes (its last
//      nonzero iterate is in ker B), and A^T v = 0 checked.
// Sums of products of residues are exact 64-bit (or 96-bit) integer sums,
// reduced once.
#include "internal.hpp"

// tval_d[e] = tval[e] * d[j] for the entries of row j of A^T (column j of A)
__global__ void k_bw_scale_rows(Fp f, u32 nrows, const u32* __restrict__ ptr, const u32* __restrict__ val,
                                const u32* __restrict__ d, u32* __restrict__ out) {
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nrows) return;
    const u32 dj = fp_reduce32(f, d[j]);
    for (u32 e = ptr[j]; e < ptr[j + 1]; ++e) out[e] = fp_mul(f, fp_reduce32(f, val[e]), dj);
}

// S64[k b + l] += sum over this workgroup's rows g of X[g][k] Z[g][l]: one
// thread per (k, l), the products summed exactly in 96 bits, reduced once
__global__ __launch_bounds__(256) void k_bw_proj(Fp f, u32 r, u32 b, u32 rows_per, const u32* __restrict__ X,
                                                 const u32* __restrict__ Z, unsigned long long* __restrict__ S64) {
    const u32 tid = threadIdx.x;
    if (tid >= b * b) return;
    const u32 k = tid / b, l = tid % b;
    const u32 g0 = blockIdx.x * rows_per, g1 = min(r, g0 + rows_per);
    u64 lo = 0;
    u32 hi = 0;
    for (u32 g = g0; g < g1; ++g) {
        const u64 t = (u64)fp_reduce32(f, X[(u64)g * b + k]) * Z[(u64)g * b + l];
        const u64 n = lo + t;
        hi += n < lo ? 1u : 0u;
        lo = n;
    }
    const u32 c64 = fp_reduce(f, (u64)f.r32 * f.r32);  // 2^64 mod p
    const u32 v = fp_reduce_any(f, (u64)fp_reduce_any(f, lo) + fp_reduce(f, (u64)fp_reduce32(f, hi) * c64));
    if (v) atomicAdd(&S64[tid], (unsigned long long)v);
}

__global__ void k_bw_reduce64(Fp f, u64 n, const unsigned long long* __restrict__ in, u32* __restrict__ out) {
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fp_reduce_any(f, in[i]);
}

static void bw_apply(Ctx& c, u32 p, const BwCsr& A, u32 w, const u32* V, u32* U, u32* Out) {
    // Out = A (D (A^T V)): U is N x w scratch
    spmm_run(c.stream, p, A.N, w, A.tptr, A.tidx, A.tval_d, V, U);
    spmm_run(c.stream, p, A.r, w, A.ptr, A.idx, A.val, U, Out);
}

void bw_scale_transpose(Ctx& c, u32 p, const BwCsr& A, const u32* d, u32* tval_d) {
    if (!A.N) return;
    hipLaunchKernelGGL(k_bw_scale_rows, dim3(ceil_div(A.N, 256)), dim3(256), 0, c.stream, make_fp(p), A.N, A.tptr,
                       A.tval, d, tval_d);
    F4_LAUNCH_CHECK();
}

void bw_sequence(Ctx& c, u32 p, const BwCsr& A, u32 b, const u32* X, const u32* Y, u32 L, u32* S) {
    hipStream_t s = c.stream;
    const Fp f = make_fp(p);
    DBuf<u32> U(&c.pool, std::max<u64>((u64)A.N * b, 1)), Z(&c.pool, std::max<u64>((u64)A.r * b, 1)),
        Z2(&c.pool, std::max<u64>((u64)A.r * b, 1));
    DBuf<u64> S64(&c.pool, std::max<u64>((u64)L * b * b, 1));
    fill_u64(S64.ptr, (u64)L * b * b, 0, s);
    bw_apply(c, p, A, b, Y, U.ptr, Z.ptr);
    const u32 groups = std::max<u32>(1, std::min<u32>(1024, ceil_div(A.r, 64)));
    const u32 rows_per = ceil_div(A.r, groups);
    for (u32 t = 0; t < L; ++t) {
        if (A.r) {
            hipLaunchKernelGGL(k_bw_proj, dim3(groups), dim3(256), 0, s, f, A.r, b, rows_per, X, Z.ptr,
                               (unsigned long long*)S64.ptr + (u64)t * b * b);
            F4_LAUNCH_CHECK();
        }
        if (t + 1 < L) {
            bw_apply(c, p, A, b, Z.ptr, U.ptr, Z2.ptr);
            std::swap(Z.ptr, Z2.ptr);
        }
    }
    const u64 n = (u64)L * b * b;
    if (n) {
        hipLaunchKernelGGL(k_bw_reduce64, dim3(ceil_div(n, 256)), dim3(256), 0, s, f, n,
                           (const unsigned long long*)S64.ptr, S);
        F4_LAUNCH_CHECK();
    }
}

// ------------------------------------------------------------ M-Basis
// P: m x m polynomial entries (m = 2b), coefficient l of entry (i, j) at
// P[(i m + j) W + l], W = L + 2 (a row's degree is at most its shift, at most
// L + 1).  Shifts start at (0^b, 1^b).

// residual coefficient of x^k of row i, column c of P F, F = [S(x)^T ; -I]:
// sum_{j<b} sum_{l<=min(k, s_i)} P[i][j][l] S[k-l][c][j] - P[i][b+c][k]
__global__ __launch_bounds__(256) void k_mb_residual(Fp f, u32 b, u32 W, u32 k, const u32* __restrict__ P,
                                                     const u32* __restrict__ S, const u32* __restrict__ shifts,
                                                     u32* __restrict__ Delta) {
    __shared__ u32 s_part[256 / F4_WAVE];
    const u32 c = blockIdx.x, i = blockIdx.y, m = 2 * b, tid = threadIdx.x;
    const u32 lmax = min(k, shifts[i]), len = lmax + 1;
    u64 lo = 0;
    u32 hi = 0;
    for (u32 x = tid; x < b * len; x += 256) {
        const u32 j = x / len, l = x % len;
        const u64 t = (u64)P[((u64)i * m + j) * W + l] * S[((u64)(k - l) * b + c) * b + j];
        const u64 n = lo + t;
        hi += n < lo ? 1u : 0u;
        lo = n;
    }
    const u32 c64 = fp_reduce(f, (u64)f.r32 * f.r32);
    u64 v = (u64)fp_reduce_any(f, lo) + fp_reduce(f, (u64)fp_reduce32(f, hi) * c64);
    for (u32 dd = F4_WAVE / 2; dd > 0; dd >>= 1) v += __shfl_xor((unsigned long long)v, dd, F4_WAVE);
    if (lane_id() == 0) s_part[tid / F4_WAVE] = fp_reduce_any(f, v);
    __syncthreads();
    if (tid == 0) {
        u64 sum = 0;
        for (u32 w = 0; w < 256 / F4_WAVE; ++w) sum += s_part[w];
        const u32 own = P[((u64)i * m + b + c) * W + k];
        Delta[i * b + c] = fp_reduce(f, fp_reduce_any(f, sum) + (u64)(f.p - own));
    }
}

// One wave: the elimination of the residual rows in the order of (shift,
// index), fraction-free (row_j <- piv row_j - D_j[c] row_i for the rows j
// after the pivot row i with D_j[c] != 0, c the pivot row's first nonzero
// column).  Writes the row transform T (m x m, applied to P as P' = T P),
// the pivot flags and the new shifts (+1 for pivot rows).
__global__ __launch_bounds__(64) void k_mb_elim(Fp f, u32 b, const u32* __restrict__ Delta,
                                                const u32* __restrict__ shifts_in, u32* __restrict__ shifts_out,
                                                u32* __restrict__ T, u32* __restrict__ piv) {
    __shared__ u32 s_D[32][16];
    __shared__ u32 s_T[32][32];
    __shared__ u32 s_order[32];
    const u32 m = 2 * b, lane = threadIdx.x;
    for (u32 x = lane; x < m * b; x += 64) s_D[x / b][x % b] = Delta[x];
    for (u32 x = lane; x < m * m; x += 64) s_T[x / m][x % m] = (x / m == x % m) ? 1u : 0u;
    u32 si = 0;
    if (lane < m) {
        si = shifts_in[lane];
        u32 rank = 0;  // position in the order of (shift, index)
        for (u32 j = 0; j < m; ++j) {
            const u32 sj = shifts_in[j];
            rank += (sj < si || (sj == si && j < lane)) ? 1u : 0u;
        }
        s_order[rank] = lane;
    }
    __syncthreads();
    u32 pivmask = 0;
    for (u32 a = 0; a < m; ++a) {
        const u32 i = s_order[a];
        const u64 nzc = __ballot(lane < b && s_D[i][lane] != 0);
        if (!nzc) continue;
        const u32 c = __ffsll((long long)nzc) - 1;
        pivmask |= 1u << i;
        const u32 pv = s_D[i][c];
        // rows after i in the order: lane handles row order[a + 1 + lane]
        const u32 jpos = a + 1 + lane;
        u32 j = 0, fj = 0;
        if (jpos < m) {
            j = s_order[jpos];
            fj = s_D[j][c];
        }
        __syncthreads();
        if (jpos < m && fj) {
            for (u32 x = 0; x < b; ++x)
                s_D[j][x] = fp_reduce(f, (u64)fp_mul(f, pv, s_D[j][x]) + (f.p - fp_mul(f, fj, s_D[i][x])));
            for (u32 x = 0; x < m; ++x)
                s_T[j][x] = fp_reduce(f, (u64)fp_mul(f, pv, s_T[j][x]) + (f.p - fp_mul(f, fj, s_T[i][x])));
        }
        __syncthreads();
    }
    for (u32 x = lane; x < m * m; x += 64) T[x] = s_T[x / m][x % m];
    if (lane < m) {
        const u32 pv = (pivmask >> lane) & 1u;
        piv[lane] = pv;
        shifts_out[lane] = si + pv;
    }
}

// P'[i][j][l] = sum_q T[i][q] P[q][j][l'] with l' = l - 1 for pivot rows i
// (multiplication by x) and l' = l otherwise, for l < lcount (higher
// coefficients are zero in both buffers)
__global__ __launch_bounds__(256) void k_mb_apply(Fp f, u32 b, u32 W, u32 lcount, const u32* __restrict__ Pin,
                                                  u32* __restrict__ Pout, const u32* __restrict__ T,
                                                  const u32* __restrict__ piv) {
    __shared__ u32 s_T[32 * 32];
    __shared__ u32 s_piv[32];
    const u32 m = 2 * b, tid = threadIdx.x;
    for (u32 x = tid; x < m * m; x += 256) s_T[x] = T[x];
    if (tid < m) s_piv[tid] = piv[tid];
    __syncthreads();
    const u64 e = (u64)blockIdx.x * 256 + tid;
    const u64 total = (u64)m * m * lcount;
    if (e >= total) return;
    const u32 l = (u32)(e % lcount), ij = (u32)(e / lcount), i = ij / m, j = ij % m;
    u32 v = 0;
    if (!(s_piv[i] && l == 0)) {
        const u32 ls = s_piv[i] ? l - 1 : l;
        u64 acc = 0;
        for (u32 q = 0; q < m; ++q) {
            const u32 t = s_T[i * m + q];
            if (t) acc += fp_mul(f, t, Pin[((u64)q * m + j) * W + ls]);
        }
        v = fp_reduce_any(f, acc);
    }
    Pout[((u64)i * m + j) * W + l] = v;
}

__global__ void k_bw_identity(u32 m, u32 W, u32* P) {
    for (u32 i = threadIdx.x; i < m; i += blockDim.x) P[((u64)i * m + i) * W] = 1u;
}

void bw_mbasis(Ctx& c, u32 p, u32 b, u32 L, const u32* S, u32* P, u32* shifts) {
    hipStream_t s = c.stream;
    const Fp f = make_fp(p);
    const u32 m = 2 * b, W = L + 2;
    const u64 psize = (u64)m * m * W;
    DBuf<u32> P2(&c.pool, psize), Delta(&c.pool, (u64)m * b), T(&c.pool, (u64)m * m), piv(&c.pool, m),
        sh2(&c.pool, m);
    fill_u32(P, psize, 0, s);
    fill_u32(P2.ptr, psize, 0, s);
    // P = I, shifts (0^b, 1^b)
    std::vector<u32> hs(m);
    for (u32 i = 0; i < m; ++i) hs[i] = i < b ? 0u : 1u;
    upload(c, shifts, hs.data(), m * 4);
    hipLaunchKernelGGL(k_bw_identity, dim3(1), dim3(64), 0, s, m, W, P);
    F4_LAUNCH_CHECK();
    u32* cur = P;
    u32* nxt = P2.ptr;
    u32* scur = shifts;
    u32* snxt = sh2.ptr;
    for (u32 k = 0; k < L; ++k) {
        hipLaunchKernelGGL(k_mb_residual, dim3(b, m), dim3(256), 0, s, f, b, W, k, cur, S, scur, Delta.ptr);
        F4_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_mb_elim, dim3(1), dim3(64), 0, s, f, b, Delta.ptr, scur, snxt, T.ptr, piv.ptr);
        F4_LAUNCH_CHECK();
        // degrees after this order are at most k + 2
        const u32 lcount = std::min(W, k + 3);
        const u64 total = (u64)m * m * lcount;
        hipLaunchKernelGGL(k_mb_apply, dim3(ceil_div(total, 256)), dim3(256), 0, s, f, b, W, lcount, cur, nxt,
                           T.ptr, piv.ptr);
        F4_LAUNCH_CHECK();
        std::swap(cur, nxt);
        std::swap(scur, snxt);
    }
    if (cur != P) F4_HIP_TRY(hipMemcpyAsync(P, cur, psize * 4, hipMemcpyDeviceToDevice, s));
    if (scur != shifts) F4_HIP_TRY(hipMemcpyAsync(shifts, scur, m * 4, hipMemcpyDeviceToDevice, s));
}

// ----------------------------------------------------- kernel vectors
// U[g][j] = (U[g][j] + sum_k Y[g][k] F[k][j]) mod p, F b x w (row-major)
__global__ void k_bw_axpy(Fp f, u32 r, u32 b, u32 w, const u32* __restrict__ Y, const u32* __restrict__ F,
                          u32* __restrict__ U) {
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (u64)r * w) return;
    const u32 g = (u32)(e / w), j = (u32)(e % w);
    u64 acc = U[e];
    for (u32 k = 0; k < b; ++k) {
        const u32 fk = F[k * w + j];
        if (fk) acc += fp_mul(f, fp_reduce32(f, Y[(u64)g * b + k]), fk);
    }
    U[e] = fp_reduce_any(f, acc);
}

// nz[j] = 1 when column j of the r x w block V has a nonzero entry
__global__ void k_bw_nzcols(u32 r, u32 w, const u32* __restrict__ V, u32* __restrict__ nz) {
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (u64)r * w && V[e]) nz[e % w] = 1u;
}

// K[:, j] = V[:, j] for the columns flagged nonzero
__global__ void k_bw_keep(u32 r, u32 w, const u32* __restrict__ V, const u32* __restrict__ nz,
                          u32* __restrict__ K) {
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (u64)r * w && nz[e % w]) K[e] = V[e];
}

void bw_kernel_vectors(Ctx& c, u32 p, const BwCsr& A, u32 b, const u32* Y, u32 w, u32 Dmax, const u32* F, u32 E,
                       u32* K, u32* nzhist, u32* nzcheck) {
    hipStream_t s = c.stream;
    const Fp f = make_fp(p);
    const u64 rw = (u64)A.r * w;
    DBuf<u32> U(&c.pool, std::max<u64>(rw, 1)), V(&c.pool, std::max<u64>(rw, 1)),
        T(&c.pool, std::max<u64>((u64)A.N * w, 1));
    const u32 g = std::max<u32>(1, ceil_div(rw, 256));
    // Horner: U = Y F_Dmax, then U <- B U + Y F_m for m = Dmax - 1 .. 0
    fill_u32(U.ptr, rw, 0, s);
    fill_u32(K, rw, 0, s);
    fill_u32(nzhist, (u64)E * w, 0, s);
    fill_u32(nzcheck, w, 0, s);
    for (u32 mm = Dmax + 1; mm-- > 0;) {
        if (mm != Dmax) {
            bw_apply(c, p, A, w, U.ptr, T.ptr, V.ptr);
            std::swap(U.ptr, V.ptr);
        }
        if (rw) {
            hipLaunchKernelGGL(k_bw_axpy, dim3(g), dim3(256), 0, s, f, A.r, b, w, Y, F + (u64)mm * b * w, U.ptr);
            F4_LAUNCH_CHECK();
        }
    }
    // iterates U, B U, B^2 U, ...: nonzero flags per iterate, nonzero columns kept
    for (u32 e = 0; e < E; ++e) {
        if (rw) {
            hipLaunchKernelGGL(k_bw_nzcols, dim3(g), dim3(256), 0, s, A.r, w, U.ptr, nzhist + (u64)e * w);
            F4_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_bw_keep, dim3(g), dim3(256), 0, s, A.r, w, U.ptr, nzhist + (u64)e * w, K);
            F4_LAUNCH_CHECK();
        }
        if (e + 1 < E) {
            bw_apply(c, p, A, w, U.ptr, T.ptr, V.ptr);
            std::swap(U.ptr, V.ptr);
        }
    }
    // A^T K: zero columns are syzygies
    spmm_run(s, p, A.N, w, A.tptr, A.tidx, A.tval, K, T.ptr);
    if ((u64)A.N * w) {
        hipLaunchKernelGGL(k_bw_nzcols, dim3(ceil_div((u64)A.N * w, 256)), dim3(256), 0, s, A.N, w, T.ptr, nzcheck);
        F4_LAUNCH_CHECK();
    }
}
