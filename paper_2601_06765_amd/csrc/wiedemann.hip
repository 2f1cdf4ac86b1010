// Block Wiedemann over F_p for left-kernel vectors of a Macaulay matrix
// (section "Block Wiedemann and Block Lanczos": kernel vectors by black-box
// linear algebra; Remark "Syzygies, revisited": v^T A = 0 is a syzygy among
// the shifted reducers by Proposition "Kernel equals syzygies under
// dictionary closure").  The square operator is B = A D A^T (D a diagonal of
// nonzero elements); every step below runs on the device:
//   1. the projected block Krylov sequence S_t = X^T B^t (B Y): two block
//      operator applications per term (k_spmm on A^T with D folded into its
//      values, then on A with the projection X^T Z added by the same launch);
//   2. the generator: an M-Basis sigma-basis of [S(x)^T ; -I_b] (one wave's
//      fraction-free elimination of the residuals at the current order in the
//      order of (shift, index), then the row operations and the
//      multiplication of pivot rows by x applied to every coefficient of the
//      basis P and of the residual series R = P [S^T ; -I], whose next
//      coefficient is the next order's residual), one order per pass;
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

__global__ void k_bw_reduce64(Fp f, u64 n, const unsigned long long* __restrict__ in, u32* __restrict__ out) {
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fp_reduce_any(f, in[i]);
}

static void bw_apply(Ctx& c, u32 p, const BwCsr& A, u32 w, const u32* V, u32* U, u32* Out,
                     const SpmmEpi& ep = SpmmEpi()) {
    // Out = A (D (A^T V)): U is N x w scratch; the epilogue (a projection of
    // Out, or an added block) runs in the second product
    spmm_run(c.stream, p, A.N, w, A.tptr, A.tidx, A.tval_d, V, U);
    spmm_run(c.stream, p, A.r, w, A.ptr, A.idx, A.val, U, Out, ep);
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
    // term t: Z = B^(t+1) Y, its projection X^T Z formed by the second block
    // product of the term (two launches per term)
    SpmmEpi ep;
    ep.PX = X;
    if (L) {
        ep.S64 = (unsigned long long*)S64.ptr;
        bw_apply(c, p, A, b, Y, U.ptr, Z.ptr, ep);
    }
    for (u32 t = 1; t < L; ++t) {
        ep.S64 = (unsigned long long*)S64.ptr + (u64)t * b * b;
        bw_apply(c, p, A, b, Z.ptr, U.ptr, Z2.ptr, ep);
        std::swap(Z.ptr, Z2.ptr);
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

// R = P F for P = I, F = [S(x)^T ; -I]: R[i][c] = sum_t S_t[c][i] x^t for
// i < b, R[b + c][c] = -1; coefficient l of R[i][c] at R[(i b + c) W + l],
// l < W (coefficients of x^L and above are never read)
__global__ void k_mb_init_r(Fp f, u32 b, u32 W, u32 L, const u32* __restrict__ S, u32* __restrict__ R) {
    const u32 m = 2 * b;
    const u64 total = (u64)m * b * W;
    for (u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (u64)gridDim.x * blockDim.x) {
        const u32 l = (u32)(e % W), ic = (u32)(e / W), i = ic / b, c = ic % b;
        u32 v = 0;
        if (i < b)
            v = l < L ? S[((u64)l * b + c) * b + i] : 0u;
        else
            v = (l == 0 && i - b == c) ? f.p - 1 : 0u;
        R[e] = v;
    }
}

// The elimination of the residual rows (coefficient k of R) in the order of
// (shift, index), fraction-free (row_j <- piv row_j - D_j[c] row_i for the
// rows j after the pivot row i with D_j[c] != 0, c the pivot row's first
// nonzero column).  One workgroup: per pivot step every (row, entry) of the
// rows after the pivot row is a thread of its own (entries of D, then of the
// row transform).  Writes the row transform T (m x m, applied to P as
// P' = T P), the pivot flags and the new shifts (+1 for pivot rows).
#define MB_ELIM_THREADS 512
__global__ __launch_bounds__(MB_ELIM_THREADS) void k_mb_elim(Fp f, u32 b, const u32* __restrict__ R, u32 W, u32 k,
                                                             const u32* __restrict__ shifts_in,
                                                             u32* __restrict__ shifts_out, u32* __restrict__ T,
                                                             u32* __restrict__ piv) {
    __shared__ u32 s_D[32][16];
    __shared__ u32 s_T[32][32];
    __shared__ u32 s_order[32];
    __shared__ u32 s_f[32];  // the pivot column's entry of every row, read before the step's updates
    __shared__ u32 s_c, s_pv, s_i;
    const u32 m = 2 * b, tid = threadIdx.x, e = b + m;  // e: entries of a row (D, then T)
    for (u32 x = tid; x < m * b; x += MB_ELIM_THREADS) s_D[x / b][x % b] = R[(u64)x * W + k];  // residuals at order k
    for (u32 x = tid; x < m * m; x += MB_ELIM_THREADS) s_T[x / m][x % m] = (x / m == x % m) ? 1u : 0u;
    u32 si = 0;
    if (tid < m) {
        si = shifts_in[tid];
        u32 rank = 0;  // position in the order of (shift, index)
        for (u32 j = 0; j < m; ++j) {
            const u32 sj = shifts_in[j];
            rank += (sj < si || (sj == si && j < tid)) ? 1u : 0u;
        }
        s_order[rank] = tid;
    }
    __syncthreads();
    u32 pivmask = 0;  // kept by thread 0
    for (u32 a = 0; a < m; ++a) {
        if (tid < F4_WAVE) {  // wave 0: the pivot column of row order[a]
            const u32 i = s_order[a];
            const u64 nzc = __ballot(tid < b && s_D[i][tid] != 0);
            if (tid == 0) {
                s_i = i;
                s_c = nzc ? (u32)(__ffsll((long long)nzc) - 1) : 0xffffffffu;
                s_pv = nzc ? s_D[i][s_c] : 0u;
                if (nzc) pivmask |= 1u << i;
            }
        }
        __syncthreads();
        const u32 c = s_c, i = s_i, pv = s_pv;
        if (c != 0xffffffffu && tid < m) s_f[tid] = s_D[tid][c];
        __syncthreads();  // every thread has read this step's s_c before wave 0 writes the next
        if (c == 0xffffffffu) continue;  // the same in every thread: no pivot in this row
        for (u32 x = tid; x < (m - 1 - a) * e; x += MB_ELIM_THREADS) {
            const u32 j = s_order[a + 1 + x / e], y = x % e, fj = s_f[j];
            if (!fj) continue;
            u32* el = y < b ? &s_D[j][y] : &s_T[j][y - b];
            const u32 src = y < b ? s_D[i][y] : s_T[i][y - b];
            *el = fp_reduce(f, (u64)fp_mul(f, pv, *el) + (f.p - fp_mul(f, fj, src)));
        }
        __syncthreads();
    }
    for (u32 x = tid; x < m * m; x += MB_ELIM_THREADS) T[x] = s_T[x / m][x % m];
    __shared__ u32 s_pm;
    if (tid == 0) s_pm = pivmask;
    __syncthreads();
    if (tid < m) {
        const u32 pvf = (s_pm >> tid) & 1u;
        piv[tid] = pvf;
        shifts_out[tid] = si + pvf;
    }
}

// P'[i][j][l] = sum_q T[i][q] P[q][j][l'] with l' = l - 1 for pivot rows i
// (multiplication by x) and l' = l otherwise, for l < lcount (higher
// coefficients are zero in both buffers); the same for the residual series,
// R'[i][c][l] for k < l < L (the coefficients still to be read)
__global__ __launch_bounds__(256) void k_mb_apply(Fp f, u32 b, u32 W, u32 lcount, u32 k, u32 L,
                                                  const u32* __restrict__ Pin, u32* __restrict__ Pout,
                                                  const u32* __restrict__ Rin, u32* __restrict__ Rout,
                                                  const u32* __restrict__ T, const u32* __restrict__ piv) {
    __shared__ u32 s_T[32 * 32];
    __shared__ u32 s_piv[32];
    const u32 m = 2 * b, tid = threadIdx.x;
    for (u32 x = tid; x < m * m; x += 256) s_T[x] = T[x];
    if (tid < m) s_piv[tid] = piv[tid];
    __syncthreads();
    const u64 e = (u64)blockIdx.x * 256 + tid;
    const u64 totalP = (u64)m * m * lcount;
    const u32 rcount = L > k + 1 ? L - k - 1 : 0u;
    const u64 totalR = (u64)m * b * rcount;
    if (e >= totalP + totalR) return;
    const bool isP = e < totalP;
    const u64 x = isP ? e : e - totalP;
    const u32 span = isP ? lcount : rcount, ncol = isP ? m : b;
    const u32 l = isP ? (u32)(x % span) : k + 1 + (u32)(x % span);
    const u32 ij = (u32)(x / span), i = ij / ncol, j = ij % ncol;
    const u32* in = isP ? Pin : Rin;
    u32 v = 0;
    if (!(s_piv[i] && l == 0)) {
        const u32 ls = s_piv[i] ? l - 1 : l;
        u64 acc = 0;
        for (u32 q = 0; q < m; ++q) {
            const u32 t = s_T[i * m + q];
            if (t) acc += fp_mul(f, t, in[((u64)q * ncol + j) * W + ls]);
        }
        v = fp_reduce_any(f, acc);
    }
    (isP ? Pout : Rout)[((u64)i * ncol + j) * W + l] = v;
}

__global__ void k_bw_identity(u32 m, u32 W, u32* P) {
    for (u32 i = threadIdx.x; i < m; i += blockDim.x) P[((u64)i * m + i) * W] = 1u;
}

void bw_mbasis(Ctx& c, u32 p, u32 b, u32 L, const u32* S, u32* P, u32* shifts) {
    hipStream_t s = c.stream;
    const Fp f = make_fp(p);
    const u32 m = 2 * b, W = L + 2;
    const u64 psize = (u64)m * m * W, rsize = (u64)m * b * W;
    DBuf<u32> P2(&c.pool, psize), R1(&c.pool, rsize), R2(&c.pool, rsize), T(&c.pool, (u64)m * m), piv(&c.pool, m),
        sh2(&c.pool, m);
    fill_u32(P, psize, 0, s);
    fill_u32(P2.ptr, psize, 0, s);
    // P = I, shifts (0^b, 1^b), R = F
    std::vector<u32> hs(m);
    for (u32 i = 0; i < m; ++i) hs[i] = i < b ? 0u : 1u;
    upload(c, shifts, hs.data(), m * 4);
    hipLaunchKernelGGL(k_bw_identity, dim3(1), dim3(64), 0, s, m, W, P);
    F4_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mb_init_r, dim3(std::max<u32>(1, std::min<u32>(1024, ceil_div(rsize, 256)))), dim3(256), 0, s,
                       f, b, W, L, S, R1.ptr);
    F4_LAUNCH_CHECK();
    u32* cur = P;
    u32* nxt = P2.ptr;
    u32* rcur = R1.ptr;
    u32* rnxt = R2.ptr;
    u32* scur = shifts;
    u32* snxt = sh2.ptr;
    for (u32 k = 0; k < L; ++k) {
        hipLaunchKernelGGL(k_mb_elim, dim3(1), dim3(MB_ELIM_THREADS), 0, s, f, b, rcur, W, k, scur, snxt, T.ptr,
                           piv.ptr);
        F4_LAUNCH_CHECK();
        // degrees after this order are at most k + 2
        const u32 lcount = std::min(W, k + 3);
        const u64 total = (u64)m * m * lcount + (u64)m * b * (L > k + 1 ? L - k - 1 : 0u);
        hipLaunchKernelGGL(k_mb_apply, dim3(ceil_div(total, 256)), dim3(256), 0, s, f, b, W, lcount, k, L, cur, nxt,
                           rcur, rnxt, T.ptr, piv.ptr);
        F4_LAUNCH_CHECK();
        std::swap(cur, nxt);
        std::swap(rcur, rnxt);
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
    if (rw) {
        hipLaunchKernelGGL(k_bw_axpy, dim3(g), dim3(256), 0, s, f, A.r, b, w, Y, F + (u64)Dmax * b * w, U.ptr);
        F4_LAUNCH_CHECK();
    }
    for (u32 mm = Dmax; mm-- > 0;) {
        // U <- B U + Y F_m: the addition is the second product's epilogue
        SpmmEpi ep;
        ep.AY = Y;
        ep.AF = F + (u64)mm * b * w;
        ep.ayb = b;
        bw_apply(c, p, A, w, U.ptr, T.ptr, V.ptr, ep);
        std::swap(U.ptr, V.ptr);
    }
    // iterates U, B U, B^2 U, ...: nonzero flags per iterate, nonzero columns
    // kept.  The product that forms iterate e + 1 also flags its nonzero
    // columns and keeps the nonzero columns of iterate e (its input, whose
    // flags are complete), so an iterate costs the two products alone.
    if (rw && E) {
        hipLaunchKernelGGL(k_bw_nzcols, dim3(g), dim3(256), 0, s, A.r, w, U.ptr, nzhist);
        F4_LAUNCH_CHECK();
    }
    for (u32 e = 0; e + 1 < E; ++e) {
        SpmmEpi ep;
        ep.NZ = nzhist + (u64)(e + 1) * w;
        ep.KP = U.ptr;
        ep.KNZ = nzhist + (u64)e * w;
        ep.K = K;
        bw_apply(c, p, A, w, U.ptr, T.ptr, V.ptr, ep);
        std::swap(U.ptr, V.ptr);
    }
    if (rw && E) {
        hipLaunchKernelGGL(k_bw_keep, dim3(g), dim3(256), 0, s, A.r, w, U.ptr, nzhist + (u64)(E - 1) * w, K);
        F4_LAUNCH_CHECK();
    }
    // A^T K: zero columns are syzygies
    spmm_run(s, p, A.N, w, A.tptr, A.tidx, A.tval, K, T.ptr);
    if ((u64)A.N * w) {
        hipLaunchKernelGGL(k_bw_nzcols, dim3(ceil_div((u64)A.N * w, 256)), dim3(256), 0, s, A.N, w, T.ptr, nzcheck);
        F4_LAUNCH_CHECK();
    }
}
