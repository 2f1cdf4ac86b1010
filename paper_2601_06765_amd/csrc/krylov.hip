// Block operator application for Krylov solvers over F_p (section "Block
// Wiedemann and Block Lanczos": the hot loop applies the matrix Pi, and often
// its transpose, to a small block of b vectors; the block form turns SpMV into
// SpMM).  Y = A X for a CSR matrix A and a row-major block X of b columns.
// A transposed product runs the same kernel on the transpose's CSR (the CSC
// of A), built once per matrix by a counting sort on the columns.
//
// Layout: a group of G lanes per output row (several rows per wave for small
// b).  The group loads G consecutive stored entries of its row with one
// coalesced access per lane, then broadcasts them inside the group: BP lanes
// per entry, lane k reading VW consecutive words of the gathered row of X
// (BP * VW >= b, VW = 2 for even b), so that the b words form one contiguous
// request, and G / BP entries per
// broadcast step, BP steps per chunk of G entries, unrolled so that the
// gathers of a chunk are in flight together.  Each lane sums the raw 64-bit
// products of its words exactly in 96 bits (a 64-bit sum and a carry count:
// at most 2^32 products of words below 2^32), so no product is reduced; the
// sum is reduced modulo p once per output (stored words and words of X may
// be any 32-bit values: they act as their residues).
#include <mutex>
#include <unordered_map>

#include "internal.hpp"
#include "../../include/f4.h"

#define SPMM_WG 256
#define SPMM_PROJ_MAX 16  // widest block of the fused projection

// Epilogues (EPI) for the Krylov branch, each saving a launch per term:
// SPMM_EPI_PROJ also adds the projection PX^T Y (b x b, PX an nrows x b
// block) into the 64-bit accumulators S64: every output word times the b
// words of its row of PX, each product reduced, summed in LDS per workgroup
// and added with one atomic per entry and workgroup (X^T B^t (B Y) of the
// sequence); SPMM_EPI_ADD adds AY AF to the output (AY nrows x ayb, AF
// ayb x b), the Horner step Y F_m of the kernel vectors; SPMM_EPI_NZKEEP
// flags the output's nonzero columns in NZ (an OR per column and
// workgroup) and copies the columns of the previous iterate KP flagged in
// KNZ into K (the kernel vectors' iterates B^e u).
#define SPMM_EPI_NONE 0
#define SPMM_EPI_PROJ 1
#define SPMM_EPI_ADD 2
#define SPMM_EPI_NZKEEP 3
template <int BP, int G, int VW, int EPI = SPMM_EPI_NONE>
__global__ __launch_bounds__(SPMM_WG) void k_spmm(Fp f, u32 nrows, u32 b, const u32* __restrict__ ptr,
                                                   const u32* __restrict__ idx, const u32* __restrict__ val,
                                                   const u32* __restrict__ X, u32* __restrict__ Y, SpmmEpi ep) {
    constexpr bool PROJ = EPI == SPMM_EPI_PROJ;
    const u32* __restrict__ PX = ep.PX;
    unsigned long long* __restrict__ S64 = ep.S64;
    __shared__ unsigned long long s_pj[PROJ ? SPMM_PROJ_MAX * SPMM_PROJ_MAX : 1];
    __shared__ u32 s_nz[EPI == SPMM_EPI_NZKEEP ? 64 : 1];
    if (PROJ) {
        for (u32 x = threadIdx.x; x < b * b; x += SPMM_WG) s_pj[x] = 0;
        __syncthreads();
    }
    if (EPI == SPMM_EPI_NZKEEP) {
        for (u32 x = threadIdx.x; x < b; x += SPMM_WG) s_nz[x] = 0;
        __syncthreads();
    }
    constexpr u32 SLOTS = G / BP;
    static_assert(G <= F4_WAVE && G % BP == 0 && (VW == 1 || VW == 2), "group layout");
    // workgroups go to the eight XCDs in turn; give each XCD a contiguous range
    // of rows (neighbouring rows gather neighbouring rows of X through the same
    // L2): workgroup w runs logical block x*q + min(x, rem) + w/8, x = w mod 8
    const u32 nb = gridDim.x, q = nb / 8, rem = nb % 8, x = blockIdx.x % 8;
    const u32 lb = x * q + min(x, rem) + blockIdx.x / 8;
    const u64 g = ((u64)lb * SPMM_WG + threadIdx.x) / G;  // output row of the group
    // lane k of an entry covers the VW columns k*VW .. k*VW + VW - 1 (VW = 2
    // needs an even b: a lane's two words are one aligned 8-byte access)
    const u32 gl = threadIdx.x % G, k = (gl % BP) * VW, slot = gl / BP;
    const bool live = g < nrows;
    const u32 e0 = live ? ptr[g] : 0u, e1 = live ? ptr[g + 1] : 0u;
    u64 lo[VW] = {};  // exact sums of this lane's products: hi * 2^64 + lo
    u32 hi[VW] = {};
    // the trip count is the same for every lane of a group, so a group's
    // lanes are active or idle together in the exchanges below; chunk loads
    // run one chunk ahead of the gathers
    u32 cnt = e1 > e0 ? min((u32)G, e1 - e0) : 0u;
    u32 mc = gl < cnt ? idx[e0 + gl] : 0u;
    u32 mv = gl < cnt ? val[e0 + gl] : 0u;
    for (u64 c0 = e0; c0 < e1; c0 += G) {  // 64-bit: c0 + G must not wrap near 2^32 entries
        const u64 c1 = c0 + G;
        const u32 cnt1 = c1 < e1 ? (u32)min((u64)G, e1 - c1) : 0u;
        const u32 nc = gl < cnt1 ? idx[c1 + gl] : 0u;
        const u32 nv = gl < cnt1 ? val[c1 + gl] : 0u;
#pragma unroll
        for (u32 j = 0; j < BP; ++j) {
            const u32 src = j * SLOTS + slot;  // entry of this step for this lane's slot
            const u32 cj = (u32)__shfl((int)mc, (int)src, G);
            const u32 vj = (u32)__shfl((int)mv, (int)src, G);
            if (src < cnt && k < b) {
                u32 xv[VW];
                if (VW == 2) {
                    const uint2 w2 = *reinterpret_cast<const uint2*>(X + (u64)cj * b + k);
                    xv[0] = w2.x;
                    xv[VW - 1] = w2.y;
                } else {
                    xv[0] = X[(u64)cj * b + k];
                }
#pragma unroll
                for (u32 v = 0; v < VW; ++v) {
                    const u64 nl = lo[v] + (u64)vj * xv[v];
                    hi[v] += nl < lo[v] ? 1u : 0u;
                    lo[v] = nl;
                }
            }
        }
        cnt = cnt1;
        mc = nc;
        mv = nv;
    }
    // residue of each lane sum, then the slots of a group (partial sums of
    // the same output columns) are added
    const u32 c64 = fp_reduce(f, (u64)f.r32 * f.r32);  // 2^64 mod p
    u32 out[VW];
#pragma unroll
    for (u32 v = 0; v < VW; ++v) {
        u64 acc = (u64)fp_reduce_any(f, lo[v]) + fp_reduce(f, (u64)fp_reduce32(f, hi[v]) * c64);
#pragma unroll
        for (u32 d = BP; d < G; d <<= 1) acc += (u64)__shfl_xor((unsigned long long)acc, (int)d, G);
        out[v] = fp_reduce_any(f, acc);
    }
    if (EPI == SPMM_EPI_ADD && live && slot == 0 && k < b) {
#pragma unroll
        for (u32 v = 0; v < VW; ++v) {
            if (k + v >= b) continue;
            u64 acc = out[v];
            for (u32 kk = 0; kk < ep.ayb; ++kk) {
                const u32 fk = ep.AF[kk * b + k + v];
                if (fk) acc += fp_mul(f, fp_reduce32(f, ep.AY[g * ep.ayb + kk]), fk);
            }
            out[v] = fp_reduce_any(f, acc);
        }
    }
    if (live && slot == 0 && k < b) {
        if (VW == 2)
            *reinterpret_cast<uint2*>(Y + g * b + k) = make_uint2(out[0], out[VW - 1]);
        else
            Y[g * b + k] = out[0];
        if (PROJ) {
            // entry (kk, l) of the projection: PX[g][kk] Y[g][l]; products
            // below p, at most SPMM_WG of them per entry and workgroup
            for (u32 kk = 0; kk < b; ++kk) {
                const u32 xk = fp_reduce32(f, PX[g * b + kk]);
#pragma unroll
                for (u32 v = 0; v < VW; ++v)
                    if (k + v < b && xk && out[v])
                        atomicAdd(&s_pj[kk * b + k + v], (unsigned long long)fp_mul(f, xk, out[v]));
            }
        }
    }
    if (EPI == SPMM_EPI_NZKEEP && live && slot == 0 && k < b) {
#pragma unroll
        for (u32 v = 0; v < VW; ++v) {
            const u32 col = k + v;
            if (col >= b) continue;
            if (out[v]) s_nz[col] = 1u;  // every writer stores 1
            if (ep.KNZ[col]) ep.K[g * b + col] = ep.KP[g * b + col];
        }
    }
    if (PROJ) {
        __syncthreads();
        for (u32 x = threadIdx.x; x < b * b; x += SPMM_WG)
            if (s_pj[x]) atomicAdd(&S64[x], s_pj[x]);
    }
    if (EPI == SPMM_EPI_NZKEEP) {
        __syncthreads();
        for (u32 x = threadIdx.x; x < b; x += SPMM_WG)
            if (s_nz[x]) atomicOr(&ep.NZ[x], 1u);
    }
}

template <int BP, int G, int VW>
static void spmm_launch(hipStream_t s, const Fp& f, u32 nrows, u32 b, const u32* ptr, const u32* idx, const u32* val,
                        const u32* X, u32* Y, const SpmmEpi& ep) {
    const u32 grid = ceil_div((u64)nrows * G, SPMM_WG);
    if (ep.PX)
        hipLaunchKernelGGL((k_spmm<BP, G, VW, SPMM_EPI_PROJ>), dim3(grid), dim3(SPMM_WG), 0, s, f, nrows, b, ptr, idx,
                           val, X, Y, ep);
    else if (ep.AY)
        hipLaunchKernelGGL((k_spmm<BP, G, VW, SPMM_EPI_ADD>), dim3(grid), dim3(SPMM_WG), 0, s, f, nrows, b, ptr, idx,
                           val, X, Y, ep);
    else if (ep.NZ)
        hipLaunchKernelGGL((k_spmm<BP, G, VW, SPMM_EPI_NZKEEP>), dim3(grid), dim3(SPMM_WG), 0, s, f, nrows, b, ptr,
                           idx, val, X, Y, ep);
    else
        hipLaunchKernelGGL((k_spmm<BP, G, VW>), dim3(grid), dim3(SPMM_WG), 0, s, f, nrows, b, ptr, idx, val, X, Y, ep);
    F4_LAUNCH_CHECK();
}

void spmm_run(hipStream_t s, u32 p, u32 nrows, u32 b, const u32* ptr, const u32* idx, const u32* val, const u32* X,
              u32* Y, const SpmmEpi& ep) {
    if (nrows == 0) return;
    if (ep.PX && b > SPMM_PROJ_MAX) throw F4Error{1, "projection wider than the fused form"};
    if (ep.NZ && b > 64) throw F4Error{1, "flagged block wider than the fused form"};
    const Fp f = make_fp(p);
    // two words per lane: an even b, and X and Y 8-byte aligned (caller
    // blocks need not be; then one word per lane)
    if (b % 2 == 0 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 7) == 0) {
        if (b <= 2)
            spmm_launch<1, 8, 2>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
        else if (b <= 4)
            spmm_launch<2, 8, 2>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
        else if (b <= 8)
            spmm_launch<4, 8, 2>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
        else if (b <= 16)
            spmm_launch<8, 8, 2>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
        else if (b <= 32)
            spmm_launch<16, 16, 2>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
        else
            spmm_launch<32, 32, 2>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
        return;
    }
    if (b <= 1)
        spmm_launch<1, 8, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
    else if (b <= 2)
        spmm_launch<2, 8, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
    else if (b <= 4)
        spmm_launch<4, 8, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
    else if (b <= 8)
        spmm_launch<8, 8, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
    else if (b <= 16)
        spmm_launch<16, 16, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
    else if (b <= 32)
        spmm_launch<32, 32, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
    else
        spmm_launch<64, 64, 1>(s, f, nrows, b, ptr, idx, val, X, Y, ep);
}

// ------------------------------------------------------------ transpose
__global__ void k_col_count(const u32* __restrict__ idx, u64 nnz, u32* __restrict__ cnt) {
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[idx[e]], 1u);
}

// one thread per row of A: its entries go to the next free places of their
// columns (the order inside a column is not fixed; sums over it are exact)
__global__ void k_col_scatter(const u32* __restrict__ ptr, u32 nrows, const u32* __restrict__ idx,
                              const u32* __restrict__ val, u32* __restrict__ cur, u32* __restrict__ tidx,
                              u32* __restrict__ tval) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (u32 e = ptr[i]; e < ptr[i + 1]; ++e) {
        const u32 pos = atomicAdd(&cur[idx[e]], 1u);
        tidx[pos] = i;
        tval[pos] = val[e];
    }
}

u64 csr_transpose_ws_words(u32 ncols) { return (u64)ncols + 1 + exclusive_scan_ws_words(ncols); }

void csr_transpose_into(hipStream_t s, u32 nrows, u32 ncols, u64 nnz, const u32* ptr, const u32* idx,
                        const u32* val, u32* tptr, u32* tidx, u32* tval, u32* ws) {
    u32* cnt = ws;  // ncols + 1 counters, then the scan's workspace
    fill_u32(cnt, (u64)ncols + 1, 0, s);
    if (nnz) {
        hipLaunchKernelGGL(k_col_count, dim3(ceil_div(nnz, 256)), dim3(256), 0, s, idx, nnz, cnt);
        F4_LAUNCH_CHECK();
    }
    exclusive_scan_u32_ws(cnt, tptr, ncols, ws + (u64)ncols + 1, s);
    if (nnz && nrows) {
        F4_HIP_TRY(hipMemcpyAsync(cnt, tptr, (u64)ncols * 4, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_col_scatter, dim3(ceil_div(nrows, 256)), dim3(256), 0, s, ptr, nrows, idx, val, cnt,
                           tidx, tval);
        F4_LAUNCH_CHECK();
    }
}

void csr_transpose(Ctx& c, u32 nrows, u32 ncols, u64 nnz, const u32* ptr, const u32* idx, const u32* val,
                   DBuf<u32>& tptr, DBuf<u32>& tidx, DBuf<u32>& tval) {
    tptr.reset(&c.pool, (u64)ncols + 1);
    tidx.reset(&c.pool, std::max<u64>(nnz, 1));
    tval.reset(&c.pool, std::max<u64>(nnz, 1));
    DBuf<u32> ws(&c.pool, csr_transpose_ws_words(ncols));
    csr_transpose_into(c.stream, nrows, ncols, nnz, ptr, idx, val, tptr.ptr, tidx.ptr, tval.ptr, ws.ptr);
}

// ------------------------------------------------- allocation-free products
// Scratch of f4_spmm_noalloc: the transpose's CSR (column pointers, row
// indices, values) and the counting sort's workspace, in one file-scope
// device array that each GPU holds until the process ends.  In host code the
// array's name is only a stand-in symbol, never a device address: the
// address every launch uses is the one hipGetSymbolAddress returns, looked up
// once per device (with that device current) when a context is created there.
static __device__ __align__(256) u32 scratch[F4_NOALLOC_SCRATCH_BYTES / 4];
static std::mutex scratch_mu;
static std::unordered_map<int, u32*> scratch_at;  // device -> address of its copy

void noalloc_scratch_init(int device) {
    std::lock_guard<std::mutex> g(scratch_mu);
    if (scratch_at.count(device)) return;
    void* ptr = nullptr;
    F4_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw F4Error{F4_E_DEVICE, "no device address for the scratch array"};
    scratch_at[device] = static_cast<u32*>(ptr);
}

static u32* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> g(scratch_mu);
    auto it = scratch_at.find(device);
    return it == scratch_at.end() ? nullptr : it->second;
}

u64 spmm_noalloc_words(u32 ncols, u64 nnz, int trans) {
    if (!trans) return 0;
    // tptr (ncols + 1, rounded to 64 words), tidx, tval, then the workspace
    return ((u64)ncols + 1 + 63) / 64 * 64 + 2 * nnz + csr_transpose_ws_words(ncols);
}

void spmm_noalloc_run(hipStream_t s, int device, u32 p, u32 nrows, u32 ncols, u64 nnz, const u32* ptr,
                      const u32* idx, const u32* val, int trans, u32 b, const u32* X, u32* Y) {
    if (!trans) {
        spmm_run(s, p, nrows, b, ptr, idx, val, X, Y);
        return;
    }
    u32* base = noalloc_scratch(device);
    if (!base) throw F4Error{F4_E_STATE, "scratch of this device not set up"};
    if (spmm_noalloc_words(ncols, nnz, trans) * 4 > F4_NOALLOC_SCRATCH_BYTES)
        throw F4Error{F4_E_RANGE, "transpose does not fit the scratch array"};
    u32* tptr = base;
    u32* tidx = tptr + ((u64)ncols + 1 + 63) / 64 * 64;
    u32* tval = tidx + nnz;
    u32* ws = tval + nnz;
    csr_transpose_into(s, nrows, ncols, nnz, ptr, idx, val, tptr, tidx, tval, ws);
    spmm_run(s, p, ncols, b, tptr, tidx, tval, X, Y);
}
