// Symbolic preprocessing of an explicit row list with two-word monomial keys
// (section "Monomial keys": multiword keys; Algorithm "FBSP" without the
// closure; Definition "Sparse Macaulay matrix for a batch").  Pipeline:
//   check every row (k in range, t a monomial, t * LM(g_k) without overflow),
//   scan the row lengths (term offsets),
//   fill: every term's shifted monomial as its complemented order key (so an
//     ascending sort gives descending grevlex), two words per term,
//   sort the 128-bit keys: a stable radix sort on the low words, then a
//     stable radix sort of the high words in that order (LSD over the pair),
//   unique + join: run heads, their exclusive scan gives every term its
//     column, the heads give the dictionary,
//   rows: (column of the leading term, k) sorted, repeats dropped,
//   CSR: the rows' lengths scanned, columns and coefficients copied.
#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "mw.hpp"

#define MW_SLOTS 64  // copies of the check's words (spread atomics)

struct MwRow {  // the record of f4_rowspec_mw
    u64 t0, t1;
    u32 k, pad;
};

__global__ void k_mw_check(const MwRow* __restrict__ R, u32 r, MwLayout L, const u64* __restrict__ lm,
                           const u32* __restrict__ len, u32 npolys, u32* __restrict__ rowlen, u32* __restrict__ info) {
    u32 err = 0, dmax = 0;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < r; q += gridDim.x * blockDim.x) {
        const MwRow x = R[q];
        u32 l = 0;
        if (x.k >= npolys || !mw_valid(L, x.t0, x.t1)) {
            err |= 1;
        } else if (mw_mul_overflows(L, x.t0, x.t1, lm[2 * x.k], lm[2 * x.k + 1])) {
            err |= 2;
        } else {
            l = len[x.k];
            dmax = max(dmax, mw_deg(x.t0) + mw_deg(lm[2 * x.k]));
        }
        rowlen[q] = l;
    }
    for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) {
        err |= (u32)__shfl_xor((int)err, (int)d, F4_WAVE);
        dmax = max(dmax, (u32)__shfl_xor((int)dmax, (int)d, F4_WAVE));
    }
    if (lane_id() == 0) {
        u32* I = info + 4 * (blockIdx.x % MW_SLOTS);
        if (err) atomicOr(&I[0], err);
        if (dmax) atomicMax(&I[1], dmax);
    }
}

// one wave per row, lanes over its terms: the complemented order key of
// t * m for every term m of g_k, high and low words, and the term's index
__global__ void k_mw_fill(const MwRow* __restrict__ R, u32 r, MwLayout L, const u32* __restrict__ toff,
                          const u64* __restrict__ mon, const u64* __restrict__ off, const u32* __restrict__ len,
                          u64* __restrict__ khi, u64* __restrict__ klo, u64* __restrict__ klo_copy,
                          u32* __restrict__ idx) {
    const u32 lane = lane_id();
    const u32 waves = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 q = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; q < r; q += waves) {
        const MwRow x = R[q];
        const u32 base = toff[q];
        const u32 l = toff[q + 1] - base;  // 0 for rejected rows (the check stops the call then)
        const u64 o = l ? off[x.k] : 0;
        for (u32 j = lane; j < l; j += F4_WAVE) {
            const u64 m0 = x.t0 + mon[2 * (o + j)], m1 = x.t1 + mon[2 * (o + j) + 1];
            const u64 c0 = ~(m0 ^ L.lanes0), c1 = ~(m1 ^ L.lanes1);
            khi[base + j] = c0;
            klo[base + j] = c1;
            klo_copy[base + j] = c1;
            idx[base + j] = base + j;
        }
    }
}

// high words in the order of the first sort
__global__ void k_mw_gather(const u64* __restrict__ khi, const u32* __restrict__ idx, u64 nnz, u64* __restrict__ out) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (u64)gridDim.x * blockDim.x)
        out[i] = khi[idx[i]];
}

// run heads of the sorted keys
__global__ void k_mw_heads(const u64* __restrict__ hi, const u32* __restrict__ idx, const u64* __restrict__ lo_by_term,
                           u64 nnz, u32* __restrict__ head) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (u64)gridDim.x * blockDim.x)
        head[i] = (i == 0 || hi[i] != hi[i - 1] || lo_by_term[idx[i]] != lo_by_term[idx[i - 1]]) ? 1u : 0u;
}

// every term's column, the dictionary (monomials, two words, descending
// grevlex) and its size
__global__ void k_mw_join(const u64* __restrict__ hi, const u32* __restrict__ idx, const u64* __restrict__ lo_by_term,
                          const u32* __restrict__ head, const u32* __restrict__ pos, u64 nnz, MwLayout L,
                          u32* __restrict__ colterm, u64* __restrict__ dict, u32* __restrict__ N) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (u64)gridDim.x * blockDim.x) {
        const u32 col = pos[i] + head[i] - 1;
        colterm[idx[i]] = col;
        if (head[i]) {
            dict[2 * (u64)col] = ~hi[i] ^ L.lanes0;
            dict[2 * (u64)col + 1] = ~lo_by_term[idx[i]] ^ L.lanes1;
        }
        if (i == nnz - 1) *N = col + 1;
    }
}

// row order key: column of the leading term (the first), then k
__global__ void k_mw_rowkeys(const MwRow* __restrict__ R, u32 r, const u32* __restrict__ toff,
                             const u32* __restrict__ colterm, u32 kbits, u64* __restrict__ keys, u32* __restrict__ vals) {
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < r; q += gridDim.x * blockDim.x) {
        keys[q] = ((u64)colterm[toff[q]] << kbits) | R[q].k;
        vals[q] = q;
    }
}

__global__ void k_mw_rowheads(const u64* __restrict__ keys, u32 r, const u32* __restrict__ vals,
                              const u32* __restrict__ toff, u32* __restrict__ head, u32* __restrict__ lens) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        const bool h = i == 0 || keys[i] != keys[i - 1];
        head[i] = h ? 1u : 0u;
        lens[i] = h ? toff[vals[i] + 1] - toff[vals[i]] : 0u;
    }
}

// distinct rows in order: their source rows and lengths
__global__ void k_mw_rowpick(const u32* __restrict__ head, const u32* __restrict__ hpos, const u32* __restrict__ vals,
                             const u32* __restrict__ lens, u32 r, u32* __restrict__ src, u32* __restrict__ olen) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x)
        if (head[i]) {
            src[hpos[i]] = vals[i];
            olen[hpos[i]] = lens[i];
        }
}

// one wave per output row: columns, coefficients, row metadata
__global__ void k_mw_csr(const MwRow* __restrict__ R, const u32* __restrict__ src, u32 ro,
                         const u32* __restrict__ rptr, const u32* __restrict__ toff, const u32* __restrict__ colterm,
                         const u32* __restrict__ coeff, const u64* __restrict__ off, u32* __restrict__ col_ind,
                         u32* __restrict__ val, u64* __restrict__ row_t, u32* __restrict__ row_k) {
    const u32 lane = lane_id();
    const u32 waves = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 i = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; i < ro; i += waves) {
        const u32 q = src[i];
        const MwRow x = R[q];
        const u32 b = rptr[i], l = rptr[i + 1] - b, tb = toff[q];
        const u64 o = off[x.k];
        for (u32 j = lane; j < l; j += F4_WAVE) {
            col_ind[b + j] = colterm[tb + j];
            val[b + j] = coeff[o + j];
        }
        if (lane == 0) {
            row_t[2 * (u64)i] = x.t0;
            row_t[2 * (u64)i + 1] = x.t1;
            row_k[i] = x.k;
        }
    }
}

static u32 mw_bits(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

void build_rows_mw(Ctx& c, u32 n, u32 npolys, const u64* mon_h, const u32* coeff_h, const u64* off_h,
                   const void* rows_h, u32 r, Matrix& out) {
    hipStream_t s = c.stream;
    const MwLayout L = mw_layout(n);
    const u64 nt = off_h[npolys];
    {
        // the term offsets are 32-bit: every row is at most the longest polynomial
        u64 lmax = 0;
        for (u32 k = 0; k < npolys; ++k) lmax = std::max<u64>(lmax, off_h[k + 1] - off_h[k]);
        if ((u64)r * lmax >= (1ull << 32)) throw F4Error{2, "2^32 or more nonzeros"};
    }
    // the basis on the device, with leading monomials and lengths
    std::vector<u64> lm(2 * (size_t)npolys);
    std::vector<u32> len(npolys);
    for (u32 k = 0; k < npolys; ++k) {
        lm[2 * k] = mon_h[2 * off_h[k]];
        lm[2 * k + 1] = mon_h[2 * off_h[k] + 1];
        len[k] = (u32)(off_h[k + 1] - off_h[k]);
    }
    DBuf<u64> dmon(&c.pool, std::max<u64>(2 * nt, 1)), doff(&c.pool, (u64)npolys + 1),
        dlm(&c.pool, std::max<u64>(2 * (u64)npolys, 1));
    DBuf<u32> dcoeff(&c.pool, std::max<u64>(nt, 1)), dlen(&c.pool, std::max<u32>(npolys, 1));
    upload(c, dmon.ptr, mon_h, 2 * nt * 8);
    upload(c, dcoeff.ptr, coeff_h, nt * 4);
    upload(c, doff.ptr, off_h, ((u64)npolys + 1) * 8);
    upload(c, dlm.ptr, lm.data(), lm.size() * 8);
    upload(c, dlen.ptr, len.data(), len.size() * 4);
    DBuf<u8> dR(&c.pool, (u64)r * sizeof(MwRow));
    upload(c, dR.ptr, rows_h, (u64)r * sizeof(MwRow));
    const MwRow* R = (const MwRow*)dR.ptr;
    // checks and row lengths
    DBuf<u32> rowlen(&c.pool, (u64)r + 1), toff(&c.pool, (u64)r + 1), info(&c.pool, 4 * MW_SLOTS);
    fill_u32(info.ptr, 4 * MW_SLOTS, 0, s);
    fill_u32(rowlen.ptr + r, 1, 0, s);
    const u32 grid = std::min<u32>(4096, ceil_div(r, 256));
    hipLaunchKernelGGL(k_mw_check, dim3(grid), dim3(256), 0, s, R, r, L, dlm.ptr, dlen.ptr, npolys, rowlen.ptr,
                       info.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(rowlen.ptr, toff.ptr, (u64)r + 1, c.pool, s);
    u32 slots[4 * MW_SLOTS];
    readback(c, slots, info.ptr, sizeof(slots));
    u32 err = 0, dmax = 0;
    for (int q = 0; q < MW_SLOTS; ++q) {
        err |= slots[4 * q];
        dmax = std::max(dmax, slots[4 * q + 1]);
    }
    if (err & 1) throw F4Error{1, "row basis index out of range or shift not a monomial"};
    if (err & 2) throw F4Error{2, "exponent lane overflow"};
    u32 nnz32 = 0;
    readback(c, &nnz32, toff.ptr + r, 4);
    const u64 nnz = nnz32;
    // fill, sort (low words, then high words), unique + join
    DBuf<u64> khi(&c.pool, std::max<u64>(nnz, 1)), klo(&c.pool, std::max<u64>(nnz, 1)),
        klo_copy(&c.pool, std::max<u64>(nnz, 1)), hs(&c.pool, std::max<u64>(nnz, 1));
    DBuf<u32> idx(&c.pool, std::max<u64>(nnz, 1));
    const u32 wgrid = std::min<u32>(8192, ceil_div(r, 4));
    hipLaunchKernelGGL(k_mw_fill, dim3(wgrid), dim3(256), 0, s, R, r, L, toff.ptr, dmon.ptr, doff.ptr, dlen.ptr,
                       khi.ptr, klo.ptr, klo_copy.ptr, idx.ptr);
    F4_LAUNCH_CHECK();
    // bits that vary: the low word's lanes (all ones after complementing
    // elsewhere), the high word's degree byte and lanes
    const u32 lo_lo = L.lanes1 ? (u32)__builtin_ctzll(L.lanes1) : 64, hi_lo = (u32)__builtin_ctzll(L.lanes0);
    if (lo_lo < 64) radix_sort_pairs(klo.ptr, idx.ptr, nnz, lo_lo, 64, c.pool, s);
    const u32 egrid = std::min<u32>(8192, ceil_div(nnz, 256));
    hipLaunchKernelGGL(k_mw_gather, dim3(egrid), dim3(256), 0, s, khi.ptr, idx.ptr, nnz, hs.ptr);
    F4_LAUNCH_CHECK();
    radix_sort_pairs(hs.ptr, idx.ptr, nnz, hi_lo, 64, c.pool, s);
    DBuf<u32> head(&c.pool, std::max<u64>(nnz, 1)), pos(&c.pool, std::max<u64>(nnz, 1)),
        colterm(&c.pool, std::max<u64>(nnz, 1)), dN(&c.pool, 1);
    hipLaunchKernelGGL(k_mw_heads, dim3(egrid), dim3(256), 0, s, hs.ptr, idx.ptr, klo_copy.ptr, nnz, head.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(head.ptr, pos.ptr, nnz, c.pool, s);
    DBuf<u64> dict(&c.pool, std::max<u64>(2 * nnz, 2));
    hipLaunchKernelGGL(k_mw_join, dim3(egrid), dim3(256), 0, s, hs.ptr, idx.ptr, klo_copy.ptr, head.ptr, pos.ptr,
                       nnz, L, colterm.ptr, dict.ptr, dN.ptr);
    F4_LAUNCH_CHECK();
    u32 N = 0;
    readback(c, &N, dN.ptr, 4);
    // rows: (column of the leading term, k), sorted, repeats dropped
    const u32 kbits = std::max<u32>(1, mw_bits(npolys - 1));
    const u32 cbits = std::max<u32>(1, mw_bits(N - 1));
    if (kbits + cbits > 64) throw F4Error{2, "row key does not fit 64 bits"};
    DBuf<u64> rkeys(&c.pool, r);
    DBuf<u32> rvals(&c.pool, r), rhead(&c.pool, (u64)r + 1), rpos(&c.pool, (u64)r + 1), rlens(&c.pool, (u64)r + 1);
    hipLaunchKernelGGL(k_mw_rowkeys, dim3(grid), dim3(256), 0, s, R, r, toff.ptr, colterm.ptr, kbits, rkeys.ptr,
                       rvals.ptr);
    F4_LAUNCH_CHECK();
    radix_sort_pairs(rkeys.ptr, rvals.ptr, r, 0, kbits + cbits, c.pool, s);
    hipLaunchKernelGGL(k_mw_rowheads, dim3(grid), dim3(256), 0, s, rkeys.ptr, r, rvals.ptr, toff.ptr, rhead.ptr,
                       rlens.ptr);
    F4_LAUNCH_CHECK();
    fill_u32(rhead.ptr + r, 1, 0, s);
    exclusive_scan_u32(rhead.ptr, rpos.ptr, (u64)r + 1, c.pool, s);
    u32 ro = 0;
    readback(c, &ro, rpos.ptr + r, 4);
    DBuf<u32> src(&c.pool, std::max<u32>(ro, 1)), olen(&c.pool, (u64)ro + 1);
    hipLaunchKernelGGL(k_mw_rowpick, dim3(grid), dim3(256), 0, s, rhead.ptr, rpos.ptr, rvals.ptr, rlens.ptr, r,
                       src.ptr, olen.ptr);
    F4_LAUNCH_CHECK();
    fill_u32(olen.ptr + ro, 1, 0, s);
    // CSR
    out = Matrix();
    out.S = 1;
    out.R = ro;
    out.key_words = 2;
    out.row_ptr.reset(&c.pool, (u64)ro + 1);
    exclusive_scan_u32(olen.ptr, out.row_ptr.ptr, (u64)ro + 1, c.pool, s);
    u32 onnz = 0;
    readback(c, &onnz, out.row_ptr.ptr + ro, 4);
    out.nnz = onnz;
    out.col_ind.reset(&c.pool, std::max<u32>(onnz, 1));
    out.val.reset(&c.pool, std::max<u32>(onnz, 1));
    out.row_t.reset(&c.pool, 2 * (u64)std::max<u32>(ro, 1));
    out.row_k.reset(&c.pool, std::max<u32>(ro, 1));
    out.row_sys.reset(&c.pool, std::max<u32>(ro, 1));
    fill_u32(out.row_sys.ptr, std::max<u32>(ro, 1), 0, s);
    hipLaunchKernelGGL(k_mw_csr, dim3(std::min<u32>(8192, ceil_div(ro, 4))), dim3(256), 0, s, R, src.ptr, ro,
                       out.row_ptr.ptr, toff.ptr, colterm.ptr, dcoeff.ptr, doff.ptr, out.col_ind.ptr, out.val.ptr,
                       out.row_t.ptr, out.row_k.ptr);
    F4_LAUNCH_CHECK();
    out.dict_keys.reset(&c.pool, 2 * (u64)std::max<u32>(N, 1));
    F4_HIP_TRY(hipMemcpyAsync(out.dict_keys.ptr, dict.ptr, 2 * (u64)N * 8, hipMemcpyDeviceToDevice, s));
    out.sys.assign(1, SysPart());
    SysPart& P = out.sys[0];
    P.n = n;
    P.deg = dmax;
    P.r = ro;
    P.N = N;
    P.nnz = onnz;
}
