// The block schedule that enriches the plan Pi (section "PSGE:
// panel-structured Gaussian elimination", "Why Pi must be enriched": panel
// boundaries and the row-to-panel incidence; section "Row assembly as a
// dictionary join; divergence control via SELL-C-sigma bucketing"), and a
// block product over its SELL-C-sigma slices.
//
// Panels are the column segments [l W, (l + 1) W); a row belongs to the panel
// of its leading column (empty rows to a last group).  Within a panel, rows in
// row order are cut into windows of sigma; each window is sorted longest row
// first (ties by row index); slices are runs of C rows inside one panel,
// padded to their longest row and stored column-major (entry k of the slice's
// row j at offset + k C + j; padding: column 0, value 0).
//
// Build: (1) a radix sort of (panel, row) groups the rows by panel in row
// order; (2) panel offsets from the group boundaries (each offset written by
// exactly one thread); (3) a radix sort of (start of the row's window, longest
// first, position in the window) orders the windows; (4) slice counts per
// panel, their scan, one thread per slice for its start, panel and width; (5)
// the scan of C * width gives the slice offsets; (6) one wave per slice writes
// its storage.
//
// Product Y = A X (b <= 8 vectors): one wave per slice, each row of the slice
// on a few lanes that split the b vectors; the lanes walk the slice's width
// with coalesced reads of the column and value words, gather words of X, and
// sum the raw 64-bit products exactly in 96 bits (a 64-bit sum and a carry
// count), reduced once per output as in the CSR product; padding values are
// 0 and add nothing.
#include <algorithm>

#include "internal.hpp"

static u32 sc_bits(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

__global__ void k_sc_panel_keys(const u32* __restrict__ ptr, const u32* __restrict__ col, u32 r, u32 W, u32 npan,
                                u32 rbits, u64* __restrict__ keys, u32* __restrict__ vals) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        const u32 pnl = ptr[i + 1] > ptr[i] ? col[ptr[i]] / W : npan;
        keys[i] = ((u64)pnl << rbits) | i;
        vals[i] = i;
    }
}

// panel_ptr[q] = first position of panel q (npan + 2 entries): position x
// writes the offsets of the panels between its predecessor's and its own
__global__ void k_sc_panel_ptr(const u64* __restrict__ keys, u32 r, u32 rbits, u32 npan, u32* __restrict__ pptr) {
    for (u32 x = blockIdx.x * blockDim.x + threadIdx.x; x <= r; x += gridDim.x * blockDim.x) {
        const u32 prev = x == 0 ? 0u : (u32)(keys[x - 1] >> rbits) + 1;
        const u32 cur = x == r ? npan + 1 : (u32)(keys[x] >> rbits);
        for (u32 q = prev; q <= cur; ++q) pptr[q] = x;
        if (x == r)
            for (u32 q = cur + 1; q <= npan + 1; ++q) pptr[q] = r;
    }
}

// window keys: global start of the row's window, then longest first, then the
// position inside the window
__global__ void k_sc_window_keys(const u64* __restrict__ pkeys, const u32* __restrict__ rows, u32 r, u32 rbits,
                                 const u32* __restrict__ pptr, const u32* __restrict__ ptr, u32 sigma, u32 wbits,
                                 u32 lbits, u64* __restrict__ keys, u32* __restrict__ vals) {
    for (u32 x = blockIdx.x * blockDim.x + threadIdx.x; x < r; x += gridDim.x * blockDim.x) {
        const u32 pnl = (u32)(pkeys[x] >> rbits), i = rows[x];
        const u32 pos = x - pptr[pnl];
        const u32 wstart = pptr[pnl] + (pos / sigma) * sigma;
        const u64 lmax = (1ull << lbits) - 1;  // every row length fits lbits bits
        const u64 len = ptr[i + 1] - ptr[i];
        keys[x] = ((u64)wstart << (lbits + wbits)) | ((lmax - len) << wbits) | (pos % sigma);
        vals[x] = i;
    }
}

__global__ void k_sc_slice_count(const u32* __restrict__ pptr, u32 ngroups, u32 C, u32* __restrict__ cnt) {
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q <= ngroups; q += gridDim.x * blockDim.x)
        cnt[q] = q < ngroups ? (pptr[q + 1] - pptr[q] + C - 1) / C : 0u;
}

// one thread per slice: its panel (binary search over the slice bases), start,
// rows and width
__global__ void k_sc_slices(const u32* __restrict__ sbase, u32 ngroups, const u32* __restrict__ pptr, u32 C,
                            const u32* __restrict__ perm, const u32* __restrict__ ptr, u32 nslices,
                            u32* __restrict__ sstart, u32* __restrict__ spanel, u32* __restrict__ swidth,
                            u64* __restrict__ ssize) {
    for (u32 s = blockIdx.x * blockDim.x + threadIdx.x; s < nslices; s += gridDim.x * blockDim.x) {
        u32 lo = 0, hi = ngroups;  // last group q with sbase[q] <= s
        while (hi - lo > 1) {
            const u32 mid = (lo + hi) >> 1;
            if (sbase[mid] <= s)
                lo = mid;
            else
                hi = mid;
        }
        const u32 s0 = pptr[lo] + (s - sbase[lo]) * C, s1 = min(s0 + C, pptr[lo + 1]);
        u32 w = 0;
        for (u32 x = s0; x < s1; ++x) w = max(w, ptr[perm[x] + 1] - ptr[perm[x]]);
        sstart[s] = s0;
        spanel[s] = lo;
        swidth[s] = w;
        ssize[s] = (u64)C * w;
    }
}

// one wave per slice: the padded column-major storage
__global__ void k_sc_sell(const u32* __restrict__ sstart, const u32* __restrict__ spanel,
                          const u32* __restrict__ swidth, const u64* __restrict__ soff, u32 nslices,
                          const u32* __restrict__ pptr, u32 C, const u32* __restrict__ perm, const u32* __restrict__ ptr,
                          const u32* __restrict__ col, const u32* __restrict__ val, u32* __restrict__ scol,
                          u32* __restrict__ sval) {
    const u32 lane = lane_id();
    const u32 waves = gridDim.x * (blockDim.x / F4_WAVE);
    for (u32 s = blockIdx.x * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE; s < nslices; s += waves) {
        const u32 s0 = sstart[s], s1 = min(s0 + C, pptr[spanel[s] + 1]), w = swidth[s];
        const u64 o = soff[s];
        for (u32 j = lane; j < C; j += F4_WAVE) {
            const bool live = s0 + j < s1;
            const u32 i = live ? perm[s0 + j] : 0u;
            const u32 e0 = live ? ptr[i] : 0u, l = live ? ptr[i + 1] - e0 : 0u;
            for (u32 k = 0; k < w; ++k) {
                scol[o + (u64)k * C + j] = k < l ? col[e0 + k] : 0u;
                sval[o + (u64)k * C + j] = k < l ? val[e0 + k] : 0u;
            }
        }
    }
}

// Product: one wave per slice.  Lane j reads word j of each step of the
// slice's storage (one coalesced read of the column words and one of the
// values, the next step's read issued before this step's gathers); BP lanes
// then share a row, lane k of a row covering the VW consecutive words
// k VW .. k VW + VW - 1 of the b vectors (one aligned request per gathered
// row of X), and take the row's entry from its reader by a shuffle; the wave
// covers 64 / BP rows at a time, the BP passes over the slice's rows
// unrolled so that their gathers are in flight together.  Workgroups go to
// the eight XCDs in turn: each XCD takes a contiguous range of slices, i.e.
// of panels, whose rows gather nearby rows of X through its L2.
template <int BP, int VW>
__global__ __launch_bounds__(256) void k_spmm_sell(Fp f, u32 b, const u32* __restrict__ sstart,
                                                    const u32* __restrict__ spanel, const u32* __restrict__ swidth,
                                                    const u64* __restrict__ soff, u32 nslices,
                                                    const u32* __restrict__ pptr, u32 C,
                                                    const u32* __restrict__ perm, const u32* __restrict__ scol,
                                                    const u32* __restrict__ sval, const u32* __restrict__ X,
                                                    u32* __restrict__ Y) {
    constexpr u32 RPW = F4_WAVE / BP;  // rows of the slice per pass
    const u32 nb = gridDim.x, q = nb / 8, rem = nb % 8, x = blockIdx.x % 8;
    const u32 lb = x * q + min(x, rem) + blockIdx.x / 8;
    const u32 s = lb * (blockDim.x / F4_WAVE) + threadIdx.x / F4_WAVE;
    if (s >= nslices) return;  // the whole wave
    const u32 lane = lane_id(), jr = lane / BP, k = (lane % BP) * VW;
    const u32 s0 = sstart[s], s1 = min(s0 + C, pptr[spanel[s] + 1]), w = swidth[s];
    const u32 rows = s1 - s0;  // live rows of the slice (<= C <= 64)
    const u64 o = soff[s];
    const bool reader = lane < rows;
    u32 mc = reader && w ? scol[o + lane] : 0u, mv = reader && w ? sval[o + lane] : 0u;
    u64 lo[BP][VW] = {};  // exact sums: hi * 2^64 + lo
    u32 hi[BP][VW] = {};
    for (u32 e = 0; e < w; ++e) {
        const bool more = reader && e + 1 < w;
        const u32 nc = more ? scol[o + (u64)(e + 1) * C + lane] : 0u;
        const u32 nv = more ? sval[o + (u64)(e + 1) * C + lane] : 0u;
#pragma unroll
        for (u32 ps = 0; ps < BP; ++ps) {
            const u32 src = ps * RPW + jr;  // the row, and the lane that read its entry
            const u32 cj = BP == 1 ? mc : (u32)__shfl((int)mc, (int)src);
            const u32 vj = BP == 1 ? mv : (u32)__shfl((int)mv, (int)src);
            if (!vj || k >= b) continue;  // padding, rows past the slice and dead lanes add nothing
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
                const u64 nl = lo[ps][v] + (u64)vj * xv[v];
                hi[ps][v] += nl < lo[ps][v] ? 1u : 0u;
                lo[ps][v] = nl;
            }
        }
        mc = nc;
        mv = nv;
    }
    const u32 c64 = fp_reduce(f, (u64)f.r32 * f.r32);  // 2^64 mod p
#pragma unroll
    for (u32 ps = 0; ps < BP; ++ps) {
        const u32 j = ps * RPW + jr;
        if (j >= rows || k >= b) continue;
        const u32 i = perm[s0 + j];
        u32 out[VW];
#pragma unroll
        for (u32 v = 0; v < VW; ++v) {
            const u64 acc = (u64)fp_reduce_any(f, lo[ps][v]) + fp_reduce(f, (u64)fp_reduce32(f, hi[ps][v]) * c64);
            out[v] = fp_reduce_any(f, acc);
        }
        if (VW == 2)
            *reinterpret_cast<uint2*>(Y + (u64)i * b + k) = make_uint2(out[0], out[VW - 1]);
        else
            Y[(u64)i * b + k] = out[0];
    }
}

void sched_build(Ctx& c, u32 r, u32 N, u64 nnz, const u32* ptr, const u32* col, const u32* val, u32 W, u32 C,
                 u32 sigma, SchedBufs& S) {
    hipStream_t s = c.stream;
    if (W == 0 || C == 0 || C > F4_WAVE || sigma == 0) throw F4Error{1, "bad schedule parameters"};
    S = SchedBufs();
    S.W = W;
    S.C = C;
    S.sigma = sigma;
    S.r = r;
    const u64 npan64 = std::max<u64>(1, ((u64)N + W - 1) / W);
    if (npan64 >= (1u << 30)) throw F4Error{2, "too many panels"};
    const u32 npan = (u32)npan64;
    S.npanels = npan;
    const u32 rbits = std::max<u32>(1, sc_bits(r));
    if (sc_bits(npan + 1) + rbits > 64) throw F4Error{2, "schedule key does not fit 64 bits"};
    S.perm.reset(&c.pool, std::max<u32>(r, 1));
    S.panel_ptr.reset(&c.pool, (u64)npan + 2);
    const u32 grid = std::min<u32>(4096, std::max<u32>(1, ceil_div(r + 1, 256)));
    DBuf<u64> pkeys(&c.pool, std::max<u32>(r, 1)), wkeys(&c.pool, std::max<u32>(r, 1));
    DBuf<u32> rows(&c.pool, std::max<u32>(r, 1));
    if (r) {
        hipLaunchKernelGGL(k_sc_panel_keys, dim3(grid), dim3(256), 0, s, ptr, col, r, W, npan, rbits, pkeys.ptr,
                           rows.ptr);
        F4_LAUNCH_CHECK();
        radix_sort_pairs(pkeys.ptr, rows.ptr, r, 0, rbits + sc_bits(npan + 1), c.pool, s);
    }
    hipLaunchKernelGGL(k_sc_panel_ptr, dim3(grid), dim3(256), 0, s, pkeys.ptr, r, rbits, npan, S.panel_ptr.ptr);
    F4_LAUNCH_CHECK();
    const u32 wbits = std::max<u32>(1, sc_bits(sigma - 1));
    const u32 lbits = std::max<u32>(1, sc_bits(nnz));  // a row holds at most nnz entries
    if (rbits + lbits + wbits > 64) throw F4Error{2, "window key does not fit 64 bits"};
    if (r) {
        hipLaunchKernelGGL(k_sc_window_keys, dim3(grid), dim3(256), 0, s, pkeys.ptr, rows.ptr, r, rbits,
                           S.panel_ptr.ptr, ptr, sigma, wbits, lbits, wkeys.ptr, S.perm.ptr);
        F4_LAUNCH_CHECK();
        radix_sort_pairs(wkeys.ptr, S.perm.ptr, r, 0, rbits + lbits + wbits, c.pool, s);
    }
    // slices
    const u32 ngroups = npan + 1;
    DBuf<u32> cnt(&c.pool, (u64)ngroups + 1), sbase(&c.pool, (u64)ngroups + 1);
    hipLaunchKernelGGL(k_sc_slice_count, dim3(std::max<u32>(1, ceil_div(ngroups + 1, 256))), dim3(256), 0, s,
                       S.panel_ptr.ptr, ngroups, C, cnt.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(cnt.ptr, sbase.ptr, (u64)ngroups + 1, c.pool, s);
    u32 ns = 0;
    readback(c, &ns, sbase.ptr + ngroups, 4);
    S.nslices = ns;
    S.slice_start.reset(&c.pool, std::max<u32>(ns, 1));
    S.slice_panel.reset(&c.pool, std::max<u32>(ns, 1));
    S.slice_width.reset(&c.pool, std::max<u32>(ns, 1));
    S.slice_off.reset(&c.pool, (u64)ns + 1);
    DBuf<u64> ssize(&c.pool, (u64)ns + 1);
    fill_u64(ssize.ptr + ns, 1, 0, s);
    if (ns) {
        hipLaunchKernelGGL(k_sc_slices, dim3(std::min<u32>(4096, ceil_div(ns, 256))), dim3(256), 0, s, sbase.ptr,
                           ngroups, S.panel_ptr.ptr, C, S.perm.ptr, ptr, ns, S.slice_start.ptr, S.slice_panel.ptr,
                           S.slice_width.ptr, ssize.ptr);
        F4_LAUNCH_CHECK();
    }
    // exclusive scan of the slice sizes, in 64 bits on the host (one value
    // per slice)
    {
        std::vector<u64> h((u64)ns + 1);
        readback(c, h.data(), ssize.ptr, h.size() * 8);
        u64 acc = 0;
        for (u64& x : h) {
            const u64 v = x;
            x = acc;
            acc += v;
        }
        S.padded = h[ns];
        upload(c, S.slice_off.ptr, h.data(), h.size() * 8);
    }
    S.sell_col.reset(&c.pool, std::max<u64>(S.padded, 1));
    S.sell_val.reset(&c.pool, std::max<u64>(S.padded, 1));
    if (ns) {
        hipLaunchKernelGGL(k_sc_sell, dim3(std::min<u32>(8192, ceil_div(ns, 4))), dim3(256), 0, s,
                           S.slice_start.ptr, S.slice_panel.ptr, S.slice_width.ptr, S.slice_off.ptr, ns,
                           S.panel_ptr.ptr, C, S.perm.ptr, ptr, col, val, S.sell_col.ptr, S.sell_val.ptr);
        F4_LAUNCH_CHECK();
    }
    S.has = true;
}

template <int BP, int VW>
static void sell_launch(hipStream_t s, const Fp& f, u32 b, const SchedBufs& S, const u32* X, u32* Y) {
    const u32 grid = ceil_div(S.nslices, 256 / F4_WAVE);
    hipLaunchKernelGGL((k_spmm_sell<BP, VW>), dim3(grid), dim3(256), 0, s, f, b, S.slice_start.ptr,
                       S.slice_panel.ptr, S.slice_width.ptr, S.slice_off.ptr, S.nslices, S.panel_ptr.ptr, S.C,
                       S.perm.ptr, S.sell_col.ptr, S.sell_val.ptr, X, Y);
    F4_LAUNCH_CHECK();
}

void spmm_sell_run(hipStream_t s, u32 p, const SchedBufs& S, u32 b, const u32* X, u32* Y) {
    if (!S.nslices) return;
    const Fp f = make_fp(p);
    // two words per lane: an even b with X and Y 8-byte aligned
    if (b % 2 == 0 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 7) == 0) {
        if (b <= 2)
            sell_launch<1, 2>(s, f, b, S, X, Y);
        else if (b <= 4)
            sell_launch<2, 2>(s, f, b, S, X, Y);
        else
            sell_launch<4, 2>(s, f, b, S, X, Y);
        return;
    }
    if (b <= 1)
        sell_launch<1, 1>(s, f, b, S, X, Y);
    else if (b <= 2)
        sell_launch<2, 1>(s, f, b, S, X, Y);
    else if (b <= 4)
        sell_launch<4, 1>(s, f, b, S, X, Y);
    else
        sell_launch<8, 1>(s, f, b, S, X, Y);
}
