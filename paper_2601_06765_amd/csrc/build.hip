// Symbolic preprocessing SP : B -> (T, R, Pi) on gfx950 (Definition "Symbolic
// preprocessing operator"; Algorithm "FBSP"; section "FBSP: frontier-based
// symbolic preprocessing as bulk set algebra").
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

#define MB_THREADS 256
#define MB_WAVES (MB_THREADS / F4_WAVE)

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
    F4_HIP_TRY(hipMemcpyAsync(buf.ptr, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, c.stream));
    F4_HIP_TRY(hipStreamSynchronize(c.stream));
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

// ----------------------------------------------------------- row emission
// Rows [range[0], range[1]): record the rank of each row's leading monomial,
// mark it processed, and mark the rank of every term t * m of the row as seen.
// One wave per row, lanes over the terms; the seen-bits are gathered in an LDS
// bitmap per workgroup and flushed with one atomic OR per nonzero word.
__global__ __launch_bounds__(MB_THREADS) void k_mark_rows(const u64* rows_t, const u32* rows_k, u32* row_lmrank,
                                                           const u32* range, DevBasis G, const u32* binom_g,
                                                           u32 tabn, u32 D, u32* present, u32* done, u32 nwords,
                                                           int local_bitmap, u32* errflag) {
    extern __shared__ u32 sm[];
    u32* tab = sm;
    u32* lbits = sm + tabn;
    for (u32 i = threadIdx.x; i < tabn; i += MB_THREADS) tab[i] = binom_g[i];
    if (local_bitmap)
        for (u32 i = threadIdx.x; i < nwords; i += MB_THREADS) lbits[i] = 0;
    __syncthreads();
    const u32 n = G.n, w = G.w, lane = lane_id();
    const u32 rb = range[0], re = range[1];
    const u32 nw_total = gridDim.x * MB_WAVES;
    for (u32 row = rb + blockIdx.x * MB_WAVES + threadIdx.x / F4_WAVE; row < re; row += nw_total) {
        const u64 t = rows_t[row];
        const u32 k = rows_k[row];
        if (lane == 0) {
            u32 q = mono_rank(t + G.lm[k], n, w, D, tab);
            if (q == F4_BAD_RANK) {
                errflag[0] = 1u;
                q = 0;
            }
            row_lmrank[row] = q;
            atomicOr(&done[q >> 5], 1u << (q & 31));
        }
        const u64 off = G.off[k];
        const u32 len = G.len[k];
        for (u32 j = lane; j < len; j += F4_WAVE) {
            u32 q = mono_rank(t + G.mon[off + j], n, w, D, tab);
            if (q == F4_BAD_RANK) {
                errflag[0] = 1u;
                continue;
            }
            if (local_bitmap)
                atomicOr(&lbits[q >> 5], 1u << (q & 31));
            else
                atomicOr(&present[q >> 5], 1u << (q & 31));
        }
    }
    if (local_bitmap) {
        __syncthreads();
        for (u32 i = threadIdx.x; i < nwords; i += MB_THREADS) {
            u32 v = lbits[i];
            if (v) atomicOr(&present[i], v);
        }
    }
}

// frontier = seen and not processed
__global__ void k_frontier_count(const u32* present, const u32* done, u32 nwords, u32* cnt) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x)
        cnt[i] = __popc(present[i] & ~done[i]);
}

// write frontier ranks in ascending order, mark them processed, and open a
// new row range [range[1], ...) for the reducer rows appended next
__global__ void k_frontier_write(const u32* present, u32* done, u32 nwords, const u32* off, u32* list, u32* range) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) {
        u32 f = present[i] & ~done[i];
        if (!f) continue;
        done[i] |= f;
        u32 pos = off[i];
        while (f) {
            u32 b = __ffs(f) - 1;
            list[pos++] = i * 32 + b;
            f &= f - 1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) range[0] = range[1];
}

// One reducer per frontier monomial m: the active element with the largest
// index whose leading monomial divides m; the new row is (m / LM(g), g).
__global__ __launch_bounds__(MB_THREADS) void k_reducers(const u32* list, const u32* count_ptr, const u64* montab,
                                                          DevBasis G, const u32* active, u32 nactive, int lds_active,
                                                          u64* rows_t, u32* rows_k, u32* row_lmrank, u32* range,
                                                          u32 rcap) {
    extern __shared__ u64 slm[];
    if (lds_active) {
        for (u32 i = threadIdx.x; i < nactive; i += MB_THREADS) slm[i] = G.lm[active[i]];
        __syncthreads();
    }
    const u32 n = G.n, w = G.w;
    const u32 cnt = *count_ptr;
    for (u32 i = blockIdx.x * MB_THREADS + threadIdx.x; i < cnt; i += gridDim.x * MB_THREADS) {
        const u32 q = list[i];
        const u64 m = montab[q];
        for (u32 a = 0; a < nactive; ++a) {
            const u64 l = lds_active ? slm[a] : G.lm[active[a]];
            if (mono_divides(l, m, n, w)) {
                u32 slot = atomicAdd(&range[1], 1u);
                if (slot >= rcap) {
                    range[3] = 2u;
                    break;
                }
                rows_t[slot] = m - l;
                rows_k[slot] = active[a];
                row_lmrank[slot] = q;
                break;
            }
        }
    }
}

__global__ void k_word_popc(const u32* present, u32 nwords, u32* cnt) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x)
        cnt[i] = __popc(present[i]);
}

// Dictionary: column of rank q = number of seen ranks below q; the columns are
// therefore the seen monomials in descending grevlex order.
__global__ void k_dict(const u32* present, u32 nwords, const u32* off, const u64* montab, u32* colmap,
                       u64* dict_keys) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) {
        u32 f = present[i];
        u32 pos = off[i];
        while (f) {
            u32 b = __ffs(f) - 1;
            u32 q = i * 32 + b;
            colmap[q] = pos;
            dict_keys[pos] = montab[q];
            ++pos;
            f &= f - 1;
        }
    }
}

// M = sum of the row lengths (first pass of the two-pass plan, reduced)
__global__ void k_sum_len(const u32* rows_k, const u32* range, const u32* len, unsigned long long* M) {
    const u32 r = range[1];
    u32 s = 0;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) s += len[rows_k[i]];
    for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, F4_WAVE);
    if (lane_id() == 0 && s) atomicAdd(M, (unsigned long long)s);
}

// Row order: leading monomial descending (= rank ascending), then basis index.
__global__ void k_row_keys(const u32* row_lmrank, const u32* rows_k, u32 r, u32 kbits, u64* keys, u32* vals) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        keys[i] = ((u64)row_lmrank[i] << kbits) | rows_k[i];
        vals[i] = i;
    }
}

__global__ void k_gather_rows(const u32* perm, const u64* rows_t, const u32* rows_k, const u32* glen, u32 r,
                              u64* out_t, u32* out_k, u32* out_len) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        u32 s = perm[i];
        u32 k = rows_k[s];
        out_t[i] = rows_t[s];
        out_k[i] = k;
        out_len[i] = glen[k];
    }
}

// Pass 2 of the two-pass plan fused with the dictionary join (dense rank):
// row i writes col_ind/val into its own segment [row_ptr[i], row_ptr[i+1]).
__global__ __launch_bounds__(MB_THREADS) void k_fill_rank(const u64* row_t, const u32* row_k, const u32* row_ptr,
                                                           u32 r, DevBasis G, const u32* binom_g, u32 tabn, u32 D,
                                                           u32 nmax, const u32* colmap, u32* col_ind, u32* val) {
    extern __shared__ u32 sm[];
    for (u32 i = threadIdx.x; i < tabn; i += MB_THREADS) sm[i] = binom_g[i];
    __syncthreads();
    const u32 n = G.n, w = G.w, lane = lane_id();
    const u32 nw_total = gridDim.x * MB_WAVES;
    for (u32 row = blockIdx.x * MB_WAVES + threadIdx.x / F4_WAVE; row < r; row += nw_total) {
        const u64 t = row_t[row];
        const u32 k = row_k[row];
        const u64 off = G.off[k];
        const u32 len = G.len[k];
        const u32 s = row_ptr[row];
        for (u32 j = lane; j < len; j += F4_WAVE) {
            u32 q = mono_rank(t + G.mon[off + j], n, w, D, sm);
            col_ind[s + j] = q < nmax ? colmap[q] : 0u;
            val[s + j] = G.coeff[off + j];
        }
    }
}

// ------------------------------------------------------- radix-sort path
// Compact order key of a monomial of degree <= D: (D - deg) on top, then the
// exponents a_n .. a_1 in fields of b = bitlength(D) bits.  Ascending keys are
// descending grevlex, and the key is injective on Mon_{<=D}.
__device__ __forceinline__ u64 compact_key(u64 P, u32 n, u32 w, u32 b, u32 D) {
    u64 k = (u64)(D - mono_deg(P)) << (n * b);
    for (u32 i = 0; i < n; ++i) k |= (u64)mono_exp(P, i, w) << (b * i);
    return k;
}
__device__ __forceinline__ u64 compact_to_P(u64 k, u32 n, u32 w, u32 b, u32 D) {
    u64 P = 0;
    u32 deg = 0;
    for (u32 i = 0; i < n; ++i) {
        u32 a = (u32)((k >> (b * i)) & ((1u << b) - 1));
        P |= (u64)a << (w * i);
        deg += a;
    }
    return P | ((u64)deg << 56);
}

// Pass 2 of the two-pass plan as written: materialise row_key / row_val
__global__ __launch_bounds__(MB_THREADS) void k_fill_keys(const u64* row_t, const u32* row_k, const u32* row_ptr,
                                                           u32 r, DevBasis G, u32 b, u32 D, u64* row_key,
                                                           u32* row_val) {
    const u32 n = G.n, w = G.w, lane = lane_id();
    const u32 nw_total = gridDim.x * MB_WAVES;
    for (u32 row = blockIdx.x * MB_WAVES + threadIdx.x / F4_WAVE; row < r; row += nw_total) {
        const u64 t = row_t[row];
        const u32 k = row_k[row];
        const u64 off = G.off[k];
        const u32 len = G.len[k];
        const u32 s = row_ptr[row];
        for (u32 j = lane; j < len; j += F4_WAVE) {
            row_key[s + j] = compact_key(t + G.mon[off + j], n, w, b, D);
            row_val[s + j] = G.coeff[off + j];
        }
    }
}

// Join: position of every row key in the sorted dictionary (binary search; the
// dictionary sits in LDS when it fits).
__global__ __launch_bounds__(MB_THREADS) void k_join(const u64* row_key, u64 M, const u64* dict, const u32* N_ptr,
                                                      u32 Ncap, int lds_dict, u32* col_ind) {
    extern __shared__ u64 sd[];
    const u32 N = min(*N_ptr, Ncap);
    if (lds_dict) {
        for (u32 i = threadIdx.x; i < N; i += MB_THREADS) sd[i] = dict[i];
        __syncthreads();
    }
    const u64* D_ = lds_dict ? sd : dict;
    for (u64 e = (u64)blockIdx.x * MB_THREADS + threadIdx.x; e < M; e += (u64)gridDim.x * MB_THREADS) {
        const u64 key = row_key[e];
        u32 lo = 0, hi = N;
        while (lo < hi) {
            u32 mid = (lo + hi) >> 1;
            if (D_[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        col_ind[e] = lo;
    }
}

__global__ void k_dict_from_compact(const u64* dictc, const u32* N_ptr, u32 Ncap, u32 n, u32 w, u32 b, u32 D,
                                    u64* dict_keys) {
    const u32 N = min(*N_ptr, Ncap);
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
        dict_keys[i] = compact_to_P(dictc[i], n, w, b, D);
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
void build_matrix(Ctx& c, const BuildArgs& a, Matrix& out) {
    hipStream_t s = c.stream;
    const u32 n = a.G.n, w = a.G.w, D = a.D;
    if (a.r0 == 0) throw F4Error{1, "empty row list"};
    const u64 nmax64 = binom_host(n + D, n);
    if (nmax64 > (1ull << 27)) throw F4Error{2, "N(n, D) too large for the dense-rank closure"};
    const u32 nmax = (u32)nmax64;
    const u32 nwords = ceil_div(nmax, 32);
    const u32* binom_g = rank_table(c, n, D);
    const u32 tabn = (n + D + 2) * F4_BSTRIDE;
    const u64* montab = unrank_table(c, n, D);

    hipEvent_t ev0 = stage_event(c);

    // bitmaps of seen / processed monomials, rows with capacity r0 + N(n, D)
    DBuf<u32> present(&c.pool, nwords), done(&c.pool, nwords);
    fill_u32(present.ptr, nwords, 0, s);
    fill_u32(done.ptr, nwords, 0, s);
    const u64 rcap = (u64)a.r0 + (a.closure ? nmax : 0);
    DBuf<u64> rows_t(&c.pool, rcap);
    DBuf<u32> rows_k(&c.pool, rcap), row_lmrank(&c.pool, rcap);
    F4_HIP_TRY(hipMemcpyAsync(rows_t.ptr, a.rows_t, (u64)a.r0 * 8, hipMemcpyDeviceToDevice, s));
    F4_HIP_TRY(hipMemcpyAsync(rows_k.ptr, a.rows_k, (u64)a.r0 * 4, hipMemcpyDeviceToDevice, s));
    // range[0..1] = current row range, range[2] = frontier count slot (unused), M at hdr
    DBuf<u32> range(&c.pool, 4);
    {
        u32 h[4] = {0, a.r0, 0, 0};
        upload(c, range.ptr, h, sizeof(h));
    }
    DBuf<unsigned long long> Mdev(&c.pool, 1);
    fill_u64((u64*)Mdev.ptr, 1, 0, s);

    const int local_bitmap = (tabn + nwords) * 4 <= 48 * 1024;
    const size_t mark_lds = (tabn + (local_bitmap ? nwords : 0)) * 4;
    const u32 mark_grid = (u32)std::max(1, c.dev.cus);
    auto mark = [&]() {
        hipLaunchKernelGGL(k_mark_rows, dim3(mark_grid), dim3(MB_THREADS), mark_lds, s, rows_t.ptr, rows_k.ptr,
                           row_lmrank.ptr, range.ptr, a.G, binom_g, tabn, D, present.ptr, done.ptr, nwords,
                           local_bitmap, range.ptr + 3);
        F4_LAUNCH_CHECK();
    };
    mark();

    DBuf<u32> cnt(&c.pool, nwords + 1), list(&c.pool, a.closure ? nmax : 1);
    const int lds_active = a.nactive * 8 <= 32 * 1024;
    const u32 wgrid = grid_for(nwords, 256, 1024);
    u32 rounds = 0;
    u32 hdr[4];
    for (;;) {
        if (a.closure) {
            // two speculative rounds per host check: dense systems converge in two
            for (int k = 0; k < 2; ++k) {
                hipLaunchKernelGGL(k_frontier_count, dim3(wgrid), dim3(256), 0, s, present.ptr, done.ptr, nwords,
                                   cnt.ptr);
                F4_LAUNCH_CHECK();
                exclusive_scan_u32(cnt.ptr, cnt.ptr, nwords, c.pool, s);
                hipLaunchKernelGGL(k_frontier_write, dim3(wgrid), dim3(256), 0, s, present.ptr, done.ptr, nwords,
                                   cnt.ptr, list.ptr, range.ptr);
                F4_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_reducers, dim3(grid_for(nmax, MB_THREADS, 1024)), dim3(MB_THREADS),
                                   lds_active ? a.nactive * 8 : 0, s, list.ptr, cnt.ptr + nwords, montab, a.G,
                                   a.active, a.nactive, lds_active, rows_t.ptr, rows_k.ptr, row_lmrank.ptr,
                                   range.ptr, (u32)rcap);
                F4_LAUNCH_CHECK();
                mark();
                ++rounds;
            }
            // remaining frontier after the rounds
            hipLaunchKernelGGL(k_frontier_count, dim3(wgrid), dim3(256), 0, s, present.ptr, done.ptr, nwords,
                               cnt.ptr);
            F4_LAUNCH_CHECK();
            exclusive_scan_u32(cnt.ptr, cnt.ptr, nwords, c.pool, s);
            F4_HIP_TRY(hipMemcpyAsync(range.ptr + 2, cnt.ptr + nwords, 4, hipMemcpyDeviceToDevice, s));
        }
        readback(c, hdr, range.ptr, sizeof(hdr));
        if (hdr[3]) throw F4Error{1, hdr[3] == 1 ? "a row term is not a monomial of degree <= D (unsorted or "
                                                   "inconsistent input terms)"
                                                 : "row capacity exceeded"};
        if (!a.closure || hdr[2] == 0) break;
        if (rounds > 4 * (D + 8)) throw F4Error{5, "closure did not converge"};
    }
    const u32 r = hdr[1];

    // dictionary (dense rank): popcount prefix of the seen bitmap
    DBuf<u32> colmap(&c.pool, nmax);
    hipLaunchKernelGGL(k_word_popc, dim3(wgrid), dim3(256), 0, s, present.ptr, nwords, cnt.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(cnt.ptr, cnt.ptr, nwords, c.pool, s);
    out.dict_keys.reset(&c.pool, nmax);  // trimmed view: first N entries are valid
    hipLaunchKernelGGL(k_dict, dim3(wgrid), dim3(256), 0, s, present.ptr, nwords, cnt.ptr, montab, colmap.ptr,
                       out.dict_keys.ptr);
    F4_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_len, dim3(grid_for(r, 256, 1024)), dim3(256), 0, s, rows_k.ptr, range.ptr, a.G.len,
                       Mdev.ptr);
    F4_LAUNCH_CHECK();
    u32 Nhost = 0;
    unsigned long long Mhost = 0;
    {
        u8* st = staging(c, 16);
        F4_HIP_TRY(hipMemcpyAsync(st, cnt.ptr + nwords, 4, hipMemcpyDeviceToHost, s));
        F4_HIP_TRY(hipMemcpyAsync(st + 8, Mdev.ptr, 8, hipMemcpyDeviceToHost, s));
        F4_HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(&Nhost, st, 4);
        std::memcpy(&Mhost, st + 8, 8);
    }
    if (Mhost >= (1ull << 32)) throw F4Error{2, "matrix has 2^32 or more entries"};
    if (Nhost >= (1u << 26)) throw F4Error{2, "dictionary has 2^26 or more columns"};
    const u32 N = Nhost;
    const u32 M = (u32)Mhost;
    hipEvent_t ev1 = stage_event(c);

    // row order: sort by (rank of LM, basis index)
    const u32 kbits = std::max<u32>(1, bitlen(a.G.npolys ? a.G.npolys - 1 : 0));
    const u32 rbits = std::max<u32>(1, bitlen(nmax - 1));
    DBuf<u64> keys(&c.pool, r);
    DBuf<u32> perm(&c.pool, r);
    const u32 rgrid = grid_for(r, 256, 4096);
    hipLaunchKernelGGL(k_row_keys, dim3(rgrid), dim3(256), 0, s, row_lmrank.ptr, rows_k.ptr, r, kbits, keys.ptr,
                       perm.ptr);
    F4_LAUNCH_CHECK();
    radix_sort_pairs(keys.ptr, perm.ptr, r, 0, rbits + kbits, c.pool, s);
    out.row_t.reset(&c.pool, r);
    out.row_k.reset(&c.pool, r);
    out.row_ptr.reset(&c.pool, (u64)r + 1);
    hipLaunchKernelGGL(k_gather_rows, dim3(rgrid), dim3(256), 0, s, perm.ptr, rows_t.ptr, rows_k.ptr, a.G.len, r,
                       out.row_t.ptr, out.row_k.ptr, out.row_ptr.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(out.row_ptr.ptr, out.row_ptr.ptr, r, c.pool, s);

    out.col_ind.reset(&c.pool, M);
    out.val.reset(&c.pool, M);
    int path = a.dict_path;
    if (path < 0) path = (c.flags & 4u) ? 1 : 0;  // F4_OPT_DICT_RADIX
    const u32 fgrid = grid_for(r, MB_WAVES, 8 * (u32)std::max(1, c.dev.cus));
    if (path == 0) {
        hipLaunchKernelGGL(k_fill_rank, dim3(fgrid), dim3(MB_THREADS), tabn * 4, s, out.row_t.ptr, out.row_k.ptr,
                           out.row_ptr.ptr, r, a.G, binom_g, tabn, D, nmax, colmap.ptr, out.col_ind.ptr,
                           out.val.ptr);
        F4_LAUNCH_CHECK();
    } else {
        const u32 b = std::max<u32>(1, bitlen(D));
        const u32 kb = (n + 1) * b;
        if (kb > 64) throw F4Error{2, "compact key does not fit 64 bits"};
        DBuf<u64> row_key(&c.pool, M), cand(&c.pool, M), dictc(&c.pool, M);
        hipLaunchKernelGGL(k_fill_keys, dim3(fgrid), dim3(MB_THREADS), 0, s, out.row_t.ptr, out.row_k.ptr,
                           out.row_ptr.ptr, r, a.G, b, D, row_key.ptr, out.val.ptr);
        F4_LAUNCH_CHECK();
        F4_HIP_TRY(hipMemcpyAsync(cand.ptr, row_key.ptr, (u64)M * 8, hipMemcpyDeviceToDevice, s));
        radix_sort_keys(cand.ptr, M, 0, kb, c.pool, s);
        DBuf<u32> ncount(&c.pool, 1);
        unique_sorted_u64(cand.ptr, M, dictc.ptr, ncount.ptr, c.pool, s);
        const int lds_dict = (u64)N * 8 <= c.dev.max_lds;
        hipLaunchKernelGGL(k_join, dim3(grid_for(M, MB_THREADS, 16 * (u32)std::max(1, c.dev.cus))), dim3(MB_THREADS),
                           lds_dict ? (size_t)N * 8 : 0, s, row_key.ptr, (u64)M, dictc.ptr, ncount.ptr, N, lds_dict,
                           out.col_ind.ptr);
        F4_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_dict_from_compact, dim3(grid_for(N, 256, 1024)), dim3(256), 0, s, dictc.ptr,
                           ncount.ptr, N, n, w, b, D, out.dict_keys.ptr);
        F4_LAUNCH_CHECK();
    }
    hipEvent_t ev2 = stage_event(c);

    out.n = n;
    out.r = r;
    out.N = N;
    out.nnz = M;
    out.deg = D;
    out.closure_rounds = rounds;
    out.dict_path = (u32)path;
    if (ev0) {
        F4_HIP_TRY(hipEventSynchronize(ev2));
        out.t_dict = event_ms(ev0, ev1);
        out.t_assemble = event_ms(ev1, ev2);
    }
}
