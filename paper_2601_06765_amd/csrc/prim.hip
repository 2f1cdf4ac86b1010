// Bulk data-parallel primitives (section "FBSP: frontier-based symbolic
// preprocessing as bulk set algebra": only scan / sort / unique synchronize).
//   - exclusive prefix sum (the two-pass count -> prefix-sum -> fill plan)
//   - stable LSD radix sort of 64-bit keys on a bit range, with wave64
//     ballot-based digit matching for the in-tile stable ranks
//   - unique of a sorted key stream
#include "internal.hpp"
#include "sort_lds.hpp"

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(u32* p, u64 n, u32 v) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u64(u64* p, u64 n, u64 v) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = v;
}

void fill_u32(u32* p, u64 n, u32 v, hipStream_t s) {
    if (!n) return;
    u32 blocks = ceil_div(n, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, n, v);
    F4_LAUNCH_CHECK();
}
void fill_u64(u64* p, u64 n, u64 v, hipStream_t s) {
    if (!n) return;
    u32 blocks = ceil_div(n, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, p, n, v);
    F4_LAUNCH_CHECK();
}

// ------------------------------------------------------------------- scan
#define SCAN_THREADS 1024
#define SCAN_ITEMS 4
#define SCAN_TILE (SCAN_THREADS * SCAN_ITEMS)

// Single-workgroup scan over the whole array (tiles in sequence with a carry).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_single(const u32* in, u32* out, u64 n) {
    __shared__ u32 s_wave[33];
    u32 carry = 0;
    for (u64 base = 0; base < n; base += SCAN_TILE) {
        u32 v[SCAN_ITEMS];
        u32 sum = 0;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + j;
            v[j] = i < n ? in[i] : 0;
            sum += v[j];
        }
        u32 total;
        u32 pre = block_exclusive_scan(sum, s_wave, &total) + carry;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + j;
            if (i < n) out[i] = pre;
            pre += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_sums(const u32* in, u64 n, u32* sums) {
    __shared__ u32 s_wave[33];
    u64 base = (u64)blockIdx.x * SCAN_TILE;
    u32 sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + j;
        sum += i < n ? in[i] : 0;
    }
    u32 total;
    block_exclusive_scan(sum, s_wave, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const u32* in, u32* out, u64 n, const u32* offs) {
    __shared__ u32 s_wave[33];
    u64 base = (u64)blockIdx.x * SCAN_TILE;
    u32 v[SCAN_ITEMS];
    u32 sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + j;
        v[j] = i < n ? in[i] : 0;
        sum += v[j];
    }
    u32 total;
    u32 pre = block_exclusive_scan(sum, s_wave, &total) + offs[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + j;
        if (i < n) out[i] = pre;
        pre += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = offs[gridDim.x];
}

u64 exclusive_scan_ws_words(u64 n) { return n <= (u64)SCAN_TILE * 16 ? 0 : (u64)ceil_div(n, SCAN_TILE) + 1; }

void exclusive_scan_u32_ws(const u32* in, u32* out, u64 n, u32* ws, hipStream_t s) {
    if (n <= (u64)SCAN_TILE * 16) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n);
        F4_LAUNCH_CHECK();
        return;
    }
    u32 tiles = ceil_div(n, SCAN_TILE);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, n, ws);
    F4_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN_THREADS), 0, s, ws, ws, (u64)tiles);
    F4_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, out, n, ws);
    F4_LAUNCH_CHECK();
}

void exclusive_scan_u32(const u32* in, u32* out, u64 n, Pool& pool, hipStream_t s) {
    const u64 w = exclusive_scan_ws_words(n);
    DBuf<u32> sums;
    if (w) sums.reset(&pool, w);
    exclusive_scan_u32_ws(in, out, n, sums.ptr, s);
}

// ------------------------------------------------------------- radix sort
#define RS_THREADS 256
#define RS_WAVES (RS_THREADS / F4_WAVE)

// Digit counts of a tile of RS_THREADS * items keys; hist is digit-major
// (digit d of tile b at d * nblocks + b) over the mask + 1 digits.
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const u64* keys, u64 n, u32 shift, u32 mask, u32 items,
                                                            u32* hist, u32 nblocks) {
    __shared__ u32 h[256];
    for (u32 i = threadIdx.x; i <= mask; i += RS_THREADS) h[i] = 0;
    __syncthreads();
    u64 base = (u64)blockIdx.x * RS_THREADS * items;
#pragma unroll 4
    for (u32 j = 0; j < items; ++j) {
        u64 i = base + (u64)j * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(u32)(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (u32 d = threadIdx.x; d <= mask; d += RS_THREADS) hist[(u64)d * nblocks + blockIdx.x] = h[d];
}

// Scatter with stable ranks.  A tile is consumed in `items` sub-rounds of
// RS_THREADS consecutive keys; inside a wave, lanes holding the same digit are
// found with 8 ballots (one per digit bit), which gives each key its rank among
// equal digits of lower lanes; per-wave digit counts in LDS order the waves.
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const u64* kin, const u32* vin, u64* kout, u32* vout,
                                                               u64 n, u32 shift, u32 mask, u32 items,
                                                               const u32* offs, u32 nblocks) {
    __shared__ u32 run[256];
    __shared__ u32 wcnt[RS_WAVES][256];
    const u32 tid = threadIdx.x, wave = tid / F4_WAVE, lane = lane_id();
    for (u32 d = tid; d <= mask; d += RS_THREADS) run[d] = offs[(u64)d * nblocks + blockIdx.x];
    const u64 base = (u64)blockIdx.x * RS_THREADS * items;
    const u64 lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (u32 j = 0; j < items; ++j) {
        for (u32 q = tid; q < RS_WAVES * 256; q += RS_THREADS) (&wcnt[0][0])[q] = 0;
        __syncthreads();
        const u64 i = base + (u64)j * RS_THREADS + tid;
        const bool valid = i < n;
        const u64 key = valid ? kin[i] : 0;
        const u32 d = (u32)(key >> shift) & mask;
        u64 m = wave_ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const u64 bb = wave_ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const u32 rank = __popcll(m & lt);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            u32 pos = run[d] + rank;
            for (u32 w2 = 0; w2 < wave; ++w2) pos += wcnt[w2][d];
            kout[pos] = key;
            if (vout) vout[pos] = vin[i];
        }
        __syncthreads();
        for (u32 dd = tid; dd <= mask; dd += RS_THREADS) {
            u32 t = 0;
            for (u32 w2 = 0; w2 < RS_WAVES; ++w2) t += wcnt[w2][dd];
            run[dd] += t;
        }
        __syncthreads();
    }
}

// Sorts of at most SS_MAX pairs in one workgroup: keys and values stay in LDS
// (double buffered) for every digit pass; each pass is a digit histogram, a
// scan of the digit counts, then the keys in order in sub-rounds of SS_THREADS
// with the same stable in-wave ranks (8 ballots) as k_radix_scatter.
#define SS_THREADS 1024
#define SS_WAVES (SS_THREADS / F4_WAVE)
#define SS_MAX SORT_SMALL_MAX
__global__ __launch_bounds__(SS_THREADS) void k_sort_small(u64* keys, u32* vals, u32 n, u32 lo_bit, u32 hi_bit,
                                                           u32 digit) {
    extern __shared__ u64 ss_mem[];
    u64* ka = ss_mem;
    u64* kb = ka + SS_MAX;
    u32* va = (u32*)(kb + SS_MAX);
    u32* vb = va + SS_MAX;
    __shared__ u32 run[256];
    __shared__ u32 wcnt[SS_WAVES * 256];
    __shared__ u32 s_wave[33];
    const u32 tid = threadIdx.x;
    for (u32 i = tid; i < n; i += SS_THREADS) {
        ka[i] = keys[i];
        if (vals) va[i] = vals[i];
    }
    const bool sw = lds_radix_sort(ka, kb, vals ? va : nullptr, vb, n, lo_bit, hi_bit, digit, SS_THREADS, run, wcnt,
                                   s_wave);
    const u64* rk = sw ? kb : ka;
    const u32* rv = sw ? vb : va;
    for (u32 i = tid; i < n; i += SS_THREADS) {
        keys[i] = rk[i];
        if (vals) vals[i] = rv[i];
    }
}

static void radix_sort_impl(u64* keys, u32* vals, u64 n, u32 lo_bit, u32 hi_bit, Pool& pool, hipStream_t s,
                            SortPlan plan) {
    if (n <= 1 || hi_bit <= lo_bit) return;
    if (plan.digit < 1 || plan.digit > 8 || plan.items < 1 || plan.items > 64)
        throw F4Error{1, "radix sort plan out of range"};
    const u32 digit = plan.digit;
    if (n <= SS_MAX) {
        const size_t lds = (size_t)SS_MAX * (2 * sizeof(u64) + 2 * sizeof(u32));
        hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(SS_THREADS), lds, s, keys, vals, (u32)n, lo_bit, hi_bit,
                           digit);
        F4_LAUNCH_CHECK();
        return;
    }
    const u32 nblocks = ceil_div(n, (u64)RS_THREADS * plan.items);
    DBuf<u64> k2(&pool, n);
    DBuf<u32> v2;
    if (vals) v2.reset(&pool, n);
    DBuf<u32> hist(&pool, ((u64)1 << digit) * nblocks + 1);
    u64 *ka = keys, *kb = k2.ptr;
    u32 *va = vals, *vb = v2.ptr;
    for (u32 shift = lo_bit; shift < hi_bit; shift += digit) {
        const u32 bits = (hi_bit - shift) < digit ? (hi_bit - shift) : digit;
        const u32 mask = (1u << bits) - 1;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(RS_THREADS), 0, s, ka, n, shift, mask, plan.items,
                           hist.ptr, nblocks);
        F4_LAUNCH_CHECK();
        exclusive_scan_u32(hist.ptr, hist.ptr, ((u64)mask + 1) * nblocks, pool, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, ka, va, kb, vb, n, shift, mask,
                           plan.items, hist.ptr, nblocks);
        F4_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        F4_HIP_TRY(hipMemcpyAsync(keys, ka, n * sizeof(u64), hipMemcpyDeviceToDevice, s));
        if (vals) F4_HIP_TRY(hipMemcpyAsync(vals, va, n * sizeof(u32), hipMemcpyDeviceToDevice, s));
    }
}

void radix_sort_pairs(u64* keys, u32* vals, u64 n, u32 lo_bit, u32 hi_bit, Pool& pool, hipStream_t s,
                      SortPlan plan) {
    radix_sort_impl(keys, vals, n, lo_bit, hi_bit, pool, s, plan);
}
void radix_sort_keys(u64* keys, u64 n, u32 lo_bit, u32 hi_bit, Pool& pool, hipStream_t s, SortPlan plan) {
    radix_sort_impl(keys, nullptr, n, lo_bit, hi_bit, pool, s, plan);
}

// Candidates: digit widths 5..8 (pass count and histogram size), and for the
// multi-workgroup passes 8 or 16 keys per thread (tile size against grid
// size).  A sort of at most 8 bits is one pass whatever the width.
void tuned_sort(Ctx& c, u64* keys, u32* vals, u64 n, u32 lo_bit, u32 hi_bit) {
    if (n <= 1 || hi_bit <= lo_bit) return;
    SortPlan plan;
    const u32 bits = hi_bit - lo_bit;
    if (c.tune.force_digit) {
        plan.digit = c.tune.force_digit;
    } else if (c.tune.on && bits > 8) {
        const bool multi = n > SS_MAX;
        std::vector<u32> cands;
        for (u32 d = 5; d <= 8; ++d) {
            if (multi) cands.push_back(d | (8u << 8));
            cands.push_back(d | (16u << 8));
        }
        const u64 key = tune_key(TUNE_SORT, vals ? 1 : 0, tune_lg(n), bits);
        DBuf<u64> kc;
        DBuf<u32> vc;
        const u32 pick = tune_pick(
            c, key, cands,
            [&](u32) {
                if (!kc.ptr) {
                    kc.reset(&c.pool, n);
                    if (vals) vc.reset(&c.pool, n);
                }
                F4_HIP_TRY(hipMemcpyAsync(kc.ptr, keys, n * sizeof(u64), hipMemcpyDeviceToDevice, c.stream));
                if (vals)
                    F4_HIP_TRY(hipMemcpyAsync(vc.ptr, vals, n * sizeof(u32), hipMemcpyDeviceToDevice, c.stream));
            },
            [&](u32 ch) {
                SortPlan pl;
                pl.digit = ch & 0xffu;
                pl.items = ch >> 8;
                radix_sort_impl(kc.ptr, vals ? vc.ptr : nullptr, n, lo_bit, hi_bit, c.pool, c.stream, pl);
            });
        plan.digit = pick & 0xffu;
        plan.items = pick >> 8;
    }
    radix_sort_impl(keys, vals, n, lo_bit, hi_bit, c.pool, c.stream, plan);
}

// ------------------------------------------------------------------ unique
__global__ void k_head_flags(const u64* k, u64 n, u32* f) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        f[i] = (i == 0 || k[i] != k[i - 1]) ? 1u : 0u;
}
__global__ void k_compact_heads(const u64* k, u64 n, const u32* pos, u64* out, u32* d_count) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        if (i == 0 || k[i] != k[i - 1]) out[pos[i]] = k[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) *d_count = pos[n];
}

void unique_sorted_u64(const u64* keys, u64 n, u64* out, u32* d_count, Pool& pool, hipStream_t s) {
    if (n == 0) {
        fill_u32(d_count, 1, 0, s);
        return;
    }
    DBuf<u32> f(&pool, n + 1);
    u32 blocks = ceil_div(n, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_head_flags, dim3(blocks), dim3(256), 0, s, keys, n, f.ptr);
    F4_LAUNCH_CHECK();
    exclusive_scan_u32(f.ptr, f.ptr, n, pool, s);
    hipLaunchKernelGGL(k_compact_heads, dim3(blocks), dim3(256), 0, s, keys, n, f.ptr, out, d_count);
    F4_LAUNCH_CHECK();
}
