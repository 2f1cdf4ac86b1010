// Radix sort of a small array held in LDS by one workgroup.
#pragma once

#include "common.hpp"

// Stable LSD radix sort of n (key, value) pairs (values optional: va == nullptr,
// then vb is never touched) already in LDS, on key bits [lo_bit, hi_bit),
// `digit` bits per pass, by one
// workgroup of `threads` threads (a multiple of the wave size, at most 1024).
// Each pass: a histogram of the digits, a scan of the counts, then the keys in
// order in sub-rounds of `threads`, each key ranked among equal digits of
// lower lanes with 8 ballots and placed after the waves before it (per-wave
// counts in wcnt, threads / 64 rows of 256).  The buffers alternate between
// passes; returns whether the result is in (kb, vb).  run: 256 words,
// s_wave: 33 words of LDS.
__device__ inline bool lds_radix_sort(u64* ka, u64* kb, u32* va, u32* vb, u32 n, u32 lo_bit, u32 hi_bit, u32 digit,
                                      u32 threads, u32* run, u32* wcnt, u32* s_wave) {
    const u32 tid = threadIdx.x, wave = tid / F4_WAVE, lane = lane_id(), nwaves = threads / F4_WAVE;
    const u64 lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const bool has_vals = va != nullptr;  // fixed here: the buffers swap every pass
    bool swapped = false;
    for (u32 shift = lo_bit; shift < hi_bit; shift += digit) {
        const u32 bits = (hi_bit - shift) < digit ? (hi_bit - shift) : digit;
        const u32 mask = (1u << bits) - 1;
        if (tid < 256) run[tid] = 0;
        __syncthreads();
        for (u32 i = tid; i < n; i += threads) atomicAdd(&run[(u32)(ka[i] >> shift) & mask], 1u);
        __syncthreads();
        {
            u32 tot;
            const u32 c = tid < 256 ? run[tid] : 0u;
            const u32 pre = block_exclusive_scan(c, s_wave, &tot);
            if (tid < 256) run[tid] = pre;
        }
        __syncthreads();
        for (u32 j0 = 0; j0 < n; j0 += threads) {
            for (u32 q = tid; q < nwaves * 256; q += threads) wcnt[q] = 0;
            __syncthreads();
            const u32 i = j0 + tid;
            const bool valid = i < n;
            const u64 key = valid ? ka[i] : 0;
            const u32 d = (u32)(key >> shift) & mask;
            u64 m = wave_ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1;
                const u64 bb = wave_ballot(bit);
                m &= bit ? bb : ~bb;
            }
            const u32 rank = __popcll(m & lt);
            if (valid && rank == 0) wcnt[wave * 256 + d] = __popcll(m);
            __syncthreads();
            if (valid) {
                u32 pos = run[d] + rank;
                for (u32 w2 = 0; w2 < wave; ++w2) pos += wcnt[w2 * 256 + d];
                kb[pos] = key;
                if (has_vals) vb[pos] = va[i];
            }
            __syncthreads();
            if (tid < 256) {
                u32 t = 0;
                for (u32 w2 = 0; w2 < nwaves; ++w2) t += wcnt[w2 * 256 + tid];
                run[tid] += t;
            }
            __syncthreads();
        }
        u64* tk = ka;
        ka = kb;
        kb = tk;
        if (has_vals) {
            u32* tv = va;
            va = vb;
            vb = tv;
        }
        swapped = !swapped;
    }
    return swapped;
}
