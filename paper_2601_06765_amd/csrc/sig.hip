// Signature admissibility in bulk (section "Discussion: Integrating
// Signatures, Admissibility, and GPU Scheduling"): the predicate of every
// candidate row evaluated as a data-parallel map over row metadata, the
// survivors compacted by an exclusive scan in input order, and a schedule of
// them bucketed by (row degree, length of g_k, signature index) by a radix
// sort of unique keys (the position breaks ties).  The predicate itself (syzygy and rewrite tests) is in sig.hpp,
// shared with the reducer search of the symbolic preprocessing.
#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "sig.hpp"

#define SIG_SLOTS 64  // copies of the filter's counters, 4 words each

// flags of rows (t, k) read with strides (an array of records or two arrays);
// LDS: the signature tables are first copied to LDS (the host checks that they
// fit: see sig_lds_bytes)
template <bool LDS>
__global__ void k_sig_flags(const SigDev* __restrict__ Sp, const u64* __restrict__ t, u32 ts,
                            const u32* __restrict__ k, u32 ks, u32 r, u32* __restrict__ keep, u8* __restrict__ flags,
                            u32* __restrict__ info) {
    extern __shared__ u64 sg_mem[];
    const SigDev S = *Sp;
    const u32 np = S.npolys, ni = S.nindex, nsyz = S.syz_off[ni];
    const u32 *sidx = S.sidx, *soff = S.syz_off, *roff = S.rw_off, *rwk = S.rw_k;
    const u64 *smon = S.smon, *syzm = S.syz_mon, *rwm = S.rw_mon;
    if (LDS) {
        u64* l_smon = sg_mem;
        u64* l_syzm = l_smon + np;
        u64* l_rwm = l_syzm + nsyz;
        u32* l_sidx = (u32*)(l_rwm + np);
        u32* l_soff = l_sidx + np;
        u32* l_roff = l_soff + ni + 1;
        u32* l_rwk = l_roff + ni + 1;
        for (u32 x = threadIdx.x; x < np; x += blockDim.x) {
            l_smon[x] = S.smon[x];
            l_rwm[x] = S.rw_mon[x];
            l_sidx[x] = S.sidx[x];
            l_rwk[x] = S.rw_k[x];
        }
        for (u32 x = threadIdx.x; x < nsyz; x += blockDim.x) l_syzm[x] = S.syz_mon[x];
        for (u32 x = threadIdx.x; x <= ni; x += blockDim.x) {
            l_soff[x] = S.syz_off[x];
            l_roff[x] = S.rw_off[x];
        }
        __syncthreads();
        sidx = l_sidx;
        soff = l_soff;
        roff = l_roff;
        rwk = l_rwk;
        smon = l_smon;
        syzm = l_syzm;
        rwm = l_rwm;
    }
    u32 cnt[3] = {0, 0, 0};
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < r; q += gridDim.x * blockDim.x) {
        const u32 f = sig_adm_thread(S, sidx, smon, soff, syzm, roff, rwk, rwm, t[(u64)q * ts], k[(u64)q * ks]);
        if (flags) flags[q] = (u8)f;
        keep[q] = f == SIG_OK ? 1u : 0u;
        if (f == SIG_OVERFLOW)
            atomicOr(&info[4 * (blockIdx.x % SIG_SLOTS)], 1u);
        else
            ++cnt[f];
    }
    // survivors, syzygy rejections, rewritten rows: summed over the wave, then
    // added to one of SIG_SLOTS copies of the counters (block b uses copy
    // b mod SIG_SLOTS: atomics on one word serialise, spread ones do not); the
    // host adds the copies up
    for (int c = 0; c < 3; ++c) {
        u32 v = cnt[c];
        for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) v += __shfl_down(v, d, F4_WAVE);
        if ((threadIdx.x & (F4_WAVE - 1)) == 0 && v) atomicAdd(&info[4 * (blockIdx.x % SIG_SLOTS) + 1 + c], v);
    }
}

// the survivors, in input order, at their exclusive-scan positions
__global__ void k_sig_scatter(const u64* __restrict__ t, u32 ts, const u32* __restrict__ k, u32 ks, u32 r,
                              const u32* __restrict__ keep, const u32* __restrict__ pos, u64* __restrict__ t2,
                              u32* __restrict__ k2, u32* __restrict__ count) {
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < r; q += gridDim.x * blockDim.x) {
        if (keep[q]) {
            t2[pos[q]] = t[(u64)q * ts];
            k2[pos[q]] = k[(u64)q * ks];
        }
        if (q == r - 1) *count = pos[q] + keep[q];
    }
}

// bucket key of each survivor, unique: from the top, the degree of
// t * LM(g_k), the length of g_k (saturated at 2^16 - 1), the signature index
// (saturated at 2^12 - 1), then the survivor's position (ties keep input
// order); each field as wide as the call's largest value needs
struct SigKeyBits {
    u32 pos, ix, len;  // shifts of the index, length and degree fields
};
#define SIG_POS_BITS 28
__global__ void k_sig_bucket(const u64* __restrict__ t2, const u32* __restrict__ k2, const u32* __restrict__ count,
                             const u64* __restrict__ lm, const u32* __restrict__ len,
                             const u32* __restrict__ sidx, SigKeyBits kb, u64* __restrict__ keys,
                             u32* __restrict__ vals) {
    const u32 r = *count;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < r; q += gridDim.x * blockDim.x) {
        const u32 k = k2[q];
        const u64 deg = min(mono_deg(t2[q]) + mono_deg(lm[k]), 255u);
        const u64 l = min(len[k], 0xffffu);
        const u64 ix = min(sidx[k], 0xfffu);
        keys[q] = (deg << kb.len) | (l << kb.ix) | (ix << kb.pos) | q;
        vals[q] = q;
    }
}

void sig_upload(Ctx& c, u32 n, u32 npolys, const u32* index, const u64* mon, u32 nindex, const u32* syz_off,
                const u64* syz_mon, SigBufs& out) {
    if (!index || !mon || !syz_off || nindex == 0 || nindex > (1u << 20)) throw F4Error{1, "bad signatures"};
    const u32 w = lane_bits(n);
    const u64 lanes = (n * w >= 64) ? ~0ull : ((1ull << (n * w)) - 1);
    auto mono_ok = [&](u64 P) {
        if (P & ~(lanes | (0xffull << 56))) return false;
        u32 d = 0;
        for (u32 i = 0; i < n; ++i) d += mono_exp(P, i, w);
        return d == mono_deg(P);
    };
    if (syz_off[0] != 0) throw F4Error{1, "bad syzygy offsets"};
    for (u32 i = 0; i < nindex; ++i)
        if (syz_off[i + 1] < syz_off[i]) throw F4Error{1, "bad syzygy offsets"};
    const u32 nsyz = syz_off[nindex];
    if (nsyz && !syz_mon) throw F4Error{1, "bad signatures"};
    for (u32 q = 0; q < nsyz; ++q)
        if (!mono_ok(syz_mon[q])) throw F4Error{1, "a syzygy monomial is not a monomial of n variables"};
    // elements grouped by index, ascending
    std::vector<u32> rw_off(nindex + 1, 0), rw_k(npolys);
    std::vector<u64> rw_mon(npolys);
    for (u32 k = 0; k < npolys; ++k) {
        if (index[k] >= nindex) throw F4Error{1, "signature index out of range"};
        if (!mono_ok(mon[k])) throw F4Error{1, "a signature monomial is not a monomial of n variables"};
        ++rw_off[index[k] + 1];
    }
    for (u32 i = 0; i < nindex; ++i) rw_off[i + 1] += rw_off[i];
    {
        std::vector<u32> fill(rw_off.begin(), rw_off.end() - 1);
        for (u32 k = 0; k < npolys; ++k) {
            const u32 x = fill[index[k]]++;
            rw_k[x] = k;
            rw_mon[x] = mon[k];
        }
    }
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_desc = 0, o_sidx = al(sizeof(SigDev)), o_smon = o_sidx + al((size_t)npolys * 4),
                 o_soff = o_smon + al((size_t)npolys * 8), o_smn = o_soff + al(((size_t)nindex + 1) * 4),
                 o_roff = o_smn + al(std::max<size_t>(nsyz, 1) * 8), o_rk = o_roff + al(((size_t)nindex + 1) * 4),
                 o_rmon = o_rk + al((size_t)npolys * 4), total = o_rmon + al((size_t)npolys * 8);
    out.blob.reset(&c.pool, total);
    u8* b = out.blob.ptr;
    SigDev d;
    std::memset(&d, 0, sizeof(d));
    d.sidx = (const u32*)(b + o_sidx);
    d.smon = (const u64*)(b + o_smon);
    d.syz_off = (const u32*)(b + o_soff);
    d.syz_mon = (const u64*)(b + o_smn);
    d.rw_off = (const u32*)(b + o_roff);
    d.rw_k = (const u32*)(b + o_rk);
    d.rw_mon = (const u64*)(b + o_rmon);
    d.nindex = nindex;
    d.npolys = npolys;
    d.n = n;
    d.w = w;
    d.lanes = lanes;
    d.H = 0;
    for (u32 i = 0; i < n; ++i) d.H |= 1ull << (w * i + w - 1);
    std::vector<u8> host(total, 0);
    std::memcpy(host.data() + o_desc, &d, sizeof(d));
    std::memcpy(host.data() + o_sidx, index, (size_t)npolys * 4);
    std::memcpy(host.data() + o_smon, mon, (size_t)npolys * 8);
    std::memcpy(host.data() + o_soff, syz_off, ((size_t)nindex + 1) * 4);
    if (nsyz) std::memcpy(host.data() + o_smn, syz_mon, (size_t)nsyz * 8);
    std::memcpy(host.data() + o_roff, rw_off.data(), ((size_t)nindex + 1) * 4);
    std::memcpy(host.data() + o_rk, rw_k.data(), (size_t)npolys * 4);
    std::memcpy(host.data() + o_rmon, rw_mon.data(), (size_t)npolys * 8);
    upload(c, b, host.data(), total);
    out.dev = (const SigDev*)(b + o_desc);
    out.sidx = d.sidx;
    out.lds_bytes = (size_t)npolys * 24 + (size_t)nsyz * 8 + ((size_t)nindex + 1) * 8;
    out.nindex = nindex;
}

void sig_filter_dev(Ctx& c, const SigBufs& S, const u64* t, u32 ts, const u32* k, u32 ks, u32 r, u8* flags,
                    DBuf<u64>& t2, DBuf<u32>& k2, DBuf<u32>& count, u32 info_out[4]) {
    hipStream_t s = c.stream;
    DBuf<u32> keep(&c.pool, std::max<u32>(r, 1)), pos(&c.pool, std::max<u32>(r, 1)), info(&c.pool, 4 * SIG_SLOTS);
    fill_u32(info.ptr, 4 * SIG_SLOTS, 0, s);
    t2.reset(&c.pool, std::max<u32>(r, 1));
    k2.reset(&c.pool, std::max<u32>(r, 1));
    count.reset(&c.pool, 1);
    fill_u32(count.ptr, 1, 0, s);
    if (r) {
        const u32 grid = std::min<u32>(4096, ceil_div(r, 256));
        if (S.lds_bytes <= 48 * 1024)
            hipLaunchKernelGGL(k_sig_flags<true>, dim3(grid), dim3(256), S.lds_bytes, s, S.dev, t, ts, k, ks, r,
                               keep.ptr, flags, info.ptr);
        else
            hipLaunchKernelGGL(k_sig_flags<false>, dim3(grid), dim3(256), 0, s, S.dev, t, ts, k, ks, r, keep.ptr,
                               flags, info.ptr);
        F4_LAUNCH_CHECK();
        exclusive_scan_u32(keep.ptr, pos.ptr, r, c.pool, s);
        hipLaunchKernelGGL(k_sig_scatter, dim3(grid), dim3(256), 0, s, t, ts, k, ks, r, keep.ptr, pos.ptr, t2.ptr,
                           k2.ptr, count.ptr);
        F4_LAUNCH_CHECK();
    }
    u32 slots[4 * SIG_SLOTS];
    readback(c, slots, info.ptr, sizeof(slots));
    for (int w = 0; w < 4; ++w) info_out[w] = 0;
    for (int q = 0; q < SIG_SLOTS; ++q) {
        info_out[0] |= slots[4 * q];
        for (int w = 1; w < 4; ++w) info_out[w] += slots[4 * q + w];
    }
    if (info_out[0]) throw F4Error{2, "a row's signature overflows an exponent lane"};
}

static u32 sig_bits(u64 x) {
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

void sig_schedule_dev(Ctx& c, const SigBufs& S, const u64* t2, const u32* k2, const u32* count, u32 nkept,
                      u32 max_deg, u32 max_len, const u64* lm, const u32* len, DBuf<u32>& order) {
    hipStream_t s = c.stream;
    order.reset(&c.pool, std::max<u32>(nkept, 1));
    if (!nkept) return;
    if (nkept >= (1u << SIG_POS_BITS)) throw F4Error{2, "too many rows to schedule"};
    SigKeyBits kb;
    kb.pos = sig_bits(nkept - 1);
    kb.ix = kb.pos + sig_bits(std::min<u32>(S.nindex, 1u << 12) - 1);
    kb.len = kb.ix + sig_bits(std::min<u32>(max_len, 0xffffu));
    const u32 hi = kb.len + sig_bits(std::min<u32>(max_deg, 255u));
    DBuf<u64> keys(&c.pool, nkept);
    const u32 grid = std::min<u32>(4096, ceil_div(nkept, 256));
    hipLaunchKernelGGL(k_sig_bucket, dim3(grid), dim3(256), 0, s, t2, k2, count, lm, len, S.sidx, kb, keys.ptr,
                       order.ptr);
    F4_LAUNCH_CHECK();
    radix_sort_pairs(keys.ptr, order.ptr, nkept, 0, std::max<u32>(hi, 1), c.pool, s);
}
