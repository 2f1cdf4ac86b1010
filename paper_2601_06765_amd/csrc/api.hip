// C-ABI (include/f4.h), context management and the F4 driver loop.
//
// The driver keeps the basis G on the device in structure-of-arrays form
// (section "Coalesced sparse polynomial storage: SoA support vectors") and
// only its leading monomials on the host, where the pair bookkeeping runs:
// the Gebauer-Moeller update (pair criteria of the batch selection stage,
// pipeline step "Batch selection (algebraic control)") and the normal
// selection strategy (all pairs of minimal lcm degree).  Each step then runs
// SP on the device (build.hip), the elimination (reduce.hip), and appends the
// reduced trailing rows to G on the device (pipeline step "Reconstruction").
#include <functional>
#include <algorithm>
#include <exception>
#include <mutex>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <set>

#include "../../include/f4.h"
#include "internal.hpp"
#include "mw.hpp"

// ------------------------------------------------------------ handles
struct f4_matrix;
struct f4_reduced;
struct f4_basis;
struct f4_server;
struct f4_ctx {
    Ctx c;
    std::set<f4_matrix*> matrices;
    std::set<f4_reduced*> reduceds;
    std::set<f4_basis*> bases;
    std::set<f4_server*> servers;
};
struct f4_matrix {
    f4_ctx* owner;
    Matrix m;
    // CSR of the transpose, built by the first transposed f4_spmm call
    DBuf<u32> t_ptr, t_idx, t_val;
    bool has_t = false;
    SchedBufs sched;  // block schedule (f4_matrix_schedule)
};
struct f4_reduced {
    f4_ctx* owner;
    Reduced r;
};
struct f4_basis {
    f4_ctx* owner;
    u32 n = 0;
    std::vector<u64> mon, off;
    std::vector<u32> coeff;
    std::vector<f4_step_stats> steps;
};

// ------------------------------------------------------------ staging
u8* staging(Ctx& c, size_t bytes) {
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (c.pinned_used + need > c.pinned_bytes) {
        // wrap around: every copy out of the arena must have finished
        if (c.staging_pending) {
            F4_HIP_TRY(hipEventSynchronize(c.staging_done));
            c.staging_pending = false;
        }
        c.pinned_used = 0;
        if (need > c.pinned_bytes) {
            const size_t nb = std::max(need, (size_t)2 * c.pinned_bytes);
            if (c.pinned) F4_HIP_TRY(hipHostFree(c.pinned));
            c.pinned = nullptr;
            c.pinned_bytes = 0;
            F4_HIP_TRY(hipHostMalloc((void**)&c.pinned, nb, hipHostMallocDefault));
            c.pinned_bytes = nb;
        }
    }
    u8* p = c.pinned + c.pinned_used;
    c.pinned_used += need;
    return p;
}

void upload(Ctx& c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (bytes > (16u << 20)) {  // large: pageable copy, synchronous w.r.t. the host buffer
        F4_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream));
        F4_HIP_TRY(hipStreamSynchronize(c.stream));
        return;
    }
    u8* st = staging(c, bytes);
    std::memcpy(st, src, bytes);
    F4_HIP_TRY(hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, c.stream));
    F4_HIP_TRY(hipEventRecord(c.staging_done, c.stream));
    c.staging_pending = true;
}

void readback(Ctx& c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    u8* st = staging(c, bytes);
    F4_HIP_TRY(hipMemcpyAsync(st, src, bytes, hipMemcpyDeviceToHost, c.stream));
    F4_HIP_TRY(hipStreamSynchronize(c.stream));
    std::memcpy(dst, st, bytes);
    // the stream is idle: no copy uses the arena any more
    c.staging_pending = false;
    c.pinned_used = 0;
}

bool timing_on(const Ctx& c) { return (c.flags & F4_OPT_TIMING) != 0; }
bool kernel_timing_on(const Ctx& c) { return (c.flags & F4_OPT_KERNEL_TIMING) != 0; }

hipEvent_t stage_event(Ctx& c) {
    if (!(c.flags & F4_OPT_TIMING)) return nullptr;
    if (c.ev_used == c.events.size()) {
        hipEvent_t e;
        F4_HIP_TRY(hipEventCreate(&e));
        c.events.push_back(e);
    }
    hipEvent_t e = c.events[c.ev_used++];
    F4_HIP_TRY(hipEventRecord(e, c.stream));
    return e;
}

hipEvent_t kernel_event(Ctx& c) {
    if (!(c.flags & F4_OPT_KERNEL_TIMING)) return nullptr;
    const u32 keep = c.flags;
    c.flags |= F4_OPT_TIMING;
    hipEvent_t e = nullptr;
    try {
        e = stage_event(c);
    } catch (...) {
        c.flags = keep;
        throw;
    }
    c.flags = keep;
    return e;
}

float event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    if (a && b) F4_HIP_TRY(hipEventElapsedTime(&ms, a, b));
    return ms;
}

#include "pairs.hpp"
#include "workpool.hpp"

// Per-system host work of a batch iteration (pair selection, pair updates):
// independent per system, so large batches spread it over the context's
// host threads (up to 8 with the caller); the first error is rethrown.
static void for_systems(Ctx& c, size_t n, const std::function<void(size_t)>& f) {
    if (n < 8) {
        for (size_t i = 0; i < n; ++i) f(i);
        return;
    }
    if (!c.cpu) {
        unsigned hw = std::thread::hardware_concurrency();
        if (hw == 0) hw = 1;
        c.cpu = new WorkPool(std::min(hw, 8u) - 1);
    }
    std::mutex em;
    std::exception_ptr first;
    c.cpu->run((unsigned)n, [&](unsigned i) {
        try {
            f(i);
        } catch (...) {
            std::lock_guard<std::mutex> g(em);
            if (!first) first = std::current_exception();
        }
    });
    if (first) std::rethrow_exception(first);
}

struct DevG {
    u32 n = 0, npolys = 0;
    u64 nterms = 0;
    DBuf<u64> mon, off, lm;
    DBuf<u32> coeff, len;
    DBuf<u32> act;  // activity flags (pair sets on the device)
    u64 cap_terms = 0, cap_polys = 0;
};

__global__ void k_basis_meta(const u64* mon, const u64* off, u32 a, u32 b, u64* lm, u32* len) {
    for (u32 k = a + blockIdx.x * blockDim.x + threadIdx.x; k < b; k += gridDim.x * blockDim.x) {
        lm[k] = mon[off[k]];
        len[k] = (u32)(off[k + 1] - off[k]);
    }
}

// append the echelon rows (CSR over the matrix columns) as new basis elements
__global__ void k_append(const u32* rptr, const u32* rcol, const u32* rval, u32 rho, const u64* dict_keys,
                         u64 term_base, u32 poly_base, u64* mon, u32* coeff, u64* off) {
    const u32 nnz = rptr[rho];
    for (u32 e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
        mon[term_base + e] = dict_keys[rcol[e]];
        coeff[term_base + e] = rval[e];
    }
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t <= rho; t += gridDim.x * blockDim.x)
        off[poly_base + t] = term_base + rptr[t];
}

static u32 gridn(u64 items, u32 per, u32 cap) {
    u64 g = (items + per - 1) / per;
    return (u32)std::max<u64>(1, std::min<u64>(g, cap));
}

// Device copies deferred to one launch (k_copy_jobs): the basis arrays of
// many systems regrow in the same iteration.  The replaced buffers are kept
// until the copies are enqueued, so the pool cannot hand them out before.
struct CopyJob {
    const u32* src;
    u32* dst;
    u64 words;
};
struct CopyBatch {
    std::vector<CopyJob> jobs;
    std::vector<DBuf<u64>> keep64;
    std::vector<DBuf<u32>> keep32;
};

__global__ void k_copy_jobs(const CopyJob* jobs) {
    const CopyJob J = jobs[blockIdx.y];
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < J.words; i += (u64)gridDim.x * blockDim.x)
        J.dst[i] = J.src[i];
}

static void copy_flush(Ctx& c, CopyBatch& cb) {
    if (!cb.jobs.empty()) {
        if (cb.jobs.size() > 65535) throw F4Error{2, "too many deferred copies"};
        DBuf<u8> d(&c.pool, cb.jobs.size() * sizeof(CopyJob));
        upload(c, d.ptr, cb.jobs.data(), cb.jobs.size() * sizeof(CopyJob));
        u64 mx = 1;
        for (const CopyJob& j : cb.jobs) mx = std::max(mx, j.words);
        hipLaunchKernelGGL(k_copy_jobs, dim3(gridn(mx, 256, 256), (u32)cb.jobs.size()), dim3(256), 0, c.stream,
                           (const CopyJob*)d.ptr);
        F4_LAUNCH_CHECK();
    }
    cb = CopyBatch();  // the replaced buffers go back to the pool after the copies were enqueued
}

// Grow the basis arrays to hold `terms` terms and `polys` polynomials (4x
// steps).  With `cb`, the copies of the existing contents are deferred to
// copy_flush; otherwise they are enqueued at once.
static void devg_reserve(Ctx& c, DevG& G, u64 terms, u32 polys, CopyBatch* cb = nullptr) {
    auto copy = [&](const void* src, void* dst, u64 bytes) {
        if (!bytes) return;
        if (cb)
            cb->jobs.push_back({(const u32*)src, (u32*)dst, bytes / 4});
        else
            F4_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.stream));
    };
    if (terms > G.cap_terms) {
        u64 cap = std::max<u64>(terms, 4 * G.cap_terms);  // few regrowths: each copies the basis
        DBuf<u64> m2(&c.pool, cap);
        DBuf<u32> c2(&c.pool, cap);
        copy(G.mon.ptr, m2.ptr, G.nterms * 8);
        copy(G.coeff.ptr, c2.ptr, G.nterms * 4);
        if (cb) {
            cb->keep64.push_back(std::move(G.mon));
            cb->keep32.push_back(std::move(G.coeff));
        }
        G.mon = std::move(m2);
        G.coeff = std::move(c2);
        G.cap_terms = cap;
    }
    if ((u64)polys + 1 > G.cap_polys) {
        u64 cap = std::max<u64>((u64)polys + 1, 4 * G.cap_polys);
        DBuf<u64> o2(&c.pool, cap), l2(&c.pool, cap);
        DBuf<u32> n2(&c.pool, cap), a2(&c.pool, cap);
        if (G.npolys) {
            copy(G.off.ptr, o2.ptr, ((u64)G.npolys + 1) * 8);
            copy(G.lm.ptr, l2.ptr, (u64)G.npolys * 8);
            copy(G.len.ptr, n2.ptr, (u64)G.npolys * 4);
            if (G.act.ptr) copy(G.act.ptr, a2.ptr, (u64)G.npolys * 4);
        }
        if (cb) {
            cb->keep64.push_back(std::move(G.off));
            cb->keep64.push_back(std::move(G.lm));
            cb->keep32.push_back(std::move(G.len));
            cb->keep32.push_back(std::move(G.act));
        }
        G.off = std::move(o2);
        G.lm = std::move(l2);
        G.len = std::move(n2);
        G.act = std::move(a2);
        G.cap_polys = cap;
    }
}

static DevBasis devg_view(const DevG& G) {
    DevBasis b;
    b.n = G.n;
    b.w = lane_bits(G.n);
    b.npolys = G.npolys;
    b.mon = G.mon.ptr;
    b.coeff = G.coeff.ptr;
    b.off = G.off.ptr;
    b.lm = G.lm.ptr;
    b.len = G.len.ptr;
    return b;
}

static u32 powmod_host(u64 a, u64 e, u64 p) {
    u64 r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = r * a % p;
        a = a * a % p;
        e >>= 1;
    }
    return (u32)r;
}

static bool is_odd_prime(u32 p) {
    if (p < 3 || !(p & 1)) return false;
    for (u64 d = 3; d * d <= p; d += 2)
        if (p % d == 0) return false;
    return true;
}

static void set_stream(f4_ctx* X, void* stream) {
    hipStream_t s = stream ? (hipStream_t)stream : X->c.own_stream;
    if (X->c.stream && s != X->c.stream) F4_HIP_TRY(hipStreamSynchronize(X->c.stream));
    X->c.stream = s;
    X->c.ev_used = 0;
}

static int fail(f4_ctx* X, const F4Error& e) {
    if (X) X->c.last_error = e.msg;
    return e.code;
}

#define F4_API_BEGIN(ctx) \
    if (!(ctx)) return F4_E_ARG; \
    try {
#define F4_API_END(ctx)                                      \
    }                                                        \
    catch (const F4Error& e) {                               \
        return fail(ctx, e);                                 \
    }                                                        \
    catch (const std::bad_alloc&) {                          \
        return fail(ctx, F4Error{F4_E_NOMEM, "host allocation failed"}); \
    }                                                        \
    return F4_OK;

// Input terms of a basis given to the matrix builders (the f4_polys contract):
// every word a P word of n variables (no bits outside the lanes and the degree
// field, lanes adding up to the degree), terms of a polynomial in strictly
// decreasing grevlex order (so no monomial repeats), coefficients in [1, p),
// and, when `monic`, leading coefficients 1.  Error bits of the check:
enum : u32 { CHK_WORD = 1, CHK_ORDER = 2, CHK_COEFF = 4, CHK_MONIC = 8, CHK_EMPTY = 16 };

static const char* check_message(u32 bits) {
    if (bits & CHK_WORD) return "a term is not a monomial word of n variables";
    if (bits & CHK_ORDER) return "terms not in strictly decreasing grevlex order (unsorted or repeated)";
    if (bits & CHK_COEFF) return "a coefficient is 0 or not below p";
    if (bits & CHK_MONIC) return "a basis element is not monic";
    if (bits & CHK_EMPTY) return "zero polynomial in basis";
    return "bad basis";
}

__host__ __device__ static u32 check_term(u64 P, u32 c, u32 n, u32 w, u64 lanes, u32 p) {
    u32 bad = 0;
    if (P & ~(lanes | (0xffull << 56))) bad |= CHK_WORD;
    u32 d = 0;
    for (u32 i = 0; i < n; ++i) d += mono_exp(P, i, w);
    if (d != mono_deg(P)) bad |= CHK_WORD;
    if (c == 0 || c >= p) bad |= CHK_COEFF;
    return bad;
}

// host arrays: the error bits of every polynomial
static u32 check_polys_host(u32 n, u32 p, u32 npolys, const u64* mon, const u32* coeff, const u64* off, bool monic) {
    const u32 w = lane_bits(n);
    const u64 lanes = (1ull << (n * w)) - 1;
    u32 bad = 0;
    for (u32 k = 0; k < npolys; ++k) {
        if (off[k + 1] <= off[k]) {
            bad |= CHK_EMPTY;
            continue;
        }
        if (monic && coeff[off[k]] != 1) bad |= CHK_MONIC;
        for (u64 e = off[k]; e < off[k + 1]; ++e) {
            bad |= check_term(mon[e], coeff[e], n, w, lanes, p);
            if (e > off[k] && (mon[e] ^ lanes) >= (mon[e - 1] ^ lanes)) bad |= CHK_ORDER;
        }
    }
    return bad;
}

// device arrays: one wave per polynomial, error bits OR-ed into *flag
__global__ void k_check_polys(const u64* mon, const u32* coeff, const u64* off, u32 npolys, u32 n, u32 p, int monic,
                              u32* flag) {
    const u32 w = lane_bits(n);
    const u64 lanes = (1ull << (n * w)) - 1;
    const u32 lane = lane_id();
    u32 bad = 0;
    for (u32 k = (blockIdx.x * blockDim.x + threadIdx.x) / F4_WAVE; k < npolys;
         k += gridDim.x * blockDim.x / F4_WAVE) {
        const u64 a = off[k], b = off[k + 1];
        if (b <= a) {
            bad |= CHK_EMPTY;
            continue;
        }
        if (lane == 0 && monic && coeff[a] != 1) bad |= CHK_MONIC;
        for (u64 e = a + lane; e < b; e += F4_WAVE) {
            bad |= check_term(mon[e], coeff[e], n, w, lanes, p);
            if (e > a && (mon[e] ^ lanes) >= (mon[e - 1] ^ lanes)) bad |= CHK_ORDER;
        }
    }
    for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) bad |= __shfl_xor(bad, d, F4_WAVE);
    if (lane == 0 && bad) atomicOr(flag, bad);
}

// stored matrix values outside [1, p) set *flag
__global__ void k_check_vals(const u32* val, u64 nnz, u32 p, u32* flag) {
    bool bad = false;
    for (u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (u64)gridDim.x * blockDim.x)
        bad |= val[e] == 0 || val[e] >= p;
    if (__ballot(bad) && lane_id() == 0) atomicOr(flag, 1u);
}

// A basis given through the C-ABI, checked against the f4_polys contract and
// moved into device SoA with metadata.
static void load_polys(Ctx& c, u32 p, const f4_polys* G, DevG& D, bool monic) {
    if (!G || G->n == 0 || G->n > 14) throw F4Error{F4_E_ARG, "bad number of variables"};
    if (!G->offset || (G->npolys && (!G->mon || !G->coeff))) throw F4Error{F4_E_ARG, "null basis array"};
    D.n = G->n;
    std::vector<u64> off(G->npolys + 1);
    if (G->on_device)
        readback(c, off.data(), G->offset, off.size() * 8);
    else
        std::memcpy(off.data(), G->offset, off.size() * 8);
    if (off[0] != 0) throw F4Error{F4_E_ARG, "offsets must start at 0"};
    for (u32 k = 0; k < G->npolys; ++k)
        if (off[k + 1] <= off[k]) throw F4Error{F4_E_ARG, check_message(CHK_EMPTY)};
    const u64 nt = off[G->npolys];
    if (nt >= (1ull << 32)) throw F4Error{F4_E_RANGE, "basis has 2^32 or more terms"};
    if (!G->on_device) {
        const u32 bad = check_polys_host(G->n, p, G->npolys, G->mon, G->coeff, off.data(), monic);
        if (bad) throw F4Error{F4_E_ARG, check_message(bad)};
    }
    devg_reserve(c, D, nt, G->npolys);
    if (G->on_device) {
        F4_HIP_TRY(hipMemcpyAsync(D.mon.ptr, G->mon, nt * 8, hipMemcpyDeviceToDevice, c.stream));
        F4_HIP_TRY(hipMemcpyAsync(D.coeff.ptr, G->coeff, nt * 4, hipMemcpyDeviceToDevice, c.stream));
    } else {
        upload(c, D.mon.ptr, G->mon, nt * 8);
        upload(c, D.coeff.ptr, G->coeff, nt * 4);
    }
    upload(c, D.off.ptr, off.data(), off.size() * 8);
    D.npolys = G->npolys;
    D.nterms = nt;
    if (G->on_device && G->npolys) {
        DBuf<u32> flag(&c.pool, 1);
        fill_u32(flag.ptr, 1, 0, c.stream);
        hipLaunchKernelGGL(k_check_polys, dim3(gridn((u64)G->npolys * F4_WAVE, 256, 1024)), dim3(256), 0, c.stream,
                           D.mon.ptr, D.coeff.ptr, D.off.ptr, G->npolys, G->n, p, monic ? 1 : 0, flag.ptr);
        F4_LAUNCH_CHECK();
        u32 bad = 0;
        readback(c, &bad, flag.ptr, 4);
        if (bad) throw F4Error{F4_E_ARG, check_message(bad)};
    }
    if (G->npolys) {
        hipLaunchKernelGGL(k_basis_meta, dim3(gridn(G->npolys, 256, 1024)), dim3(256), 0, c.stream, D.mon.ptr,
                           D.off.ptr, 0u, G->npolys, D.lm.ptr, D.len.ptr);
        F4_LAUNCH_CHECK();
    }
}

static u32 deg_of(u64 P) { return (u32)(P >> 56); }

// Per-system state of the F4 loop.  The basis lives on the device, and so do
// the pair set and the activity flags (DevPairs, D.act); with the host-pairs
// option the host keeps them instead (P, active).  The host keeps a copy of
// the leading monomials either way (they come back with each step's sizes).
struct SysState {
    u32 n = 0, p = 0;
    MonoOps mo;
    DevG D;
    std::vector<u64> lm;
    std::vector<u8> active;
    std::vector<HPair> P;
    GmScratch gm;
    bool host_pairs = false;
    bool pairs_pending = false;  // inputs not yet in the device pair set
    DevPairs dp;
    bool unit = false, done = false;
    std::vector<f4_step_stats> steps;
    // reduced basis (host), filled at the end
    std::vector<u64> gmon, goff{0};
    std::vector<u32> gcoeff;
    // scratch of the current step
    std::vector<u64> rt;
    std::vector<u32> rk, act;
    u32 d = 0, nsel = 0;
    float tpairs = 0;
    std::chrono::steady_clock::time_point t0;
};

static bool has_pairs(const SysState& S) { return S.host_pairs ? !S.P.empty() : S.dp.kept > 0; }

// halves (t, k) deduplicated and sorted, active list (descending index)
static void prepare_rows(SysState& S, std::vector<std::pair<u64, u32>>& rows) {
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    S.rt.resize(rows.size());
    S.rk.resize(rows.size());
    for (size_t i = 0; i < rows.size(); ++i) {
        S.rt[i] = rows[i].first;
        S.rk[i] = rows[i].second;
    }
    S.act.clear();
    for (u32 g = S.D.npolys; g-- > 0;)
        if (S.active.size() > g && S.active[g]) S.act.push_back(g);
}

static BuildArgs args_of(const SysState& S, bool closure) {
    BuildArgs a;
    a.G = devg_view(S.D);
    a.rows_t_host = S.rt.data();
    a.rows_k_host = S.rk.data();
    a.r0 = (u32)S.rt.size();
    a.active_host = S.act.data();
    a.nactive = (u32)S.act.size();
    a.D = S.d;
    a.closure = closure;
    return a;
}

// new basis elements of one system, appended on the device
struct AppendSeg {
    u32 row_base, rho;
    u64 nnz_base;
    u32 dict_base, poly_base;
    u64 term_base;
    u64* mon;
    u32* coeff;
    u64* off;
    u64* lm;
    u32* len;
    u32 lm_out;  // first slot in the leading-monomial readback array
    u32 pad;
};

// append the echelon rows (CSR over the matrix columns) as new basis elements,
// with their leading monomial and length; one workgroup row per system
__global__ void k_append(const AppendSeg* segs, const u32* rptr, const u32* rcol, const u32* rval,
                         const u64* dict_keys, u64* lm_out) {
    const AppendSeg A = segs[blockIdx.y];
    const u32 e0 = rptr[A.row_base], e1 = rptr[A.row_base + A.rho];
    for (u32 e = e0 + blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += gridDim.x * blockDim.x) {
        A.mon[A.term_base + (e - e0)] = dict_keys[A.dict_base + rcol[e]];
        A.coeff[A.term_base + (e - e0)] = rval[e];
    }
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t <= A.rho; t += gridDim.x * blockDim.x) {
        A.off[A.poly_base + t] = A.term_base + (rptr[A.row_base + t] - e0);
        if (t < A.rho) {
            const u64 l = dict_keys[A.dict_base + rcol[rptr[A.row_base + t]]];
            A.lm[A.poly_base + t] = l;
            A.len[A.poly_base + t] = rptr[A.row_base + t + 1] - rptr[A.row_base + t];
            if (lm_out) lm_out[A.lm_out + t] = l;
        }
    }
}

// P words of the tail entries of the final rows (dictionary of each row's system)
__global__ void k_tail_words(const u32* tptr, const u32* tcol, const u32* row_sys, const u32* dict_base, u32 R,
                             const u64* dict_keys, u64* out) {
    for (u32 i = blockIdx.x; i < R; i += gridDim.x) {
        const u32 db = dict_base[row_sys[i]];
        for (u32 e = tptr[i] + threadIdx.x; e < tptr[i + 1]; e += blockDim.x) out[e] = dict_keys[db + tcol[e]];
    }
}

// Normalise one input system and insert its polynomials (Gebauer-Moeller).
// Input bases of one or more systems staged for one upload: per system its
// device arrays and its slice of the packed terms (offsets local to the
// system); k_init_bases copies every slice and forms the leading monomials
// and lengths.
struct InitSeg {
    u64* mon;
    u32* coeff;
    u64* off;
    u64* lm;
    u32* len;
    u64 t0, o0;  // first term and first offset of the system in the pack
    u32 nt, np;
};
struct InitPack {
    std::vector<InitSeg> segs;
    std::vector<u64> mon, off;
    std::vector<u32> coeff;
};

__global__ void k_init_bases(const InitSeg* segs, const u64* mon, const u32* coeff, const u64* off) {
    const InitSeg g = segs[blockIdx.y];
    for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nt; t += gridDim.x * blockDim.x) {
        g.mon[t] = mon[g.t0 + t];
        g.coeff[t] = coeff[g.t0 + t];
    }
    for (u32 k = blockIdx.x * blockDim.x + threadIdx.x; k <= g.np; k += gridDim.x * blockDim.x) {
        const u64 o = off[g.o0 + k];
        g.off[k] = o;
        if (k < g.np) {
            g.lm[k] = mon[g.t0 + o];
            g.len[k] = (u32)(off[g.o0 + k + 1] - o);
        }
    }
}

// One upload and one launch for every staged system.
static void init_flush(Ctx& c, InitPack& pk) {
    if (pk.segs.empty()) return;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_mon = al(pk.segs.size() * sizeof(InitSeg));
    const size_t o_coeff = o_mon + al(pk.mon.size() * 8);
    const size_t o_off = o_coeff + al(pk.coeff.size() * 4);
    std::vector<u8> buf(o_off + pk.off.size() * 8);
    std::memcpy(buf.data(), pk.segs.data(), pk.segs.size() * sizeof(InitSeg));
    std::memcpy(buf.data() + o_mon, pk.mon.data(), pk.mon.size() * 8);
    std::memcpy(buf.data() + o_coeff, pk.coeff.data(), pk.coeff.size() * 4);
    std::memcpy(buf.data() + o_off, pk.off.data(), pk.off.size() * 8);
    DBuf<u8> d(&c.pool, buf.size());
    upload(c, d.ptr, buf.data(), buf.size());
    u32 mx = 1;
    for (const InitSeg& g : pk.segs) mx = std::max(mx, std::max(g.nt, g.np + 1));
    hipLaunchKernelGGL(k_init_bases, dim3(gridn(mx, 256, 64), (u32)pk.segs.size()), dim3(256), 0, c.stream,
                       (const InitSeg*)d.ptr, (const u64*)(d.ptr + o_mon), (const u32*)(d.ptr + o_coeff),
                       (const u64*)(d.ptr + o_off));
    F4_LAUNCH_CHECK();
    pk = InitPack();
}

static void init_system(Ctx& c, SysState& S, u32 p, const f4_polys* F, InitPack& pk) {
    if (!F || F->on_device || F->n == 0 || F->n > 14 || !is_odd_prime(p) || p >= (1u << 31))
        throw F4Error{F4_E_ARG, "bad argument"};
    const u32 n = F->n;
    S.n = n;
    S.p = p;
    S.mo.init(n);
    const u32 w = S.mo.w;
    std::vector<std::vector<std::pair<u64, u32>>> inputs;
    for (u32 k = 0; k < F->npolys; ++k) {
        std::vector<std::pair<u64, u32>> f;  // (order key, coeff)
        for (u64 e = F->offset[k]; e < F->offset[k + 1]; ++e) {
            const u64 P = F->mon[e];
            if ((P & ~(S.mo.lanes | (0xffull << 56))) != 0) throw F4Error{F4_E_ARG, "bad monomial word"};
            u32 d = 0;
            for (u32 i = 0; i < n; ++i) d += mono_exp(P, i, w);
            if (d != deg_of(P)) throw F4Error{F4_E_ARG, "monomial degree field mismatch"};
            f.push_back({S.mo.order_key(P), (u32)(F->coeff[e] % p)});
        }
        std::sort(f.begin(), f.end(), [](auto& a, auto& b) { return a.first > b.first; });
        std::vector<std::pair<u64, u32>> g;
        for (auto& t : f) {
            if (!g.empty() && g.back().first == t.first)
                g.back().second = (u32)(((u64)g.back().second + t.second) % p);
            else
                g.push_back(t);
        }
        std::vector<std::pair<u64, u32>> h;
        for (auto& t : g)
            if (t.second) h.push_back({t.first ^ S.mo.lanes, t.second});  // back to P words
        if (h.empty()) continue;
        const u64 inv = powmod_host(h[0].second, p - 2, p);
        for (auto& t : h) t.second = (u32)((u64)t.second * inv % p);
        if (deg_of(h[0].first) == 0) S.unit = true;
        inputs.push_back(std::move(h));
    }
    if (S.unit || inputs.empty()) {
        S.done = true;
        return;
    }
    DevG& D = S.D;
    D.n = n;
    std::vector<u64> mon, off{0};
    std::vector<u32> coeff;
    for (auto& f : inputs) {
        for (auto& t : f) {
            mon.push_back(t.first);
            coeff.push_back(t.second);
        }
        off.push_back(mon.size());
    }
    devg_reserve(c, D, 16 * mon.size(), 16 * (u32)inputs.size());
    D.npolys = (u32)inputs.size();
    D.nterms = mon.size();
    if (mon.size() >= (1ull << 32)) throw F4Error{F4_E_RANGE, "input too large"};
    pk.segs.push_back({D.mon.ptr, D.coeff.ptr, D.off.ptr, D.lm.ptr, D.len.ptr, pk.mon.size(), pk.off.size(),
                       (u32)mon.size(), D.npolys});
    pk.mon.insert(pk.mon.end(), mon.begin(), mon.end());
    pk.coeff.insert(pk.coeff.end(), coeff.begin(), coeff.end());
    pk.off.insert(pk.off.end(), off.begin(), off.end());
    S.host_pairs = (c.flags & F4_OPT_HOST_PAIRS) != 0;
    S.pairs_pending = !S.host_pairs;
    for (u32 k = 0; k < D.npolys; ++k) {
        S.lm.push_back(inputs[k][0].first);
        S.active.push_back(0);
        if (S.host_pairs) gm_insert(S.mo, S.gm, S.lm, S.active, S.P, k);
    }
}

// The inputs of every system initialised since (init_flush done) enter its
// device pair set: one update step with all of them as new elements, for all
// such systems together.
static void init_pairs(Ctx& c, const std::vector<SysState*>& sys) {
    std::vector<GmInsert> v;
    for (SysState* S : sys)
        if (S->pairs_pending) {
            S->pairs_pending = false;
            if (!S->done && !S->unit) v.push_back({&S->dp, S->D.lm.ptr, S->D.act.ptr, S->n, 0u, S->D.npolys});
        }
    gm_insert_batch(c, v);
}

// One F4 iteration for a batch of systems: every system that still has pairs
// advances by one step (symbolic preprocessing and elimination of all of them
// in one batched launch sequence).  Returns the number of systems advanced.
static size_t f4_iterate(Ctx& c, const std::vector<SysState*>& sys) {
    {
        init_pairs(c, sys);
        std::vector<SysState*> work;
        for (SysState* S : sys)
            if (!S->done && !S->unit && has_pairs(*S)) work.push_back(S);
        if (work.empty()) return 0;
        std::vector<BuildArgs> args(work.size());
        std::vector<u32> primes(work.size());
        // device pair sets: the normal selection of every system in one launch;
        // the halves and active lists stay on the device for the build
        const bool dev = !work[0]->host_pairs;
        DBuf<u64> grt, gkeep;
        DBuf<u32> grk;
        u32* gout = nullptr;
        float tsel_ms = 0;
        hipEvent_t es0 = nullptr, es1 = nullptr;
        if (dev) {
            const auto ts0 = std::chrono::steady_clock::now();
            std::vector<GmSelect> gsel;
            u64 rows_room = 0;
            for (SysState* S : work) {
                S->t0 = ts0;
                const u32 d = S->dp.dmin;
                if (d >= (1u << S->mo.w)) throw F4Error{F4_E_RANGE, "step degree overflows an exponent lane"};
                S->d = d;
                S->nsel = S->dp.nsel;
                gsel.push_back({&S->dp, S->D.lm.ptr, S->n, S->D.npolys, d, (u32)rows_room});
                rows_room += 2ull * S->dp.nsel;
            }
            if (rows_room >= (1ull << 31)) throw F4Error{F4_E_RANGE, "batch too large"};
            grt.reset(&c.pool, rows_room);
            grk.reset(&c.pool, rows_room);
            es0 = stage_event(c);
            gout = gm_select_batch(c, gsel, grt.ptr, grk.ptr, gkeep);
            for (size_t wi = 0; wi < work.size(); ++wi) {
                SysState* S = work[wi];
                BuildArgs& a = args[wi];
                a.G = devg_view(S->D);
                a.rows_t_dev = grt.ptr;
                a.rows_k_dev = grk.ptr;
                a.r0 = 2 * S->nsel;
                a.r0_dev = gout + 4 * wi;
                a.active_dev = S->dp.alist.ptr;
                a.nactive = S->dp.nact;
                a.D = S->d;
                a.closure = true;
                primes[wi] = S->p;
            }
            es1 = stage_event(c);
            tsel_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - ts0).count();
        }
        for_systems(c, dev ? 0 : work.size(), [&](size_t wi) {
            SysState* S = work[wi];
            S->t0 = std::chrono::steady_clock::now();
            const auto tp0 = S->t0;
            u32 d = 255;
            for (auto& q : S->P) d = std::min(d, deg_of(q.lcm));
            if (d >= (1u << S->mo.w)) throw F4Error{F4_E_RANGE, "step degree overflows an exponent lane"};
            std::vector<HPair> sel, rest;
            for (auto& q : S->P) (deg_of(q.lcm) == d ? sel : rest).push_back(q);
            S->P.swap(rest);
            std::vector<std::pair<u64, u32>> rows;
            for (auto& q : sel) {
                rows.push_back({q.lcm - S->lm[q.i], q.i});
                rows.push_back({q.lcm - S->lm[q.j], q.j});
            }
            prepare_rows(*S, rows);
            S->d = d;
            S->nsel = (u32)sel.size();
            S->tpairs = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - tp0).count();
            args[wi] = args_of(*S, true);
            primes[wi] = S->p;
        });
        Matrix A;
        build_batch(c, args, A);
        Reduced R;
        reduce_batch(c, primes, A, R);
        // ---- new elements: append the echelon rows to each basis on the device
        std::vector<AppendSeg> ap;
        CopyBatch grow;  // basis regrowths of this iteration, copied in one launch
        std::vector<u32> lmbase(work.size(), 0);
        u32 nl = 0, maxr = 1;
        for (size_t i = 0; i < work.size(); ++i) {
            SysState& S = *work[i];
            const RedPart& P = R.sys[i];
            lmbase[i] = nl;
            if (!P.rho) continue;
            devg_reserve(c, S.D, S.D.nterms + P.nnz, S.D.npolys + P.rho, &grow);
            AppendSeg g;
            std::memset(&g, 0, sizeof(g));
            g.row_base = P.row_base;
            g.rho = P.rho;
            g.nnz_base = P.nnz_base;
            g.dict_base = A.sys[i].dict_base;
            g.poly_base = S.D.npolys;
            g.term_base = S.D.nterms;
            g.mon = S.D.mon.ptr;
            g.coeff = S.D.coeff.ptr;
            g.off = S.D.off.ptr;
            g.lm = S.D.lm.ptr;
            g.len = S.D.len.ptr;
            g.lm_out = nl;
            ap.push_back(g);
            nl += P.rho;
            maxr = std::max<u32>(maxr, std::max<u32>(P.rho, (u32)std::min<u64>(P.nnz, 1u << 30)));
        }
        // the new leading monomials came back with the echelon's sizes: the
        // rows are appended on the device while the host updates the pairs
        if (R.newlm.size() != nl) throw F4Error{5, "echelon rows and their leading monomials disagree"};
        const std::vector<u64>& newlm = R.newlm;
        copy_flush(c, grow);
        if (!ap.empty()) {
            DBuf<AppendSeg> dap(&c.pool, ap.size());
            upload(c, dap.ptr, ap.data(), ap.size() * sizeof(AppendSeg));
            hipLaunchKernelGGL(k_append, dim3(gridn(maxr, 256, 64), (u32)ap.size()), dim3(256), 0, c.stream, dap.ptr,
                               R.row_ptr.ptr, R.col_ind.ptr, R.val.ptr, A.dict_keys.ptr, (u64*)nullptr);
            F4_LAUNCH_CHECK();
        }
        A.read_times();
        R.read_times();
        for_systems(c, work.size(), [&](size_t i) {
            SysState& S = *work[i];
            const RedPart& P = R.sys[i];
            const SysPart& M = A.sys[i];
            S.D.npolys += P.rho;
            S.D.nterms += P.nnz;
            f4_step_stats st;
            std::memset(&st, 0, sizeof(st));
            st.deg = S.d;
            st.nsel = S.nsel;
            st.r = M.r;
            st.N = M.N;
            st.nnz = M.nnz;
            st.npivot = P.npivot;
            st.lower = P.lower;
            st.rho = P.rho;
            st.rank = P.rank;
            st.closure_rounds = A.closure_rounds;
            st.dict_path = A.dict_path;
            st.t_dict_ms = A.t_dict;
            st.t_assemble_ms = A.t_assemble;
            st.t_numeric_ms = R.t_split + R.t_trsm + R.t_echelon + R.t_emit;
            st.t_trsm_ms = R.t_trsm;
            st.t_echelon_ms = R.t_echelon;
            st.t_k_trsm_ms = R.t_k_trsm;
            st.n_k_trsm = (u32)R.ev_trsm.size();
            st.trsm_ops = R.trsm_ops;
            st.t_k_block_ms = R.t_k_block;
            st.n_k_block = (u32)R.ev_block.size();
            st.block_ops = R.block_ops;
            const auto tg0 = std::chrono::steady_clock::now();
            // a constant among the new elements ends the computation ({1});
            // otherwise the step's elements enter the pair set together
            for (u32 t = 0; t < P.rho; ++t)
                if (deg_of(newlm[lmbase[i] + t]) == 0) S.unit = true;
            if (!S.unit && P.rho) {
                const u32 h0 = (u32)S.lm.size();
                for (u32 t = 0; t < P.rho; ++t) {
                    S.lm.push_back(newlm[lmbase[i] + t]);
                    S.active.push_back(0);
                }
                if (S.host_pairs) gm_insert_step(S.mo, S.gm, S.lm, S.active, S.P, h0, h0 + P.rho);
            }
            const auto tg1 = std::chrono::steady_clock::now();
            st.t_pairs_ms = S.tpairs + std::chrono::duration<float, std::milli>(tg1 - tg0).count();
            st.t_step_ms = std::chrono::duration<float, std::milli>(tg1 - S.t0).count();
            S.steps.push_back(st);
            if (c.stop_deg && S.d == c.stop_deg && !S.unit) S.done = true;  // stopped: no basis
        });
        if (dev) {
            // the step's elements enter the device pair sets (every system
            // still running: also those without new elements, whose
            // summary the selection consumed)
            const auto tg0 = std::chrono::steady_clock::now();
            std::vector<GmInsert> gi;
            for (size_t i = 0; i < work.size(); ++i) {
                SysState& S = *work[i];
                if (S.unit || S.done) continue;
                gi.push_back({&S.dp, S.D.lm.ptr, S.D.act.ptr, S.n, S.D.npolys - R.sys[i].rho, R.sys[i].rho,
                              gout + 4 * i, 2 * S.nsel});
            }
            hipEvent_t eg0 = stage_event(c);
            gm_insert_batch(c, gi);
            hipEvent_t eg1 = stage_event(c);
            const auto tg1 = std::chrono::steady_clock::now();
            float tp = tsel_ms + std::chrono::duration<float, std::milli>(tg1 - tg0).count();
            if (es0 && eg0) {
                (void)hipEventSynchronize(eg1);
                tp = event_ms(es0, es1) + (gi.empty() ? 0.f : event_ms(eg0, eg1));
            }
            for (SysState* S : work) {
                S->steps.back().t_pairs_ms = tp;
                S->steps.back().t_step_ms = std::chrono::duration<float, std::milli>(tg1 - S->t0).count();
            }
        }
        c.ev_used = 0;
        return work.size();
    }
}

// Reduced bases of the systems that have no pairs left: minimal leading
// monomials, tails reduced by the others (all such systems in one batch).
static void f4_finish(Ctx& c, const std::vector<SysState*>& sys) {
    std::vector<SysState*> fin;
    std::vector<BuildArgs> args;
    std::vector<u32> primes;
    std::vector<std::set<u32>> minimal;
    {
        // activity flags of the device pair sets, fetched in one readback
        std::vector<SysState*> dl;
        u64 words = 0;
        for (SysState* S : sys)
            if (!S->done && !S->unit && !S->host_pairs && !has_pairs(*S)) {
                dl.push_back(S);
                words += S->D.npolys;
            }
        if (words) {
            DBuf<u32> pack(&c.pool, words);
            CopyBatch cb;
            u64 o = 0;
            for (SysState* S : dl) {
                if (S->D.npolys) cb.jobs.push_back({S->D.act.ptr, pack.ptr + o, S->D.npolys});
                o += S->D.npolys;
            }
            copy_flush(c, cb);
            std::vector<u32> h(words);
            readback(c, h.data(), pack.ptr, words * 4);
            o = 0;
            for (SysState* S : dl) {
                S->active.assign(h.begin() + o, h.begin() + o + S->D.npolys);
                o += S->D.npolys;
            }
        }
    }
    for (SysState* S : sys) {
        if (S->done || (!S->unit && has_pairs(*S))) continue;
        S->done = true;
        if (S->unit) continue;
        std::vector<u32> mins;
        for (u32 g = 0; g < S->lm.size(); ++g) {
            if (!S->active[g]) continue;
            bool mn = true;
            for (u32 h = 0; h < S->lm.size() && mn; ++h)
                if (h != g && S->active[h] && S->mo.divides(S->lm[h], S->lm[g])) mn = false;
            if (mn) mins.push_back(g);
        }
        std::vector<std::pair<u64, u32>> rows;
        u32 dmax = 0;
        for (u32 g : mins) {
            rows.push_back({0ull, g});
            dmax = std::max(dmax, deg_of(S->lm[g]));
        }
        prepare_rows(*S, rows);
        S->d = dmax;
        fin.push_back(S);
        args.push_back(args_of(*S, true));
        primes.push_back(S->p);
        minimal.emplace_back(mins.begin(), mins.end());
    }
    if (fin.empty()) return;
    Matrix A;
    build_batch(c, args, A);
    DBuf<u32> tptr, tcol, tval;
    tail_reduce_batch(c, primes, A, tptr, tcol, tval);
    const u32 R = A.R;
    std::vector<u64> rt(R);
    std::vector<u32> rk(R), hp((u64)R + 1);
    readback(c, rt.data(), A.row_t.ptr, (u64)R * 8);
    readback(c, rk.data(), A.row_k.ptr, (u64)R * 4);
    readback(c, hp.data(), tptr.ptr, ((u64)R + 1) * 4);
    const u32 nt = hp[R];
    std::vector<u64> hw(nt);
    std::vector<u32> hv(nt);
    if (nt) {
        std::vector<u32> db(fin.size());
        for (size_t i = 0; i < fin.size(); ++i) db[i] = A.sys[i].dict_base;
        DBuf<u32> ddb(&c.pool, db.size());
        DBuf<u64> dw(&c.pool, nt);
        upload(c, ddb.ptr, db.data(), db.size() * 4);
        hipLaunchKernelGGL(k_tail_words, dim3(gridn(R, 1, 4096)), dim3(64), 0, c.stream, tptr.ptr, tcol.ptr,
                           A.row_sys.ptr, ddb.ptr, R, A.dict_keys.ptr, dw.ptr);
        F4_LAUNCH_CHECK();
        readback(c, hw.data(), dw.ptr, (u64)nt * 8);
        readback(c, hv.data(), tval.ptr, (u64)nt * 4);
    }
    for (size_t i = 0; i < fin.size(); ++i) {
        SysState& S = *fin[i];
        const SysPart& M = A.sys[i];
        std::set<u32>& mset = minimal[i];
        // rows of a system are sorted by leading monomial, largest first
        for (u32 r = M.row_base; r < M.row_base + M.r; ++r) {
            if (rt[r] != 0 || !mset.count(rk[r])) continue;
            S.gmon.push_back(S.lm[rk[r]]);
            S.gcoeff.push_back(1);
            for (u32 e = hp[r]; e < hp[r + 1]; ++e) {
                S.gmon.push_back(hw[e]);
                S.gcoeff.push_back(hv[e]);
            }
            S.goff.push_back(S.gmon.size());
            mset.erase(rk[r]);
        }
        if (!mset.empty()) throw F4Error{F4_E_STATE, "inter-reduction lost a basis element"};
    }
}

// The F4 loop for a batch of systems, then their reduced bases.
static void run_f4(Ctx& c, std::vector<SysState*>& sys) {
    while (f4_iterate(c, sys)) {
    }
    f4_finish(c, sys);
}

static f4_basis* basis_of(f4_ctx* X, SysState& S) {
    f4_basis* B = new f4_basis();
    B->owner = X;
    B->n = S.n;
    if (S.unit) {
        B->mon = {0};
        B->coeff = {1};
        B->off = {0, 1};
    } else {
        B->mon = std::move(S.gmon);
        B->coeff = std::move(S.gcoeff);
        B->off = std::move(S.goff);
    }
    B->steps = std::move(S.steps);
    return B;
}

// ---------------------------------------------------------------- serving state
struct ServerReq {
    u64 footprint = 0;
    std::unique_ptr<SysState> st;
};

struct f4_server {
    f4_ctx* owner = nullptr;
    u64 budget = 0, used = 0;
    u32 max_slots = 0;
    u64 next_ticket = 1;
    std::map<u64, ServerReq> reqs;
};

// ====================================================================== API
extern "C" {

int f4_create(f4_ctx** out, int device, const f4_opts* opts) {
    if (!out) return F4_E_ARG;
    *out = nullptr;
    f4_ctx* X = new (std::nothrow) f4_ctx();
    if (!X) return F4_E_NOMEM;
    try {
        F4_HIP_TRY(hipSetDevice(device));
        noalloc_scratch_init(device);  // once per device: address of the allocation-free calls' scratch
        hipDeviceProp_t prop;
        F4_HIP_TRY(hipGetDeviceProperties(&prop, device));
        X->c.dev.device = device;
        X->c.dev.cus = prop.multiProcessorCount;
        X->c.dev.max_lds = prop.sharedMemPerBlock;
        X->c.flags = opts ? opts->flags : 0;
        X->c.stop_deg = opts ? opts->stop_deg : 0;
        X->c.tune.on = (X->c.flags & F4_OPT_AUTOTUNE) != 0;
        X->c.tune.force_rr = opts ? opts->trsm_rows : 0;
        X->c.tune.force_digit = opts ? opts->radix_bits : 0;
        if (X->c.tune.force_rr > 4 || X->c.tune.force_digit > 8)
            throw F4Error{F4_E_ARG, "trsm_rows must be at most 4 and radix_bits at most 8"};
        if (opts && (!opts->alloc) != (!opts->free)) throw F4Error{F4_E_ARG, "alloc and free must be set together"};
        X->c.pool.stream = &X->c.stream;
        if (opts && opts->alloc) {
            X->c.pool.ualloc = opts->alloc;
            X->c.pool.ufree = opts->free;
            X->c.pool.uuser = opts->alloc_user;
        }
        F4_HIP_TRY(hipStreamCreateWithFlags(&X->c.own_stream, hipStreamNonBlocking));
        X->c.stream = X->c.own_stream;
        F4_HIP_TRY(hipEventCreateWithFlags(&X->c.staging_done, hipEventDisableTiming));
        staging(X->c, 8u << 20);
        X->c.pinned_used = 0;
    } catch (const F4Error& e) {
        int code = e.code;
        delete X;
        return code;
    }
    *out = X;
    return F4_OK;
}

int f4_destroy(f4_ctx* X) {
    if (!X) return F4_E_ARG;
    (void)hipSetDevice(X->c.dev.device);
    if (X->c.stream) (void)hipStreamSynchronize(X->c.stream);
    // live handles own pool memory: free them before the pool goes
    for (f4_server* v : X->servers) delete v;
    X->servers.clear();
    for (f4_matrix* m : X->matrices) delete m;
    for (f4_reduced* r : X->reduceds) delete r;
    for (f4_basis* b : X->bases) delete b;
    X->matrices.clear();
    X->reduceds.clear();
    X->bases.clear();
    X->c.binom.clear();
    X->c.montab.clear();
    for (hipEvent_t e : X->c.events) (void)hipEventDestroy(e);
    if (X->c.staging_done) (void)hipEventDestroy(X->c.staging_done);
    if (X->c.pinned) (void)hipHostFree(X->c.pinned);
    X->c.pool.trim();
    X->c.pool.stream = nullptr;
    if (X->c.own_stream) (void)hipStreamDestroy(X->c.own_stream);
    delete X->c.cpu;
    delete X;
    return F4_OK;
}

const char* f4_last_error(const f4_ctx* X) { return X ? X->c.last_error.c_str() : "null context"; }

int f4_tune_export(f4_ctx* X, char* buf, size_t cap, size_t* len) {
    F4_API_BEGIN(X)
    if (!len) throw F4Error{F4_E_ARG, "null length pointer"};
    const std::string t = tune_text(X->c);
    *len = t.size();
    if (buf) {
        if (cap <= t.size()) throw F4Error{F4_E_RANGE, "tune table: buffer too small"};
        memcpy(buf, t.c_str(), t.size() + 1);
    }
    F4_API_END(X)
}

int f4_tune_import(f4_ctx* X, const char* text) {
    F4_API_BEGIN(X)
    if (!text) throw F4Error{F4_E_ARG, "null text"};
    tune_parse(X->c, text);
    F4_API_END(X)
}

int f4_modloop(f4_ctx* X, uint32_t p, uint32_t form, uint32_t nchains, uint32_t iters, const uint32_t* x0,
               const uint32_t* a, const uint32_t* b, uint32_t* out, f4_modloop_stats* st) {
    F4_API_BEGIN(X)
    if (!x0 || !a || !b || !out || !st) throw F4Error{F4_E_ARG, "null pointer"};
    if (!is_odd_prime(p) || p >= (1u << 31) || form > F4_MODLOOP_MONTGOMERY) throw F4Error{F4_E_ARG, "bad argument"};
    if (form <= F4_MODLOOP_BARRETT32 && p >= 65536) throw F4Error{F4_E_ARG, "16-bit form needs p < 2^16"};
    if (nchains == 0 || nchains > (1u << 26) || iters == 0) throw F4Error{F4_E_ARG, "bad chain count or length"};
    for (u32 i = 0; i < nchains; ++i)
        if (x0[i] >= p || a[i] >= p || b[i] >= p) throw F4Error{F4_E_ARG, "input value is not a residue"};
    ModloopResult r;
    modloop_run(X->c, p, form, nchains, iters, x0, a, b, out, r);
    st->updates_per_s = r.updates_per_s;
    st->kernel_ms = r.kernel_ms;
    st->regs = r.regs;
    st->private_bytes = r.private_bytes;
    F4_API_END(X)
}

uint32_t f4_lane_bits(uint32_t n) { return lane_bits(n); }

int f4_download(f4_ctx* X, void* dst, const void* src, size_t bytes) {
    F4_API_BEGIN(X)
    if ((!dst || !src) && bytes) throw F4Error{F4_E_ARG, "null pointer"};
    if (bytes) {
        F4_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, X->c.stream));
        F4_HIP_TRY(hipStreamSynchronize(X->c.stream));
    }
    F4_API_END(X)
}

static std::vector<u32> host_binom(u32 n, u32 D) {
    std::vector<u32> tab((size_t)(n + D + 2) * F4_BSTRIDE, 0);
    for (u32 x = 0; x < n + D + 2; ++x)
        for (u32 y = 0; y < F4_BSTRIDE; ++y) {
            u64 v = binom_host(x, y);
            tab[(size_t)x * F4_BSTRIDE + y] = v > 0xffffffffull ? 0xffffffffu : (u32)v;
        }
    return tab;
}

int f4_grevlex_rank(uint32_t n, uint32_t D, uint64_t word, uint32_t* rank) {
    const u32 w = lane_bits(n);
    if (!w || !rank || binom_host(n + D, n) > 0xffffffffull) return F4_E_ARG;
    if ((word >> 56) > D) return F4_E_RANGE;
    std::vector<u32> B = host_binom(n, D);
    *rank = mono_rank(word, n, w, D, B.data());
    return F4_OK;
}

int f4_grevlex_unrank(uint32_t n, uint32_t D, uint32_t rank, uint64_t* word) {
    const u32 w = lane_bits(n);
    if (!w || !word || binom_host(n + D, n) > 0xffffffffull) return F4_E_ARG;
    if (rank >= binom_host(n + D, n)) return F4_E_RANGE;
    std::vector<u32> B = host_binom(n, D);
    *word = mono_unrank(rank, n, w, D, B.data());
    return F4_OK;
}

int f4_pack(uint32_t n, const uint32_t* exps, uint64_t* out) {
    if (!exps || !out) return F4_E_ARG;
    const u32 w = lane_bits(n);
    if (!w) return F4_E_ARG;
    u64 P = 0;
    u32 d = 0;
    for (u32 i = 0; i < n; ++i) {
        if (exps[i] >= (1u << w)) return F4_E_RANGE;
        P |= (u64)exps[i] << (w * i);
        d += exps[i];
    }
    if (d > 255) return F4_E_RANGE;
    *out = P | ((u64)d << 56);
    return F4_OK;
}

int f4_check_polys(uint32_t p, const f4_polys* G, int monic, uint32_t* bits) {
    if (bits) *bits = 0;
    if (!G || G->on_device || !G->offset || G->n == 0 || G->n > 14 || !is_odd_prime(p) || p >= (1u << 31))
        return F4_E_ARG;
    if (G->npolys && G->offset[G->npolys] && (!G->mon || !G->coeff)) return F4_E_ARG;
    if (G->offset[0] != 0) return F4_E_ARG;
    const u32 bad = check_polys_host(G->n, p, G->npolys, G->mon, G->coeff, G->offset, monic != 0);
    if (bits) *bits = bad;
    return bad ? F4_E_ARG : F4_OK;
}

int f4_normalize_polys(uint32_t p, const f4_polys* in, int monic, uint64_t* mon_out, uint32_t* coeff_out,
                       uint64_t* off_out) {
    if (!in || in->on_device || !in->offset || !off_out || in->n == 0 || in->n > 14 || !is_odd_prime(p) ||
        p >= (1u << 31))
        return F4_E_ARG;
    const u32 n = in->n, w = lane_bits(n);
    const u64 lanes = (1ull << (n * w)) - 1;
    const u64 nt = in->offset[in->npolys];
    if (nt && (!in->mon || !in->coeff || !mon_out || !coeff_out)) return F4_E_ARG;
    try {
        std::vector<std::pair<u64, u32>> f;
        u64 o = 0;
        off_out[0] = 0;
        for (u32 k = 0; k < in->npolys; ++k) {
            if (in->offset[k + 1] < in->offset[k]) return F4_E_ARG;
            f.clear();
            for (u64 e = in->offset[k]; e < in->offset[k + 1]; ++e) {
                if (check_term(in->mon[e], 1, n, w, lanes, p) & CHK_WORD) return F4_E_ARG;
                f.push_back({in->mon[e] ^ lanes, (u32)(in->coeff[e] % p)});  // order key
            }
            std::sort(f.begin(), f.end(), [](const std::pair<u64, u32>& a, const std::pair<u64, u32>& b) {
                return a.first > b.first;
            });
            const u64 o0 = o;
            for (size_t i = 0; i < f.size();) {
                u64 sum = 0;
                size_t j = i;
                for (; j < f.size() && f[j].first == f[i].first; ++j) sum += f[j].second;
                const u32 cf = (u32)(sum % p);
                if (cf) {
                    mon_out[o] = f[i].first ^ lanes;
                    coeff_out[o] = cf;
                    ++o;
                }
                i = j;
            }
            if (monic && o > o0 && coeff_out[o0] != 1) {
                const u64 inv = powmod_host(coeff_out[o0], p - 2, p);
                for (u64 e = o0; e < o; ++e) coeff_out[e] = (u32)(coeff_out[e] * inv % p);
            }
            off_out[k + 1] = o;
        }
    } catch (const std::bad_alloc&) {
        return F4_E_NOMEM;
    }
    return F4_OK;
}

uint32_t f4_mw_lane_bits(uint32_t n) { return mw_lane_bits(n); }

int f4_pack_mw(uint32_t n, const uint32_t* exps, uint64_t* out) {
    if (!exps || !out) return F4_E_ARG;
    const MwLayout L = mw_layout(n);
    if (!L.w) return F4_E_ARG;
    u64 m[2] = {0, 0};
    u32 d = 0;
    for (u32 v = 0; v < n; ++v) {
        if (exps[v] >= (1u << L.w)) return F4_E_RANGE;
        const u32 p = n - 1 - v;
        if (p < L.a)
            m[0] |= (u64)exps[v] << (56 - (p + 1) * L.w);
        else
            m[1] |= (u64)exps[v] << (64 - (p - L.a + 1) * L.w);
        d += exps[v];
    }
    if (d > 255) return F4_E_RANGE;
    out[0] = m[0] | ((u64)d << 56);
    out[1] = m[1];
    return F4_OK;
}

int f4_unpack_mw(uint32_t n, const uint64_t* in, uint32_t* exps) {
    const MwLayout L = mw_layout(n);
    if (!L.w || !in || !exps) return F4_E_ARG;
    for (u32 v = 0; v < n; ++v) exps[v] = mw_exp(L, in[0], in[1], v);
    return F4_OK;
}

int f4_normalize_polys_mw(uint32_t p, const f4_polys_mw* in, uint64_t* mon_out, uint32_t* coeff_out,
                          uint64_t* off_out) {
    if (!in || !in->offset || !off_out || !is_odd_prime(p) || p >= (1u << 31)) return F4_E_ARG;
    const MwLayout L = mw_layout(in->n);
    if (!L.w) return F4_E_ARG;
    const u64 nt = in->offset[in->npolys];
    if (nt && (!in->mon || !in->coeff || !mon_out || !coeff_out)) return F4_E_ARG;
    struct Term {
        u64 k0, k1;  // order key
        u32 c;
    };
    try {
        std::vector<Term> f;
        u64 o = 0;
        off_out[0] = 0;
        for (u32 k = 0; k < in->npolys; ++k) {
            if (in->offset[k + 1] < in->offset[k]) return F4_E_ARG;
            f.clear();
            for (u64 e = in->offset[k]; e < in->offset[k + 1]; ++e) {
                const u64 m0 = in->mon[2 * e], m1 = in->mon[2 * e + 1];
                if (!mw_valid(L, m0, m1)) return F4_E_ARG;
                f.push_back({m0 ^ L.lanes0, m1 ^ L.lanes1, (u32)(in->coeff[e] % p)});
            }
            std::sort(f.begin(), f.end(), [](const Term& a, const Term& b) {
                return a.k0 != b.k0 ? a.k0 > b.k0 : a.k1 > b.k1;
            });
            for (size_t i = 0; i < f.size();) {
                u64 sum = 0;
                size_t j = i;
                for (; j < f.size() && f[j].k0 == f[i].k0 && f[j].k1 == f[i].k1; ++j) sum += f[j].c;
                const u32 cf = (u32)(sum % p);
                if (cf) {
                    mon_out[2 * o] = f[i].k0 ^ L.lanes0;
                    mon_out[2 * o + 1] = f[i].k1 ^ L.lanes1;
                    coeff_out[o] = cf;
                    ++o;
                }
                i = j;
            }
            off_out[k + 1] = o;
        }
    } catch (const std::bad_alloc&) {
        return F4_E_NOMEM;
    }
    return F4_OK;
}

int f4_build_matrix_rows_mw(f4_ctx* X, uint32_t p, const f4_polys_mw* G, const f4_rowspec_mw* R, uint32_t r,
                            f4_matrix** A, void* stream) {
    F4_API_BEGIN(X)
    if (!A || !G || !R || !r || !is_odd_prime(p) || p >= (1u << 31)) throw F4Error{F4_E_ARG, "bad argument"};
    *A = nullptr;
    const MwLayout L = mw_layout(G->n);
    if (!L.w) throw F4Error{F4_E_ARG, "bad number of variables"};
    if (!G->offset || !G->npolys || !G->mon || !G->coeff) throw F4Error{F4_E_ARG, "null basis array"};
    set_stream(X, stream);
    // the basis form, on the host: monomials, strictly decreasing order keys
    // (high words, then low words), coefficients in [1, p), no empty polynomial
    const u64* off = G->offset;
    if (off[0] != 0) throw F4Error{F4_E_ARG, "offsets must start at 0"};
    for (u32 k = 0; k < G->npolys; ++k) {
        if (off[k + 1] <= off[k]) throw F4Error{F4_E_ARG, "a zero polynomial"};
        for (u64 e = off[k]; e < off[k + 1]; ++e) {
            const u64 m0 = G->mon[2 * e], m1 = G->mon[2 * e + 1];
            if (!mw_valid(L, m0, m1)) throw F4Error{F4_E_ARG, "a word pair that is not a monomial of n variables"};
            if (G->coeff[e] == 0 || G->coeff[e] >= p) throw F4Error{F4_E_ARG, "coefficient outside [1, p)"};
            if (e > off[k]) {
                const u64 a0 = G->mon[2 * e - 2] ^ L.lanes0, a1 = G->mon[2 * e - 1] ^ L.lanes1;
                const u64 b0 = m0 ^ L.lanes0, b1 = m1 ^ L.lanes1;
                if (!(a0 > b0 || (a0 == b0 && a1 > b1))) throw F4Error{F4_E_ARG, "terms not in decreasing grevlex"};
            }
        }
    }
    f4_matrix* M = new f4_matrix();
    M->owner = X;
    try {
        build_rows_mw(X->c, G->n, G->npolys, G->mon, G->coeff, off, R, r, M->m);
        M->m.built_p = p;
    } catch (...) {
        delete M;
        throw;
    }
    X->matrices.insert(M);
    *A = M;
    F4_API_END(X)
}

int f4_unpack(uint32_t n, uint64_t word, uint32_t* exps) {
    const u32 w = lane_bits(n);
    if (!w || !exps) return F4_E_ARG;
    for (u32 i = 0; i < n; ++i) exps[i] = mono_exp(word, i, w);
    return F4_OK;
}

int f4_build_matrix(f4_ctx* X, uint32_t p, const f4_polys* G, const uint8_t* active, const f4_pair* sel,
                    uint32_t nsel, f4_matrix** A, void* stream) {
    F4_API_BEGIN(X)
    if (!A || !G || !active || (!sel && nsel) || !is_odd_prime(p) || p >= (1u << 31))
        throw F4Error{F4_E_ARG, "bad argument"};
    if (nsel == 0) throw F4Error{F4_E_ARG, "empty selection"};
    *A = nullptr;
    set_stream(X, stream);
    Ctx& c = X->c;
    DevG D;
    load_polys(c, p, G, D, true);
    std::vector<u64> lm(D.npolys);
    readback(c, lm.data(), D.lm.ptr, (u64)D.npolys * 8);
    MonoOps mo;
    mo.init(D.n);
    std::vector<std::pair<u64, u32>> rows;
    u32 deg = 0;
    for (u32 q = 0; q < nsel; ++q) {
        const u32 i = sel[q].i, j = sel[q].j;
        if (i >= D.npolys || j >= D.npolys || i == j) throw F4Error{F4_E_ARG, "pair index out of range"};
        const u64 L = mono_lcm(lm[i], lm[j], D.n, mo.w);
        deg = std::max(deg, deg_of(L));
        rows.push_back({L - lm[i], i});
        rows.push_back({L - lm[j], j});
    }
    if (deg >= (1u << mo.w)) throw F4Error{F4_E_RANGE, "step degree overflows an exponent lane"};
    std::vector<u32> act;
    for (u32 g = D.npolys; g-- > 0;)
        if (active[g]) act.push_back(g);
    SysState st;
    st.D = std::move(D);
    st.d = deg;
    prepare_rows(st, rows);
    st.act = act;
    f4_matrix* M = new f4_matrix();
    M->owner = X;
    try {
        build_batch(c, std::vector<BuildArgs>{args_of(st, true)}, M->m);
        M->m.built_p = p;
    } catch (...) {
        delete M;
        throw;
    }
    X->matrices.insert(M);
    *A = M;
    F4_API_END(X)
}

// Device planning of an explicit row list (f4_build_matrix_rows): checks of
// every (t, k), the largest row degree, then the distinct rows by sorting the
// keys rank(t) npolys + k (rank: the dense grevlex rank of t among the
// monomials up to the largest shift degree) and dropping repeats.
// info: [0] error bits (1 bad index or shift word, 2 lane overflow),
// [1] largest degree of t LM(g_k), [2] largest degree of t.
#define ROWS_SLOTS 64
__global__ void k_rows_check(const f4_rowspec* __restrict__ R, u32 r, const u64* __restrict__ lm, u32 npolys,
                             u32 n, u32 w, u32* info) {
    u32 err = 0, dmax = 0, tmax = 0;
    const u64 lanes = (1ull << (n * w)) - 1;
    u64 H = 0;
    for (u32 v = 0; v < n; ++v) H |= 1ull << (w * v + w - 1);
    const u32 lmask = (1u << w) - 1;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x) {
        const u64 t = R[i].t;
        const u32 k = R[i].k;
        u32 sum = 0;
        u64 x = t & lanes;
        for (u32 v = 0; v < n; ++v, x >>= w) sum += (u32)x & lmask;
        if (k >= npolys || (t & ~lanes & ((1ull << 56) - 1)) || sum != mono_deg(t)) {
            err |= 1;
            continue;
        }
        const u64 g = lm[k];
        // lanes without their top bit cannot overflow when added
        if ((t | g) & H)
            for (u32 v = 0; v < n; ++v)
                if (mono_exp(t, v, w) + mono_exp(g, v, w) >= (1u << w)) err |= 2;
        dmax = max(dmax, mono_deg(t) + mono_deg(g));
        tmax = max(tmax, mono_deg(t));
    }
    for (u32 d = F4_WAVE / 2; d > 0; d >>= 1) {
        err |= (u32)__shfl_xor((int)err, (int)d, F4_WAVE);
        dmax = max(dmax, (u32)__shfl_xor((int)dmax, (int)d, F4_WAVE));
        tmax = max(tmax, (u32)__shfl_xor((int)tmax, (int)d, F4_WAVE));
    }
    // one of ROWS_SLOTS copies of the three words per block (atomics on one
    // word serialise across the grid); the host combines the copies
    if (lane_id() == 0) {
        u32* I = info + 4 * (blockIdx.x % ROWS_SLOTS);
        if (err) atomicOr(&I[0], err);
        if (dmax) atomicMax(&I[1], dmax);
        if (tmax) atomicMax(&I[2], tmax);
    }
}

// the copies of k_rows_check's words combined (err | ..., max, max)
static void rows_info(Ctx& c, const u32* dinfo, u32 hi[4]) {
    u32 slots[4 * ROWS_SLOTS];
    readback(c, slots, dinfo, sizeof(slots));
    hi[0] = hi[1] = hi[2] = hi[3] = 0;
    for (int q = 0; q < ROWS_SLOTS; ++q) {
        hi[0] |= slots[4 * q];
        hi[1] = std::max(hi[1], slots[4 * q + 1]);
        hi[2] = std::max(hi[2], slots[4 * q + 2]);
    }
}

__global__ void k_rows_keys(const f4_rowspec* __restrict__ R, u32 r, u32 n, u32 w, u32 Dt, const u32* __restrict__ B,
                            u32 npolys, u64* __restrict__ keys) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x)
        keys[i] = (u64)mono_rank(R[i].t, n, w, Dt, B) * npolys + R[i].k;
}

__global__ void k_rows_decode(const u64* __restrict__ keys, const u32* __restrict__ cnt, u32 npolys,
                              const u64* __restrict__ montab, u64* __restrict__ rows_t, u32* __restrict__ rows_k) {
    const u32 m = *cnt;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const u64 key = keys[i];
        rows_t[i] = montab[key / npolys];
        rows_k[i] = (u32)(key % npolys);
    }
}

// An explicit row list planned on the device: checked, deduplicated and
// decoded into (rt, rk) (r0 distinct rows); deg = the largest row degree.
// Rd keeps the uploaded records.
static void plan_rows(Ctx& c, const DevG& D, const f4_rowspec* R, u32 r, DBuf<u8>& Rd, DBuf<u64>& rt, DBuf<u32>& rk,
                      u32& r0, u32& deg) {
    hipStream_t s = c.stream;
    if (D.npolys == 0) throw F4Error{F4_E_ARG, "row basis index out of range"};
    const u32 w = lane_bits(D.n);
    // the row list on the device, checked there
    Rd.reset(&c.pool, (u64)r * sizeof(f4_rowspec));
    upload(c, Rd.ptr, R, (u64)r * sizeof(f4_rowspec));
    const f4_rowspec* Rdev = (const f4_rowspec*)Rd.ptr;
    DBuf<u32> info(&c.pool, 4 * ROWS_SLOTS);
    fill_u32(info.ptr, 4 * ROWS_SLOTS, 0, s);
    const u32 grid = std::min<u32>(4096, ceil_div(r, 256));
    hipLaunchKernelGGL(k_rows_check, dim3(grid), dim3(256), 0, s, Rdev, r, D.lm.ptr, D.npolys, D.n, w, info.ptr);
    F4_LAUNCH_CHECK();
    u32 hi[4];
    rows_info(c, info.ptr, hi);
    if (hi[0] & 1) throw F4Error{F4_E_ARG, "row basis index out of range or shift not a monomial"};
    if (hi[0] & 2) throw F4Error{F4_E_RANGE, "exponent lane overflow"};
    deg = hi[1];
    const u32 Dt = hi[2];
    if (deg >= (1u << w)) throw F4Error{F4_E_RANGE, "degree overflows an exponent lane"};
    const u64 nt = binom_host(D.n + Dt, D.n);
    if (nt * D.npolys >= (1ull << 63)) throw F4Error{F4_E_RANGE, "row keys do not fit 64 bits"};
    // distinct rows: sort the keys, drop repeats, decode
    const u32* B = rank_table(c, D.n, Dt);
    const u64* montab = unrank_table(c, D.n, Dt);
    DBuf<u64> keys(&c.pool, r), ukeys(&c.pool, r);
    DBuf<u32> cnt(&c.pool, 1);
    hipLaunchKernelGGL(k_rows_keys, dim3(grid), dim3(256), 0, s, Rdev, r, D.n, w, Dt, B, D.npolys, keys.ptr);
    F4_LAUNCH_CHECK();
    u32 bits = 1;
    while (bits < 64 && (nt * D.npolys - 1) >> bits) ++bits;
    radix_sort_keys(keys.ptr, r, 0, bits, c.pool, s);
    unique_sorted_u64(keys.ptr, r, ukeys.ptr, cnt.ptr, c.pool, s);
    r0 = 0;
    readback(c, &r0, cnt.ptr, 4);
    rt.reset(&c.pool, std::max<u32>(r0, 1));
    rk.reset(&c.pool, std::max<u32>(r0, 1));
    hipLaunchKernelGGL(k_rows_decode, dim3(std::min<u32>(4096, ceil_div(r0, 256))), dim3(256), 0, s, ukeys.ptr,
                       cnt.ptr, D.npolys, montab, rt.ptr, rk.ptr);
    F4_LAUNCH_CHECK();
}

static f4_matrix* build_one(f4_ctx* X, u32 p, const BuildArgs& a) {
    f4_matrix* M = new f4_matrix();
    M->owner = X;
    try {
        build_batch(X->c, std::vector<BuildArgs>{a}, M->m);
        M->m.built_p = p;
    } catch (...) {
        delete M;
        throw;
    }
    X->matrices.insert(M);
    return M;
}

int f4_build_matrix_rows(f4_ctx* X, uint32_t p, const f4_polys* G, const f4_rowspec* R, uint32_t r, f4_matrix** A,
                         void* stream) {
    F4_API_BEGIN(X)
    if (!A || !G || !R || !r || !is_odd_prime(p) || p >= (1u << 31)) throw F4Error{F4_E_ARG, "bad argument"};
    *A = nullptr;
    set_stream(X, stream);
    Ctx& c = X->c;
    DevG D;
    load_polys(c, p, G, D, false);
    DBuf<u8> Rd;
    DBuf<u64> rt;
    DBuf<u32> rk;
    u32 r0 = 0, deg = 0;
    plan_rows(c, D, R, r, Rd, rt, rk, r0, deg);
    BuildArgs a;
    a.G = devg_view(D);
    a.rows_t_dev = rt.ptr;
    a.rows_k_dev = rk.ptr;
    a.r0 = r0;
    a.nactive = 0;
    a.D = deg;
    a.closure = false;
    *A = build_one(X, p, a);
    F4_API_END(X)
}

static void sig_of(Ctx& c, const DevG& D, const f4_sigs* S, SigBufs& out) {
    if (!S || S->npolys != D.npolys) throw F4Error{F4_E_ARG, "signatures do not match the basis"};
    sig_upload(c, D.n, D.npolys, S->index, S->mon, S->nindex, S->syz_off, S->syz_mon, out);
}

int f4_sig_filter(f4_ctx* X, uint32_t p, const f4_polys* G, const f4_sigs* S, const f4_rowspec* R, uint32_t r,
                  uint8_t* flags, f4_rowspec* kept, uint32_t* nkept, uint32_t* order, f4_sig_stats* st,
                  void* stream) {
    F4_API_BEGIN(X)
    if (!G || !R || !r || !nkept || !is_odd_prime(p) || p >= (1u << 31)) throw F4Error{F4_E_ARG, "bad argument"};
    set_stream(X, stream);
    Ctx& c = X->c;
    hipStream_t s = c.stream;
    DevG D;
    load_polys(c, p, G, D, false);
    if (D.npolys == 0) throw F4Error{F4_E_ARG, "row basis index out of range"};
    SigBufs SB;
    sig_of(c, D, S, SB);
    const u32 w = lane_bits(D.n);
    DBuf<u8> Rd(&c.pool, (u64)r * sizeof(f4_rowspec));
    upload(c, Rd.ptr, R, (u64)r * sizeof(f4_rowspec));
    u32 max_deg = 0;
    {
        DBuf<u32> info(&c.pool, 4 * ROWS_SLOTS);
        fill_u32(info.ptr, 4 * ROWS_SLOTS, 0, s);
        hipLaunchKernelGGL(k_rows_check, dim3(std::min<u32>(4096, ceil_div(r, 256))), dim3(256), 0, s,
                           (const f4_rowspec*)Rd.ptr, r, D.lm.ptr, D.npolys, D.n, w, info.ptr);
        F4_LAUNCH_CHECK();
        u32 hi[4];
        rows_info(c, info.ptr, hi);
        if (hi[0] & 1) throw F4Error{F4_E_ARG, "row basis index out of range or shift not a monomial"};
        if (hi[0] & 2) throw F4Error{F4_E_RANGE, "exponent lane overflow"};
        max_deg = hi[1];
    }
    u32 max_len = 1;
    {
        std::vector<u64> off(D.npolys + 1);
        readback(c, off.data(), D.off.ptr, off.size() * 8);
        for (u32 k = 0; k < D.npolys; ++k) max_len = std::max<u32>(max_len, (u32)(off[k + 1] - off[k]));
    }
    hipEvent_t e0, e1;
    F4_HIP_TRY(hipEventCreate(&e0));
    F4_HIP_TRY(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    DBuf<u8> fl(&c.pool, flags ? r : 1);
    DBuf<u64> t2;
    DBuf<u32> k2, cnt, ord;
    u32 info[4];
    F4_HIP_TRY(hipEventRecord(e0, s));
    // the records are (t, k, pad): t every 2 words, k every 4 words from word 2
    sig_filter_dev(c, SB, (const u64*)Rd.ptr, 2, (const u32*)Rd.ptr + 2, 4, r, flags ? fl.ptr : nullptr, t2, k2,
                   cnt, info);
    const u32 nk = info[1];
    if (order) sig_schedule_dev(c, SB, t2.ptr, k2.ptr, cnt.ptr, nk, max_deg, max_len, D.lm.ptr, D.len.ptr, ord);
    F4_HIP_TRY(hipEventRecord(e1, s));
    if (flags) readback(c, flags, fl.ptr, r);
    if (kept && nk) {
        std::vector<u64> ht(nk);
        std::vector<u32> hk(nk);
        readback(c, ht.data(), t2.ptr, (u64)nk * 8);
        readback(c, hk.data(), k2.ptr, (u64)nk * 4);
        for (u32 q = 0; q < nk; ++q) {
            kept[q].t = ht[q];
            kept[q].k = hk[q];
            kept[q].pad = 0;
        }
    }
    if (order && nk) readback(c, order, ord.ptr, (u64)nk * 4);
    F4_HIP_TRY(hipEventSynchronize(e1));
    *nkept = nk;
    if (st) {
        st->kept = info[1];
        st->syzygy = info[2];
        st->rewritten = info[3];
        st->pad = 0;
        float ms = 0;
        F4_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        st->t_device_ms = ms;
    }
    F4_API_END(X)
}

int f4_build_matrix_sig(f4_ctx* X, uint32_t p, const f4_polys* G, const uint8_t* active, const f4_sigs* S,
                        const f4_rowspec* R, uint32_t r, f4_matrix** A, f4_sig_stats* st, void* stream) {
    F4_API_BEGIN(X)
    if (!A || !G || !active || !R || !r || !is_odd_prime(p) || p >= (1u << 31))
        throw F4Error{F4_E_ARG, "bad argument"};
    *A = nullptr;
    set_stream(X, stream);
    Ctx& c = X->c;
    hipStream_t s = c.stream;
    DevG D;
    load_polys(c, p, G, D, true);
    SigBufs SB;
    sig_of(c, D, S, SB);
    DBuf<u8> Rd;
    DBuf<u64> rt, t2;
    DBuf<u32> rk, k2, cnt;
    u32 r0 = 0, deg = 0;
    plan_rows(c, D, R, r, Rd, rt, rk, r0, deg);
    hipEvent_t e0, e1;
    F4_HIP_TRY(hipEventCreate(&e0));
    F4_HIP_TRY(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    F4_HIP_TRY(hipEventRecord(e0, s));
    u32 info[4];
    sig_filter_dev(c, SB, rt.ptr, 1, rk.ptr, 1, r0, nullptr, t2, k2, cnt, info);
    if (info[1] == 0) throw F4Error{F4_E_ARG, "no admissible row"};
    std::vector<u32> act;
    for (u32 g = D.npolys; g-- > 0;)
        if (active[g]) act.push_back(g);
    BuildArgs a;
    a.G = devg_view(D);
    a.rows_t_dev = t2.ptr;
    a.rows_k_dev = k2.ptr;
    a.r0 = info[1];
    a.active_host = act.data();
    a.nactive = (u32)act.size();
    a.D = deg;
    a.closure = true;
    a.sig_dev = SB.dev;
    *A = build_one(X, p, a);
    F4_HIP_TRY(hipEventRecord(e1, s));
    F4_HIP_TRY(hipEventSynchronize(e1));
    if (st) {
        st->kept = info[1];
        st->syzygy = info[2];
        st->rewritten = info[3];
        st->pad = 0;
        float ms = 0;
        F4_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        st->t_device_ms = ms;
    }
    F4_API_END(X)
}

int f4_matrix_from_csr(f4_ctx* X, uint32_t r, uint32_t N, const uint32_t* row_ptr, const uint32_t* col_ind,
                       const uint32_t* val, f4_matrix** A, void* stream) {
    F4_API_BEGIN(X)
    if (!A || !row_ptr || (!col_ind && row_ptr[r]) || (!val && row_ptr[r])) throw F4Error{F4_E_ARG, "bad argument"};
    *A = nullptr;
    set_stream(X, stream);
    Ctx& c = X->c;
    const u32 nnz = row_ptr[r];
    for (u32 i = 0; i < r; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) throw F4Error{F4_E_ARG, "row_ptr not monotone"};
        for (u32 e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col_ind[e] >= N) throw F4Error{F4_E_ARG, "column out of range"};
            if (e > row_ptr[i] && col_ind[e] <= col_ind[e - 1]) throw F4Error{F4_E_ARG, "columns not ascending"};
            if (val[e] == 0) throw F4Error{F4_E_ARG, "explicit zero"};
        }
    }
    f4_matrix* M = new f4_matrix();
    M->owner = X;
    Matrix& m = M->m;
    m.S = 1;
    m.R = r;
    m.nnz = nnz;
    m.sys.assign(1, SysPart());
    m.sys[0].r = r;
    m.sys[0].N = N;
    m.sys[0].nnz = nnz;
    m.row_sys.reset(&c.pool, std::max<u32>(r, 1));
    fill_u32(m.row_sys.ptr, r, 0, c.stream);
    m.row_ptr.reset(&c.pool, (u64)r + 1);
    m.col_ind.reset(&c.pool, std::max<u32>(nnz, 1));
    m.val.reset(&c.pool, std::max<u32>(nnz, 1));
    upload(c, m.row_ptr.ptr, row_ptr, ((u64)r + 1) * 4);
    upload(c, m.col_ind.ptr, col_ind, (u64)nnz * 4);
    upload(c, m.val.ptr, val, (u64)nnz * 4);
    X->matrices.insert(M);
    *A = M;
    F4_API_END(X)
}

// Checks f4_spmm's arguments, builds the transpose when asked for the first
// time, and returns the launch of one product.
static std::function<void()> spmm_call(f4_ctx* X, uint32_t p, f4_matrix* A, int trans, uint32_t b,
                                       const uint32_t* Xin, uint32_t* Y) {
    if (!A || A->owner != X || X->matrices.count(A) == 0) throw F4Error{F4_E_STATE, "unknown matrix handle"};
    if (!is_odd_prime(p) || p >= (1u << 31) || b == 0 || b > 64 || (trans != 0 && trans != 1))
        throw F4Error{F4_E_ARG, "bad argument"};
    if (A->m.S != 1) throw F4Error{F4_E_ARG, "matrix of a batch"};
    const SysPart& P = A->m.sys[0];
    const u32 nout = trans ? P.N : P.r, nin = trans ? P.r : P.N;
    if ((nout && !Y) || (nin && P.nnz && !Xin)) throw F4Error{F4_E_ARG, "null block"};
    Ctx& c = X->c;
    if (!trans) {
        const u32* ptr = A->m.row_ptr.ptr;
        const u32* idx = A->m.col_ind.ptr;
        const u32* val = A->m.val.ptr;
        const u32 r = P.r;
        return [&c, p, r, b, ptr, idx, val, Xin, Y]() { spmm_run(c.stream, p, r, b, ptr, idx, val, Xin, Y); };
    }
    if (!A->has_t) {
        csr_transpose(c, P.r, P.N, P.nnz, A->m.row_ptr.ptr, A->m.col_ind.ptr, A->m.val.ptr, A->t_ptr, A->t_idx,
                      A->t_val);
        A->has_t = true;
    }
    const u32* ptr = A->t_ptr.ptr;
    const u32* idx = A->t_idx.ptr;
    const u32* val = A->t_val.ptr;
    const u32 N = P.N;
    return [&c, p, N, b, ptr, idx, val, Xin, Y]() { spmm_run(c.stream, p, N, b, ptr, idx, val, Xin, Y); };
}

int f4_spmm(f4_ctx* X, uint32_t p, f4_matrix* A, int trans, uint32_t b, const uint32_t* Xin, uint32_t* Y,
            void* stream) {
    F4_API_BEGIN(X)
    set_stream(X, stream);
    spmm_call(X, p, A, trans, b, Xin, Y)();
    F4_API_END(X)
}

// Block Wiedemann: the handle's CSR and its transpose (built on first use, kept
// with the handle) and the transpose's values times d (a diagonal of N
// elements, device).
static BwCsr bw_prepare(f4_ctx* X, uint32_t p, f4_matrix* A, const uint32_t* d, DBuf<u32>& tval_d) {
    if (!A || A->owner != X || X->matrices.count(A) == 0) throw F4Error{F4_E_STATE, "unknown matrix handle"};
    if (A->m.S != 1) throw F4Error{F4_E_ARG, "matrix of a batch"};
    const SysPart& P = A->m.sys[0];
    if (P.N && !d) throw F4Error{F4_E_ARG, "null diagonal"};
    Ctx& c = X->c;
    if (!A->has_t) {
        csr_transpose(c, P.r, P.N, P.nnz, A->m.row_ptr.ptr, A->m.col_ind.ptr, A->m.val.ptr, A->t_ptr, A->t_idx,
                      A->t_val);
        A->has_t = true;
    }
    BwCsr B;
    B.r = P.r;
    B.N = P.N;
    B.nnz = P.nnz;
    B.ptr = A->m.row_ptr.ptr;
    B.idx = A->m.col_ind.ptr;
    B.val = A->m.val.ptr;
    B.tptr = A->t_ptr.ptr;
    B.tidx = A->t_idx.ptr;
    B.tval = A->t_val.ptr;
    tval_d.reset(&c.pool, std::max<u64>(P.nnz, 1));
    B.tval_d = tval_d.ptr;
    bw_scale_transpose(c, p, B, d, tval_d.ptr);
    return B;
}

static void bw_check(uint32_t p, uint32_t b, uint32_t L) {
    if (!is_odd_prime(p) || p >= (1u << 31) || b == 0 || b > F4_BW_MAX_B || L == 0)
        throw F4Error{F4_E_ARG, "bad argument"};
}

int f4_bw_sequence(f4_ctx* X, uint32_t p, f4_matrix* A, uint32_t b, const uint32_t* d, const uint32_t* Xp,
                   const uint32_t* Yp, uint32_t L, uint32_t* S, void* stream) {
    F4_API_BEGIN(X)
    bw_check(p, b, L);
    if (!S || !Xp || !Yp) throw F4Error{F4_E_ARG, "null block"};
    set_stream(X, stream);
    DBuf<u32> tvd;
    const BwCsr B = bw_prepare(X, p, A, d, tvd);
    bw_sequence(X->c, p, B, b, Xp, Yp, L, S);
    F4_API_END(X)
}

int f4_bw_mbasis(f4_ctx* X, uint32_t p, uint32_t b, uint32_t L, const uint32_t* S, uint32_t* P, uint32_t* shifts,
                 void* stream) {
    F4_API_BEGIN(X)
    bw_check(p, b, L);
    if (!S || !P || !shifts) throw F4Error{F4_E_ARG, "null array"};
    set_stream(X, stream);
    bw_mbasis(X->c, p, b, L, S, P, shifts);
    F4_API_END(X)
}

int f4_block_wiedemann(f4_ctx* X, uint32_t p, f4_matrix* A, uint32_t b, const uint32_t* d, const uint32_t* Xp,
                       const uint32_t* Yp, uint32_t* V, uint32_t cap, uint32_t* nvec, f4_bw_stats* st) {
    F4_API_BEGIN(X)
    if (!A || A->owner != X || X->matrices.count(A) == 0) throw F4Error{F4_E_STATE, "unknown matrix handle"};
    if (A->m.S != 1) throw F4Error{F4_E_ARG, "matrix of a batch"};
    const u32 r = A->m.sys[0].r;
    const u32 L = 2 * ceil_div(r, std::max<u32>(b, 1)) + 4;
    bw_check(p, b, L);
    if (!nvec || !Xp || !Yp || (cap && !V)) throw F4Error{F4_E_ARG, "null argument"};
    *nvec = 0;
    set_stream(X, nullptr);
    Ctx& c = X->c;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point z) {
        return std::chrono::duration<double, std::milli>(z - a).count();
    };
    const auto t0 = now();
    DBuf<u32> tvd;
    const BwCsr B = bw_prepare(X, p, A, d, tvd);
    const u32 m = 2 * b, W = L + 2;
    DBuf<u32> S(&c.pool, (u64)L * b * b), P(&c.pool, (u64)m * m * W), sh(&c.pool, m);
    bw_sequence(c, p, B, b, Xp, Yp, L, S.ptr);
    F4_HIP_TRY(hipStreamSynchronize(c.stream));
    const auto t1 = now();
    bw_mbasis(c, p, b, L, S.ptr, P.ptr, sh.ptr);
    std::vector<u32> hP((u64)m * m * W), hs(m);
    F4_HIP_TRY(hipMemcpyAsync(hP.data(), P.ptr, hP.size() * 4, hipMemcpyDeviceToHost, c.stream));
    F4_HIP_TRY(hipMemcpyAsync(hs.data(), sh.ptr, m * 4, hipMemcpyDeviceToHost, c.stream));
    F4_HIP_TRY(hipStreamSynchronize(c.stream));
    const auto t2 = now();
    // generators: rows (g, h) with g != 0 and 2 s + 2 <= L, in the order of
    // (shift, index); f_m = g_{s - m}, shifted down past its zero low
    // coefficients (m0), so column j evaluates sum_m B^m Y f_{m + m0}
    std::vector<u32> rows(m);
    for (u32 i = 0; i < m; ++i) rows[i] = i;
    std::stable_sort(rows.begin(), rows.end(), [&](u32 a, u32 z) { return hs[a] < hs[z]; });
    struct Gen {
        u32 s, m0;
        std::vector<u32> f;  // (s + 1) x b: f[m * b + k] = g_k at s - m
    };
    std::vector<Gen> gens;
    for (u32 i : rows) {
        const u32 sdeg = hs[i];
        if (2 * (u64)sdeg + 2 > L) continue;
        Gen g;
        g.s = sdeg;
        g.f.assign((u64)(sdeg + 1) * b, 0);
        bool any = false;
        for (u32 mm = 0; mm <= sdeg; ++mm)
            for (u32 k = 0; k < b; ++k) {
                const u32 v = hP[((u64)i * m + k) * W + (sdeg - mm)];
                g.f[(u64)mm * b + k] = v;
                any = any || v;
            }
        if (!any) continue;
        g.m0 = 0;
        while (g.m0 <= sdeg) {
            bool nz = false;
            for (u32 k = 0; k < b; ++k) nz = nz || g.f[(u64)g.m0 * b + k];
            if (nz) break;
            ++g.m0;
        }
        gens.push_back(std::move(g));
    }
    const u32 w = (u32)gens.size();
    u32 found = 0;
    if (w) {
        u32 Dmax = 0, smax = 0;
        for (const Gen& g : gens) {
            Dmax = std::max(Dmax, g.s - g.m0);
            smax = std::max(smax, g.s);
        }
        const u32 E = smax + 3;  // iterates v_0 .. v_{s+2}: the first zero one is at most v_{s+2}
        std::vector<u32> hF((u64)(Dmax + 1) * b * w, 0);
        for (u32 j = 0; j < w; ++j) {
            const Gen& g = gens[j];
            for (u32 mm = 0; mm + g.m0 <= g.s; ++mm)
                for (u32 k = 0; k < b; ++k) hF[((u64)mm * b + k) * w + j] = g.f[(u64)(mm + g.m0) * b + k];
        }
        DBuf<u32> F(&c.pool, hF.size()), K(&c.pool, std::max<u64>((u64)r * w, 1)), nzh(&c.pool, (u64)E * w),
            nzc(&c.pool, w);
        F4_HIP_TRY(hipMemcpyAsync(F.ptr, hF.data(), hF.size() * 4, hipMemcpyHostToDevice, c.stream));
        bw_kernel_vectors(c, p, B, b, Yp, w, Dmax, F.ptr, E, K.ptr, nzh.ptr, nzc.ptr);
        std::vector<u32> hK((u64)r * w), hz((u64)E * w), hc(w);
        F4_HIP_TRY(hipMemcpyAsync(hK.data(), K.ptr, hK.size() * 4, hipMemcpyDeviceToHost, c.stream));
        F4_HIP_TRY(hipMemcpyAsync(hz.data(), nzh.ptr, hz.size() * 4, hipMemcpyDeviceToHost, c.stream));
        F4_HIP_TRY(hipMemcpyAsync(hc.data(), nzc.ptr, w * 4, hipMemcpyDeviceToHost, c.stream));
        F4_HIP_TRY(hipStreamSynchronize(c.stream));
        for (u32 j = 0; j < w; ++j) {
            // first zero iterate: the one before it is in ker B
            u32 z = E;
            for (u32 e = 0; e < E; ++e)
                if (!hz[(u64)e * w + j]) {
                    z = e;
                    break;
                }
            if (z == 0 || z > gens[j].s + 2 || z == E) continue;
            if (hc[j]) continue;  // in ker B but A^T v != 0: not a syzygy
            if (found < cap)
                for (u32 g = 0; g < r; ++g) V[(u64)found * r + g] = hK[(u64)g * w + j];
            ++found;
        }
    }
    const auto t3 = now();
    *nvec = found;
    if (st) {
        st->L = L;
        st->generators = w;
        st->t_sequence_ms = ms(t0, t1);
        st->t_mbasis_ms = ms(t1, t2);
        st->t_vectors_ms = ms(t2, t3);
    }
    F4_API_END(X)
}

int f4_spmm_noalloc(f4_ctx* X, uint32_t p, uint32_t r, uint32_t N, uint64_t nnz, const uint32_t* row_ptr,
                    const uint32_t* col_ind, const uint32_t* val, int trans, uint32_t b, const uint32_t* Xin,
                    uint32_t* Y, void* stream) {
    F4_API_BEGIN(X)
    if (!is_odd_prime(p) || p >= (1u << 31) || b == 0 || b > 64 || (trans != 0 && trans != 1) || !row_ptr ||
        nnz >= (1ull << 32) || (nnz && (!col_ind || !val)))
        throw F4Error{F4_E_ARG, "bad argument"};
    const u32 nout = trans ? N : r, nin = trans ? r : N;
    if ((nout && !Y) || (nin && nnz && !Xin)) throw F4Error{F4_E_ARG, "null block"};
    const u64 need = spmm_noalloc_words(N, nnz, trans) * 4;
    if (need > F4_NOALLOC_SCRATCH_BYTES)
        throw F4Error{F4_E_RANGE, "the transpose needs " + std::to_string(need) + " bytes of scratch; the maximum is " +
                                      std::to_string((u64)F4_NOALLOC_SCRATCH_BYTES)};
    set_stream(X, stream);
    spmm_noalloc_run(X->c.stream, X->c.dev.device, p, r, N, nnz, row_ptr, col_ind, val, trans, b, Xin, Y);
    F4_API_END(X)
}

int f4_spmm_timed(f4_ctx* X, uint32_t p, f4_matrix* A, int trans, uint32_t b, const uint32_t* Xin, uint32_t* Y,
                  uint32_t reps, double* ms_per_call) {
    F4_API_BEGIN(X)
    if (reps == 0 || !ms_per_call) throw F4Error{F4_E_ARG, "bad argument"};
    set_stream(X, nullptr);
    Ctx& c = X->c;
    auto run = spmm_call(X, p, A, trans, b, Xin, Y);
    hipEvent_t e[2] = {nullptr, nullptr};
    try {
        F4_HIP_TRY(hipEventCreate(&e[0]));
        F4_HIP_TRY(hipEventCreate(&e[1]));
        F4_HIP_TRY(hipEventRecord(e[0], c.stream));
        for (u32 i = 0; i < reps; ++i) run();
        F4_HIP_TRY(hipEventRecord(e[1], c.stream));
        F4_HIP_TRY(hipEventSynchronize(e[1]));
        float ms = 0.f;
        F4_HIP_TRY(hipEventElapsedTime(&ms, e[0], e[1]));
        *ms_per_call = (double)ms / reps;
    } catch (...) {
        for (hipEvent_t v : e)
            if (v) (void)hipEventDestroy(v);
        throw;
    }
    for (hipEvent_t v : e) (void)hipEventDestroy(v);
    F4_API_END(X)
}

static f4_matrix* own_matrix(f4_ctx* X, const f4_matrix* A) {
    if (!A || A->owner != X || X->matrices.count(const_cast<f4_matrix*>(A)) == 0)
        throw F4Error{F4_E_STATE, "unknown matrix handle"};
    if (A->m.S != 1) throw F4Error{F4_E_ARG, "matrix of a batch"};
    return const_cast<f4_matrix*>(A);
}

static void schedule_view(const SchedBufs& S, f4_schedule_view* out) {
    out->W = S.W;
    out->C = S.C;
    out->sigma = S.sigma;
    out->npanels = S.npanels;
    out->nslices = S.nslices;
    out->pad = 0;
    out->padded = S.padded;
    out->perm = S.perm.ptr;
    out->panel_ptr = S.panel_ptr.ptr;
    out->slice_start = S.slice_start.ptr;
    out->slice_panel = S.slice_panel.ptr;
    out->slice_width = S.slice_width.ptr;
    out->slice_off = S.slice_off.ptr;
    out->sell_col = S.sell_col.ptr;
    out->sell_val = S.sell_val.ptr;
}

int f4_matrix_schedule(f4_ctx* X, f4_matrix* A, uint32_t W, uint32_t C, uint32_t sigma, f4_schedule_view* out,
                       void* stream) {
    F4_API_BEGIN(X)
    f4_matrix* M = own_matrix(X, A);
    if (W == 0 || C == 0 || C > 64 || sigma == 0) throw F4Error{F4_E_ARG, "bad schedule parameters"};
    set_stream(X, stream);
    const SysPart& P = M->m.sys[0];
    SchedBufs S;
    sched_build(X->c, P.r, P.N, P.nnz, M->m.row_ptr.ptr, M->m.col_ind.ptr, M->m.val.ptr, W, C, sigma, S);
    M->sched = std::move(S);
    if (out) schedule_view(M->sched, out);
    F4_API_END(X)
}

static std::function<void()> spmm_sell_call(f4_ctx* X, uint32_t p, const f4_matrix* A, uint32_t b,
                                            const uint32_t* Xin, uint32_t* Y) {
    f4_matrix* M = own_matrix(X, A);
    if (!M->sched.has) throw F4Error{F4_E_STATE, "the matrix has no block schedule (f4_matrix_schedule)"};
    if (!is_odd_prime(p) || p >= (1u << 31) || b == 0 || b > 8) throw F4Error{F4_E_ARG, "bad argument"};
    const SysPart& P = M->m.sys[0];
    if ((P.N && !Xin) || (P.r && !Y)) throw F4Error{F4_E_ARG, "null block"};
    Ctx* c = &X->c;
    return [c, p, M, b, Xin, Y]() { spmm_sell_run(c->stream, p, M->sched, b, Xin, Y); };
}

int f4_spmm_sell(f4_ctx* X, uint32_t p, const f4_matrix* A, uint32_t b, const uint32_t* Xin, uint32_t* Y,
                 void* stream) {
    F4_API_BEGIN(X)
    set_stream(X, stream);
    spmm_sell_call(X, p, A, b, Xin, Y)();
    F4_API_END(X)
}

int f4_spmm_sell_timed(f4_ctx* X, uint32_t p, const f4_matrix* A, uint32_t b, const uint32_t* Xin, uint32_t* Y,
                       uint32_t reps, double* ms_per_call) {
    F4_API_BEGIN(X)
    if (reps == 0 || !ms_per_call) throw F4Error{F4_E_ARG, "bad argument"};
    set_stream(X, nullptr);
    Ctx& c = X->c;
    auto run = spmm_sell_call(X, p, A, b, Xin, Y);
    hipEvent_t e[2] = {nullptr, nullptr};
    try {
        F4_HIP_TRY(hipEventCreate(&e[0]));
        F4_HIP_TRY(hipEventCreate(&e[1]));
        F4_HIP_TRY(hipEventRecord(e[0], c.stream));
        for (u32 i = 0; i < reps; ++i) run();
        F4_HIP_TRY(hipEventRecord(e[1], c.stream));
        F4_HIP_TRY(hipEventSynchronize(e[1]));
        float ms = 0.f;
        F4_HIP_TRY(hipEventElapsedTime(&ms, e[0], e[1]));
        *ms_per_call = (double)ms / reps;
    } catch (...) {
        for (hipEvent_t v : e)
            if (v) (void)hipEventDestroy(v);
        throw;
    }
    for (hipEvent_t v : e) (void)hipEventDestroy(v);
    F4_API_END(X)
}

int f4_device_alloc(f4_ctx* X, size_t bytes, void** ptr) {
    F4_API_BEGIN(X)
    if (!ptr) throw F4Error{F4_E_ARG, "null pointer"};
    *ptr = X->c.pool.alloc(bytes ? bytes : 1);
    F4_API_END(X)
}

int f4_device_free(f4_ctx* X, void* ptr) {
    F4_API_BEGIN(X)
    // blocks go back to the cache in stream order: wait for the work that may still use it
    F4_HIP_TRY(hipStreamSynchronize(X->c.stream));
    X->c.pool.release(ptr);
    F4_API_END(X)
}

int f4_upload(f4_ctx* X, void* dst, const void* src, size_t bytes) {
    F4_API_BEGIN(X)
    if ((!dst || !src) && bytes) throw F4Error{F4_E_ARG, "null pointer"};
    if (bytes) {
        F4_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, X->c.stream));
        F4_HIP_TRY(hipStreamSynchronize(X->c.stream));
    }
    F4_API_END(X)
}

int f4_matrix_get(const f4_matrix* A, f4_matrix_view* out) {
    if (!A || !out) return F4_E_ARG;
    const Matrix& m = A->m;
    const SysPart& P = m.sys[0];
    out->n = P.n;
    out->r = P.r;
    out->N = P.N;
    out->deg = P.deg;
    out->nnz = P.nnz;
    out->row_ptr = m.row_ptr.ptr;
    out->col_ind = m.col_ind.ptr;
    out->val = m.val.ptr;
    out->dict_keys = m.dict_keys.ptr;
    out->row_t = m.row_t.ptr;
    out->row_k = m.row_k.ptr;
    out->key_words = m.key_words;
    out->pad = 0;
    return F4_OK;
}

int f4_matrix_free(f4_matrix* A) {
    if (!A) return F4_E_ARG;
    A->owner->matrices.erase(A);
    delete A;
    return F4_OK;
}

int f4_reduce(f4_ctx* X, uint32_t p, const f4_matrix* A, f4_reduced** out, void* stream) {
    F4_API_BEGIN(X)
    if (!A || !out || !is_odd_prime(p) || p >= (1u << 31)) throw F4Error{F4_E_ARG, "bad argument"};
    *out = nullptr;
    if (A->owner != X || X->matrices.count(const_cast<f4_matrix*>(A)) == 0)
        throw F4Error{F4_E_STATE, "unknown matrix handle"};
    set_stream(X, stream);
    if (A->m.built_p != p && A->m.nnz) {
        // values not known to be residues mod p (a caller CSR, or a matrix
        // built for another prime): every stored value must lie in [1, p)
        DBuf<u32> flag(&X->c.pool, 1);
        fill_u32(flag.ptr, 1, 0, X->c.stream);
        hipLaunchKernelGGL(k_check_vals, dim3(gridn(A->m.nnz, 256, 1024)), dim3(256), 0, X->c.stream, A->m.val.ptr,
                           A->m.nnz, p, flag.ptr);
        F4_LAUNCH_CHECK();
        u32 bad = 0;
        readback(X->c, &bad, flag.ptr, 4);
        if (bad) throw F4Error{F4_E_ARG, "a matrix value is not a nonzero residue mod p"};
    }
    f4_reduced* R = new f4_reduced();
    R->owner = X;
    try {
        reduce_batch(X->c, std::vector<u32>{p}, A->m, R->r);
    } catch (...) {
        delete R;
        throw;
    }
    X->reduceds.insert(R);
    *out = R;
    F4_API_END(X)
}

int f4_reduced_get(const f4_reduced* R, f4_reduced_view* out) {
    if (!R || !out) return F4_E_ARG;
    const Reduced& r = R->r;
    const RedPart& P = r.sys[0];
    out->N = P.N;
    out->npivot = P.npivot;
    out->rho = P.rho;
    out->rank = P.rank;
    out->nnz = P.nnz;
    out->pivot_cols = r.pivot_cols.ptr;
    out->row_ptr = r.row_ptr.ptr;
    out->col_ind = r.col_ind.ptr;
    out->val = r.val.ptr;
    return F4_OK;
}

int f4_reduced_free(f4_reduced* R) {
    if (!R) return F4_E_ARG;
    R->owner->reduceds.erase(R);
    delete R;
    return F4_OK;
}

int f4_groebner(f4_ctx* X, uint32_t p, const f4_polys* F, f4_basis** gb, void* stream) {
    F4_API_BEGIN(X)
    if (!gb) throw F4Error{F4_E_ARG, "bad argument"};
    *gb = nullptr;
    set_stream(X, stream);
    SysState S;
    InitPack pk;
    init_system(X->c, S, p, F, pk);
    init_flush(X->c, pk);
    std::vector<SysState*> v{&S};
    run_f4(X->c, v);
    f4_basis* B = basis_of(X, S);
    X->bases.insert(B);
    *gb = B;
    F4_API_END(X)
}

int f4_groebner_batch(f4_ctx* X, uint32_t nsys, const uint32_t* p, const f4_polys* F, f4_basis** gb,
                      void* stream) {
    F4_API_BEGIN(X)
    if (!gb || !p || !F || nsys == 0) throw F4Error{F4_E_ARG, "bad argument"};
    for (u32 i = 0; i < nsys; ++i) gb[i] = nullptr;
    set_stream(X, stream);
    std::vector<std::unique_ptr<SysState>> own(nsys);
    std::vector<SysState*> v;
    InitPack pk;
    for (u32 i = 0; i < nsys; ++i) {
        own[i].reset(new SysState());
        init_system(X->c, *own[i], p[i], &F[i], pk);
        v.push_back(own[i].get());
    }
    init_flush(X->c, pk);
    run_f4(X->c, v);
    for (u32 i = 0; i < nsys; ++i) {
        gb[i] = basis_of(X, *own[i]);
        X->bases.insert(gb[i]);
    }
    F4_API_END(X)
}

int f4_basis_view(const f4_basis* B, f4_polys* out) {
    if (!B || !out) return F4_E_ARG;
    out->n = B->n;
    out->npolys = (u32)(B->off.size() - 1);
    out->mon = B->mon.data();
    out->coeff = B->coeff.data();
    out->offset = B->off.data();
    out->on_device = 0;
    return F4_OK;
}

int f4_basis_stats(const f4_basis* B, const f4_step_stats** steps, uint32_t* nsteps) {
    if (!B || !steps || !nsteps) return F4_E_ARG;
    *steps = B->steps.data();
    *nsteps = (u32)B->steps.size();
    return F4_OK;
}

int f4_basis_free(f4_basis* B) {
    if (!B) return F4_E_ARG;
    B->owner->bases.erase(B);
    delete B;
    return F4_OK;
}


// ---------------------------------------------------------------- serving
}  // extern "C"

static u64 footprint_of(u32 n, u32 m) {
    // degree of regularity of m generic quadratics in n variables
    std::vector<long double> hs(64, 0.0L);
    hs[0] = 1;
    for (u32 k = 0; k < m; ++k)  // multiply by (1 - t^2)
        for (int d = 63; d >= 2; --d) hs[d] -= hs[d - 2];
    for (u32 k = 0; k < n; ++k)  // divide by (1 - t)
        for (int d = 1; d < 64; ++d) hs[d] += hs[d - 1];
    u32 D = 63;
    for (u32 d = 0; d < 64; ++d)
        if (hs[d] <= 0) {
            D = d;
            break;
        }
    if (D < 2) D = 2;
    const long double a = (long double)binom_host(n + D, n), b = (long double)binom_host(n + D - 1, n);
    const long double bytes = 8.0L * a * b + (long double)(64u << 20);
    return bytes > 1.8e19L ? ~0ull : (u64)bytes;
}

extern "C" {

int f4_server_footprint(uint32_t n, uint32_t m, uint64_t* bytes) {
    if (!bytes || n == 0 || n > 14) return F4_E_ARG;
    *bytes = footprint_of(n, m);
    return F4_OK;
}

int f4_server_create(f4_ctx* X, uint64_t hbm_budget, uint32_t max_slots, f4_server** out) {
    F4_API_BEGIN(X)
    if (!out || max_slots == 0) throw F4Error{F4_E_ARG, "bad argument"};
    f4_server* S = new f4_server();
    S->owner = X;
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    X->servers.insert(S);
    *out = S;
    F4_API_END(X)
}

int f4_server_submit(f4_server* srv, uint32_t p, const f4_polys* F, uint64_t* ticket) {
    if (!srv) return F4_E_ARG;
    f4_ctx* X = srv->owner;
    F4_API_BEGIN(X)
    if (!F || !ticket) throw F4Error{F4_E_ARG, "bad argument"};
    const u64 fp = footprint_of(F->n ? F->n : 1, F->npolys);
    if (srv->reqs.size() >= srv->max_slots || srv->used + fp > srv->budget) return F4_E_BUSY;
    set_stream(X, nullptr);
    ServerReq r;
    r.footprint = fp;
    r.st.reset(new SysState());
    InitPack pk;
    init_system(X->c, *r.st, p, F, pk);
    init_flush(X->c, pk);
    srv->used += fp;
    const u64 t = srv->next_ticket++;
    srv->reqs.emplace(t, std::move(r));
    *ticket = t;
    F4_API_END(X)
}

int f4_server_step(f4_server* srv, uint32_t* completed) {
    if (!srv) return F4_E_ARG;
    f4_ctx* X = srv->owner;
    F4_API_BEGIN(X)
    set_stream(X, nullptr);
    std::vector<SysState*> live;
    for (auto& kv : srv->reqs)
        if (!kv.second.st->done) live.push_back(kv.second.st.get());
    f4_iterate(X->c, live);
    f4_finish(X->c, live);
    u32 k = 0;
    for (SysState* S : live) k += S->done ? 1 : 0;
    if (completed) *completed = k;
    F4_API_END(X)
}

int f4_server_poll(f4_server* srv, uint64_t ticket, f4_basis** gb, int* done) {
    if (!srv) return F4_E_ARG;
    f4_ctx* X = srv->owner;
    F4_API_BEGIN(X)
    if (!gb || !done) throw F4Error{F4_E_ARG, "bad argument"};
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) throw F4Error{F4_E_STATE, "unknown ticket"};
    *done = 0;
    *gb = nullptr;
    if (it->second.st->done) {
        f4_basis* B = basis_of(X, *it->second.st);
        X->bases.insert(B);
        *gb = B;
        *done = 1;
        srv->used -= it->second.footprint;
        srv->reqs.erase(it);
    }
    F4_API_END(X)
}

int f4_server_load(const f4_server* srv, uint32_t* resident, uint32_t* running, uint64_t* used) {
    if (!srv) return F4_E_ARG;
    u32 run = 0;
    for (auto& kv : srv->reqs) run += kv.second.st->done ? 0 : 1;
    if (resident) *resident = (u32)srv->reqs.size();
    if (running) *running = run;
    if (used) *used = srv->used;
    return F4_OK;
}

int f4_server_destroy(f4_server* srv) {
    if (!srv) return F4_E_ARG;
    srv->owner->servers.erase(srv);
    delete srv;
    return F4_OK;
}

}  // extern "C"
