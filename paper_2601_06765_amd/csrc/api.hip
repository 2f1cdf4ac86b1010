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
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <set>

#include "../../include/f4.h"
#include "internal.hpp"

// ------------------------------------------------------------ handles
struct f4_matrix;
struct f4_reduced;
struct f4_basis;
struct f4_ctx {
    Ctx c;
    std::set<f4_matrix*> matrices;
    std::set<f4_reduced*> reduceds;
    std::set<f4_basis*> bases;
};
struct f4_matrix {
    f4_ctx* owner;
    Matrix m;
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
    if (c.staging_pending) {
        F4_HIP_TRY(hipEventSynchronize(c.staging_done));
        c.staging_pending = false;
    }
    if (bytes > c.pinned_bytes) {
        if (c.pinned) F4_HIP_TRY(hipHostFree(c.pinned));
        c.pinned = nullptr;
        size_t nb = std::max(bytes, (size_t)2 * c.pinned_bytes);
        F4_HIP_TRY(hipHostMalloc((void**)&c.pinned, nb, hipHostMallocDefault));
        c.pinned_bytes = nb;
    }
    return c.pinned;
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
}

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

float event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    if (a && b) F4_HIP_TRY(hipEventElapsedTime(&ms, a, b));
    return ms;
}

// ----------------------------------------------------- packed monomials (host)
// SWAR forms valid while every exponent is below 2^(w-1) (guard bit free).
struct MonoOps {
    u32 n, w;
    u64 lanes, H;  // lane bits, lane top bits
    void init(u32 n_) {
        n = n_;
        w = lane_bits(n);
        lanes = (n * w >= 64) ? ~0ull : ((1ull << (n * w)) - 1);
        H = 0;
        for (u32 i = 0; i < n; ++i) H |= 1ull << (w * i + w - 1);
    }
    bool divides(u64 a, u64 b) const {  // a | b
        return ((((b & lanes) | H) - (a & lanes)) & H) == H;
    }
    u64 lcm(u64 a, u64 b) const {
        u64 ge = (((a & lanes) | H) - (b & lanes)) & H;  // lanes where a >= b
        u64 m = (ge >> (w - 1)) * ((1ull << w) - 1);
        u64 l = (a & m) | (b & ~m & lanes);
        u32 d = 0;
        for (u32 i = 0; i < n; ++i) d += (u32)((l >> (w * i)) & ((1u << w) - 1));
        return l | ((u64)d << 56);
    }
    bool coprime(u64 a, u64 b) const {
        for (u32 i = 0; i < n; ++i)
            if (mono_exp(a, i, w) && mono_exp(b, i, w)) return false;
        return true;
    }
    u64 order_key(u64 P) const { return P ^ lanes; }
};

// ------------------------------------------------------------ driver state
struct HPair {
    u32 i, j;
    u64 lcm;
};

struct DevG {
    u32 n = 0, npolys = 0;
    u64 nterms = 0;
    DBuf<u64> mon, off, lm;
    DBuf<u32> coeff, len;
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

static void devg_reserve(Ctx& c, DevG& G, u64 terms, u32 polys) {
    if (terms > G.cap_terms) {
        u64 cap = std::max<u64>(terms, 2 * G.cap_terms);
        DBuf<u64> m2(&c.pool, cap);
        DBuf<u32> c2(&c.pool, cap);
        if (G.nterms) {
            F4_HIP_TRY(hipMemcpyAsync(m2.ptr, G.mon.ptr, G.nterms * 8, hipMemcpyDeviceToDevice, c.stream));
            F4_HIP_TRY(hipMemcpyAsync(c2.ptr, G.coeff.ptr, G.nterms * 4, hipMemcpyDeviceToDevice, c.stream));
        }
        G.mon = std::move(m2);
        G.coeff = std::move(c2);
        G.cap_terms = cap;
    }
    if ((u64)polys + 1 > G.cap_polys) {
        u64 cap = std::max<u64>((u64)polys + 1, 2 * G.cap_polys);
        DBuf<u64> o2(&c.pool, cap), l2(&c.pool, cap);
        DBuf<u32> n2(&c.pool, cap);
        if (G.npolys) {
            F4_HIP_TRY(hipMemcpyAsync(o2.ptr, G.off.ptr, ((u64)G.npolys + 1) * 8, hipMemcpyDeviceToDevice, c.stream));
            F4_HIP_TRY(hipMemcpyAsync(l2.ptr, G.lm.ptr, (u64)G.npolys * 8, hipMemcpyDeviceToDevice, c.stream));
            F4_HIP_TRY(hipMemcpyAsync(n2.ptr, G.len.ptr, (u64)G.npolys * 4, hipMemcpyDeviceToDevice, c.stream));
        }
        G.off = std::move(o2);
        G.lm = std::move(l2);
        G.len = std::move(n2);
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

// Gebauer-Moeller update inserting basis element h (Becker-Weispfenning):
// new pairs (h, g) are pruned by the chain and product criteria, old pairs
// whose lcm is a proper multiple witnessed by LM(h) are removed, and basis
// elements whose leading monomial LM(h) divides become inactive.
static void gm_update(const MonoOps& mo, std::vector<u64>& lm, std::vector<u8>& active, std::vector<HPair>& P,
                      u32 h) {
    const u64 lh = lm[h];
    std::vector<u32> C;
    for (u32 g = 0; g < h; ++g)
        if (active[g]) C.push_back(g);
    const size_t nc = C.size();
    std::vector<u64> L(nc);
    for (size_t a = 0; a < nc; ++a) L[a] = mo.lcm(lh, lm[C[a]]);
    std::vector<u8> kept(nc, 0);
    for (size_t a = 0; a < nc; ++a) {
        bool keep = mo.coprime(lh, lm[C[a]]);
        if (!keep) {
            bool covered = false;
            // still-pending pairs (b > a) and already kept ones (b < a)
            for (size_t b = 0; b < nc && !covered; ++b) {
                if (b == a) continue;
                if ((b > a || kept[b]) && mo.divides(L[b], L[a])) covered = true;
            }
            keep = !covered;
        }
        kept[a] = keep;
    }
    std::vector<HPair> Pn;
    Pn.reserve(P.size() + nc);
    for (const HPair& q : P) {
        bool drop = mo.divides(lh, q.lcm) && mo.lcm(lm[q.i], lh) != q.lcm && mo.lcm(lh, lm[q.j]) != q.lcm;
        if (!drop) Pn.push_back(q);
    }
    for (size_t a = 0; a < nc; ++a)
        if (kept[a] && !mo.coprime(lh, lm[C[a]])) Pn.push_back({C[a], h, L[a]});
    P.swap(Pn);
    for (u32 g = 0; g < h; ++g)
        if (active[g] && mo.divides(lh, lm[g])) active[g] = 0;
    active[h] = 1;
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

// A basis given through the C-ABI, moved into device SoA with metadata.
static void load_polys(Ctx& c, const f4_polys* G, DevG& D) {
    if (!G || G->n == 0 || G->n > 14) throw F4Error{F4_E_ARG, "bad number of variables"};
    D.n = G->n;
    std::vector<u64> off(G->npolys + 1);
    if (G->on_device)
        readback(c, off.data(), G->offset, off.size() * 8);
    else
        std::memcpy(off.data(), G->offset, off.size() * 8);
    const u64 nt = off[G->npolys];
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
    for (u32 k = 0; k < G->npolys; ++k)
        if (off[k + 1] <= off[k]) throw F4Error{F4_E_ARG, "zero polynomial in basis"};
    if (G->npolys) {
        hipLaunchKernelGGL(k_basis_meta, dim3(gridn(G->npolys, 256, 1024)), dim3(256), 0, c.stream, D.mon.ptr,
                           D.off.ptr, 0u, G->npolys, D.lm.ptr, D.len.ptr);
        F4_LAUNCH_CHECK();
    }
}

static u32 deg_of(u64 P) { return (u32)(P >> 56); }

// One F4 step's matrix for given halves; rows deduplicated on the host.
static void build_step(Ctx& c, const DevG& D, std::vector<std::pair<u64, u32>>& rows, const std::vector<u32>& act,
                       u32 deg, bool closure, Matrix& A) {
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    const u32 r0 = (u32)rows.size();
    std::vector<u64> t(r0);
    std::vector<u32> k(r0);
    for (u32 i = 0; i < r0; ++i) {
        t[i] = rows[i].first;
        k[i] = rows[i].second;
    }
    DBuf<u64> dt(&c.pool, r0);
    DBuf<u32> dk(&c.pool, r0), da(&c.pool, std::max<size_t>(act.size(), 1));
    upload(c, dt.ptr, t.data(), (u64)r0 * 8);
    upload(c, dk.ptr, k.data(), (u64)r0 * 4);
    upload(c, da.ptr, act.data(), act.size() * 4);
    BuildArgs a;
    a.G = devg_view(D);
    a.rows_t = dt.ptr;
    a.rows_k = dk.ptr;
    a.r0 = r0;
    a.active = da.ptr;
    a.nactive = (u32)act.size();
    a.D = deg;
    a.closure = closure;
    build_matrix(c, a, A);
}

// ====================================================================== API
extern "C" {

int f4_create(f4_ctx** out, int device, const f4_opts* opts) {
    if (!out) return F4_E_ARG;
    *out = nullptr;
    f4_ctx* X = new (std::nothrow) f4_ctx();
    if (!X) return F4_E_NOMEM;
    try {
        F4_HIP_TRY(hipSetDevice(device));
        hipDeviceProp_t prop;
        F4_HIP_TRY(hipGetDeviceProperties(&prop, device));
        X->c.dev.device = device;
        X->c.dev.cus = prop.multiProcessorCount;
        X->c.dev.max_lds = prop.sharedMemPerBlock;
        X->c.flags = opts ? opts->flags : 0;
        F4_HIP_TRY(hipStreamCreateWithFlags(&X->c.own_stream, hipStreamNonBlocking));
        X->c.stream = X->c.own_stream;
        F4_HIP_TRY(hipEventCreateWithFlags(&X->c.staging_done, hipEventDisableTiming));
        staging(X->c, 1 << 20);
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
    if (X->c.own_stream) (void)hipStreamDestroy(X->c.own_stream);
    delete X;
    return F4_OK;
}

const char* f4_last_error(const f4_ctx* X) { return X ? X->c.last_error.c_str() : "null context"; }

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
    load_polys(c, G, D);
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
    f4_matrix* M = new f4_matrix();
    M->owner = X;
    try {
        build_step(c, D, rows, act, deg, true, M->m);
    } catch (...) {
        delete M;
        throw;
    }
    X->matrices.insert(M);
    *A = M;
    F4_API_END(X)
}

int f4_build_matrix_rows(f4_ctx* X, uint32_t p, const f4_polys* G, const f4_rowspec* R, uint32_t r, f4_matrix** A,
                         void* stream) {
    F4_API_BEGIN(X)
    if (!A || !G || !R || !r || !is_odd_prime(p) || p >= (1u << 31)) throw F4Error{F4_E_ARG, "bad argument"};
    *A = nullptr;
    set_stream(X, stream);
    Ctx& c = X->c;
    DevG D;
    load_polys(c, G, D);
    std::vector<u64> lm(D.npolys);
    readback(c, lm.data(), D.lm.ptr, (u64)D.npolys * 8);
    const u32 w = lane_bits(D.n);
    std::vector<std::pair<u64, u32>> rows;
    u32 deg = 0;
    for (u32 i = 0; i < r; ++i) {
        if (R[i].k >= D.npolys) throw F4Error{F4_E_ARG, "row basis index out of range"};
        // t * LM(g): every lane must stay below 2^w
        for (u32 v = 0; v < D.n; ++v)
            if (mono_exp(R[i].t, v, w) + mono_exp(lm[R[i].k], v, w) >= (1u << w))
                throw F4Error{F4_E_RANGE, "exponent lane overflow"};
        deg = std::max(deg, deg_of(R[i].t + lm[R[i].k]));
        rows.push_back({R[i].t, R[i].k});
    }
    if (deg >= (1u << w)) throw F4Error{F4_E_RANGE, "degree overflows an exponent lane"};
    std::vector<u32> act;
    f4_matrix* M = new f4_matrix();
    M->owner = X;
    try {
        build_step(c, D, rows, act, deg, false, M->m);
    } catch (...) {
        delete M;
        throw;
    }
    X->matrices.insert(M);
    *A = M;
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
    m.r = r;
    m.N = N;
    m.nnz = nnz;
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

int f4_matrix_get(const f4_matrix* A, f4_matrix_view* out) {
    if (!A || !out) return F4_E_ARG;
    const Matrix& m = A->m;
    out->n = m.n;
    out->r = m.r;
    out->N = m.N;
    out->deg = m.deg;
    out->nnz = m.nnz;
    out->row_ptr = m.row_ptr.ptr;
    out->col_ind = m.col_ind.ptr;
    out->val = m.val.ptr;
    out->dict_keys = m.dict_keys.ptr;
    out->row_t = m.row_t.ptr;
    out->row_k = m.row_k.ptr;
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
    set_stream(X, stream);
    f4_reduced* R = new f4_reduced();
    R->owner = X;
    try {
        reduce_matrix(X->c, p, A->m, R->r);
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
    out->N = r.N;
    out->npivot = r.npivot;
    out->rho = r.rho;
    out->rank = r.rank;
    out->nnz = r.nnz;
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
    if (!gb || !F || F->on_device || F->n == 0 || F->n > 14 || !is_odd_prime(p) || p >= (1u << 31))
        throw F4Error{F4_E_ARG, "bad argument"};
    *gb = nullptr;
    set_stream(X, stream);
    Ctx& c = X->c;
    const u32 n = F->n;
    MonoOps mo;
    mo.init(n);
    const u32 w = mo.w;
    // ---- normalise inputs: reduce mod p, merge, sort by monomial, drop zeros, monic
    std::vector<std::vector<std::pair<u64, u32>>> inputs;
    bool unit = false;
    for (u32 k = 0; k < F->npolys; ++k) {
        std::vector<std::pair<u64, u32>> f;  // (order key, coeff)
        for (u64 e = F->offset[k]; e < F->offset[k + 1]; ++e) {
            const u64 P = F->mon[e];
            if ((P & ~(mo.lanes | (0xffull << 56))) != 0) throw F4Error{F4_E_ARG, "bad monomial word"};
            u32 d = 0;
            for (u32 i = 0; i < n; ++i) d += mono_exp(P, i, w);
            if (d != deg_of(P)) throw F4Error{F4_E_ARG, "monomial degree field mismatch"};
            f.push_back({mo.order_key(P), (u32)(F->coeff[e] % p)});
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
            if (t.second) h.push_back({t.first ^ mo.lanes, t.second});  // back to P words
        if (h.empty()) continue;
        const u64 inv = powmod_host(h[0].second, p - 2, p);
        for (auto& t : h) t.second = (u32)((u64)t.second * inv % p);
        if (deg_of(h[0].first) == 0) unit = true;
        inputs.push_back(std::move(h));
    }
    f4_basis* B = new f4_basis();
    B->owner = X;
    B->n = n;
    std::unique_ptr<f4_basis> Bguard(B);
    B->off.push_back(0);
    auto finish_unit = [&]() {
        B->mon = {0};
        B->coeff = {1};
        B->off = {0, 1};
    };
    if (unit) {
        finish_unit();
    } else if (!inputs.empty()) {
        DevG D;
        D.n = n;
        std::vector<u64> lm;
        std::vector<u8> active;
        std::vector<HPair> P;
        // ---- upload inputs, GM-insert each in order
        {
            std::vector<u64> mon, off{0};
            std::vector<u32> coeff;
            for (auto& f : inputs) {
                for (auto& t : f) {
                    mon.push_back(t.first);
                    coeff.push_back(t.second);
                }
                off.push_back(mon.size());
            }
            devg_reserve(c, D, mon.size(), (u32)inputs.size());
            upload(c, D.mon.ptr, mon.data(), mon.size() * 8);
            upload(c, D.coeff.ptr, coeff.data(), coeff.size() * 4);
            upload(c, D.off.ptr, off.data(), off.size() * 8);
            D.npolys = (u32)inputs.size();
            D.nterms = mon.size();
            hipLaunchKernelGGL(k_basis_meta, dim3(gridn(D.npolys, 256, 1024)), dim3(256), 0, c.stream, D.mon.ptr,
                               D.off.ptr, 0u, D.npolys, D.lm.ptr, D.len.ptr);
            F4_LAUNCH_CHECK();
            for (u32 k = 0; k < D.npolys; ++k) {
                lm.push_back(inputs[k][0].first);
                active.push_back(0);
                gm_update(mo, lm, active, P, k);
            }
        }
        const u32 guard = 1u << (w - 1);
        while (!unit && !P.empty()) {
            auto t0 = std::chrono::steady_clock::now();
            u32 d = 255;
            for (auto& q : P) d = std::min(d, deg_of(q.lcm));
            if (d >= guard) throw F4Error{F4_E_RANGE, "step degree reaches an exponent lane's guard bit"};
            std::vector<HPair> sel, rest;
            for (auto& q : P) (deg_of(q.lcm) == d ? sel : rest).push_back(q);
            P.swap(rest);
            std::vector<std::pair<u64, u32>> rows;
            for (auto& q : sel) {
                rows.push_back({q.lcm - lm[q.i], q.i});
                rows.push_back({q.lcm - lm[q.j], q.j});
            }
            std::vector<u32> act;
            for (u32 g = D.npolys; g-- > 0;)
                if (active[g]) act.push_back(g);
            Matrix A;
            build_step(c, D, rows, act, d, true, A);
            Reduced R;
            reduce_matrix(c, p, A, R);
            // ---- new elements: append the echelon rows to G on the device
            const u32 rho = R.rho;
            std::vector<u64> newlm(rho);
            if (rho) {
                devg_reserve(c, D, D.nterms + R.nnz, D.npolys + rho);
                hipLaunchKernelGGL(k_append, dim3(gridn(std::max<u64>(R.nnz, rho + 1), 256, 4096)), dim3(256), 0,
                                   c.stream, R.row_ptr.ptr, R.col_ind.ptr, R.val.ptr, rho, A.dict_keys.ptr, D.nterms,
                                   D.npolys, D.mon.ptr, D.coeff.ptr, D.off.ptr);
                F4_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_basis_meta, dim3(gridn(rho, 256, 1024)), dim3(256), 0, c.stream, D.mon.ptr,
                                   D.off.ptr, D.npolys, D.npolys + rho, D.lm.ptr, D.len.ptr);
                F4_LAUNCH_CHECK();
                readback(c, newlm.data(), D.lm.ptr + D.npolys, (u64)rho * 8);
                D.npolys += rho;
                D.nterms += R.nnz;
            }
            f4_step_stats st;
            memset(&st, 0, sizeof(st));
            st.deg = d;
            st.nsel = (u32)sel.size();
            st.r = A.r;
            st.N = A.N;
            st.nnz = A.nnz;
            st.npivot = R.npivot;
            st.lower = R.lower;
            st.rho = rho;
            st.rank = R.rank;
            st.closure_rounds = A.closure_rounds;
            st.dict_path = A.dict_path;
            st.t_dict_ms = A.t_dict;
            st.t_assemble_ms = A.t_assemble;
            st.t_numeric_ms = R.t_split + R.t_trsm + R.t_echelon + R.t_emit;
            st.t_trsm_ms = R.t_trsm;
            st.t_echelon_ms = R.t_echelon;
            for (u32 t = 0; t < rho && !unit; ++t) {
                const u32 h = (u32)lm.size();
                lm.push_back(newlm[t]);
                active.push_back(0);
                if (deg_of(newlm[t]) == 0) {
                    unit = true;
                    break;
                }
                gm_update(mo, lm, active, P, h);
            }
            st.t_step_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
            B->steps.push_back(st);
            c.ev_used = 0;
        }
        if (unit) {
            finish_unit();
        } else {
            // ---- reduced basis: minimal leading monomials, tails reduced by the others
            std::vector<u32> minimal;
            for (u32 g = 0; g < lm.size(); ++g) {
                if (!active[g]) continue;
                bool mn = true;
                for (u32 h = 0; h < lm.size() && mn; ++h)
                    if (h != g && active[h] && mo.divides(lm[h], lm[g])) mn = false;
                if (mn) minimal.push_back(g);
            }
            std::vector<std::pair<u64, u32>> rows;
            u32 dmax = 0;
            for (u32 g : minimal) {
                rows.push_back({0ull, g});
                dmax = std::max(dmax, deg_of(lm[g]));
            }
            std::vector<u32> act;
            for (u32 g = D.npolys; g-- > 0;)
                if (active[g]) act.push_back(g);
            Matrix A;
            build_step(c, D, rows, act, dmax, true, A);
            DBuf<u32> tptr, tcol, tval;
            tail_reduce_matrix(c, p, A, tptr, tcol, tval);
            std::vector<u64> rt(A.r), dict(A.N);
            std::vector<u32> rk(A.r), hp((u64)A.r + 1);
            readback(c, rt.data(), A.row_t.ptr, (u64)A.r * 8);
            readback(c, rk.data(), A.row_k.ptr, (u64)A.r * 4);
            readback(c, dict.data(), A.dict_keys.ptr, (u64)A.N * 8);
            readback(c, hp.data(), tptr.ptr, ((u64)A.r + 1) * 4);
            std::vector<u32> hc(hp[A.r]), hv(hp[A.r]);
            readback(c, hc.data(), tcol.ptr, (u64)hp[A.r] * 4);
            readback(c, hv.data(), tval.ptr, (u64)hp[A.r] * 4);
            std::set<u32> mset(minimal.begin(), minimal.end());
            // rows of A are sorted by leading monomial, largest first
            for (u32 i = 0; i < A.r; ++i) {
                if (rt[i] != 0 || !mset.count(rk[i])) continue;
                B->mon.push_back(lm[rk[i]]);
                B->coeff.push_back(1);
                for (u32 e = hp[i]; e < hp[i + 1]; ++e) {
                    B->mon.push_back(dict[hc[e]]);
                    B->coeff.push_back(hv[e]);
                }
                B->off.push_back(B->mon.size());
                mset.erase(rk[i]);
            }
            if (!mset.empty()) throw F4Error{F4_E_STATE, "inter-reduction lost a basis element"};
        }
    }
    X->bases.insert(B);
    *gb = Bguard.release();
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

}  // extern "C"
