// Internal host-side interfaces shared by the library's translation units.
#pragma once

#include <functional>
#include <map>
#include <unordered_map>
#include <vector>

#include "common.hpp"

// --------------------------------------------------------------- device cache
// A caching device allocator.  Blocks are reused in stream order: every launch
// of a context goes to one stream, so a block released after enqueueing the
// kernels that read it can be handed to kernels enqueued later on that stream.
struct Pool {
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> size_;
    size_t live_bytes = 0, cached_bytes = 0, peak_bytes = 0;
    // caller allocator (f4_opts.alloc / .free): used instead of hipMalloc /
    // hipFree when set; `stream` points at the context's current stream
    void* (*ualloc)(void* user, size_t bytes, void* stream) = nullptr;
    void (*ufree)(void* user, void* ptr, void* stream) = nullptr;
    void* uuser = nullptr;
    hipStream_t* stream = nullptr;

    static size_t round_size(size_t b) {
        if (b < 256) b = 256;
        size_t c = 256;
        while (c < b) c <<= 1;
        if (c > (64u << 20)) c = (b + (4u << 20) - 1) & ~size_t((4u << 20) - 1);  // 4 MiB steps above 64 MiB
        return c;
    }
    void* raw_alloc(size_t want) {
        if (ualloc) return ualloc(uuser, want, stream ? (void*)*stream : nullptr);
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void raw_free(void* p) {
        if (ufree)
            ufree(uuser, p, stream ? (void*)*stream : nullptr);
        else
            (void)hipFree(p);
    }
    void* alloc(size_t bytes) {
        size_t want = round_size(bytes);
        auto it = free_.lower_bound(want);
        if (it != free_.end() && it->first <= 2 * want) {
            void* p = it->second;
            cached_bytes -= it->first;
            live_bytes += it->first;
            free_.erase(it);
            return p;
        }
        void* p = raw_alloc(want);
        if (!p) {
            trim();
            p = raw_alloc(want);
            if (!p) throw F4Error{3, "device allocation of " + std::to_string(want) + " bytes failed"};
        }
        size_[p] = want;
        live_bytes += want;
        if (live_bytes > peak_bytes) peak_bytes = live_bytes;
        return p;
    }
    void release(void* p) {
        if (!p) return;
        auto it = size_.find(p);
        if (it == size_.end()) return;
        live_bytes -= it->second;
        cached_bytes += it->second;
        free_.insert({it->second, p});
    }
    // hand the cached blocks back (work enqueued earlier may still read them:
    // wait for the stream first)
    void trim() {
        if (free_.empty()) return;
        if (stream && *stream) (void)hipStreamSynchronize(*stream);
        for (auto& kv : free_) {
            raw_free(kv.second);
            size_.erase(kv.second);
        }
        free_.clear();
        cached_bytes = 0;
    }
    ~Pool() {
        for (auto& kv : size_) raw_free(kv.first);
    }
};

// A typed device buffer owned by a pool (released on destruction).
template <class T>
struct DBuf {
    Pool* pool = nullptr;
    T* ptr = nullptr;
    size_t n = 0;
    DBuf() {}
    DBuf(Pool* p, size_t count) { reset(p, count); }
    void reset(Pool* p, size_t count) {
        free();
        pool = p;
        n = count;
        ptr = (T*)pool->alloc((count ? count : 1) * sizeof(T));
    }
    void free() {
        if (pool && ptr) pool->release(ptr);
        ptr = nullptr;
        n = 0;
    }
    T* release_owner() {  // hand ownership to someone else
        T* p = ptr;
        ptr = nullptr;
        n = 0;
        return p;
    }
    ~DBuf() { free(); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : pool(o.pool), ptr(o.ptr), n(o.n) {
        o.ptr = nullptr;
        o.n = 0;
    }
    DBuf& operator=(DBuf&& o) noexcept {
        free();
        pool = o.pool;
        ptr = o.ptr;
        n = o.n;
        o.ptr = nullptr;
        o.n = 0;
        return *this;
    }
};

// -------------------------------------------------------------- primitives
// (prim.hip)
void fill_u32(u32* p, u64 n, u32 v, hipStream_t s);
void fill_u64(u64* p, u64 n, u64 v, hipStream_t s);
// Exclusive scan of n u32 values into out (may alias in); out[n] = total.
// out must have room for n + 1 values.
void exclusive_scan_u32(const u32* in, u32* out, u64 n, Pool& pool, hipStream_t s);
// The same with a caller workspace of exclusive_scan_ws_words(n) words (none
// for short inputs).
u64 exclusive_scan_ws_words(u64 n);
void exclusive_scan_u32_ws(const u32* in, u32* out, u64 n, u32* ws, hipStream_t s);
// Schedule of an LSD radix sort: bits per digit pass (1..8) and keys per
// thread in a tile of the multi-workgroup passes (sorts of at most
// SORT_SMALL_MAX keys run in one workgroup and use the digit width only).
struct SortPlan {
    u32 digit = 8, items = 16;
};
#define SORT_SMALL_MAX 5120
// Stable LSD radix sort of (key, val) pairs on key bits [lo_bit, hi_bit).
// keys/vals hold the input and receive the output; tmp buffers come from pool.
void radix_sort_pairs(u64* keys, u32* vals, u64 n, u32 lo_bit, u32 hi_bit, Pool& pool, hipStream_t s,
                      SortPlan plan = SortPlan());
// Sort keys only (vals unused)
void radix_sort_keys(u64* keys, u64 n, u32 lo_bit, u32 hi_bit, Pool& pool, hipStream_t s,
                     SortPlan plan = SortPlan());
// Unique of sorted keys: writes distinct keys to out, count to *d_count (device).
void unique_sorted_u64(const u64* keys, u64 n, u64* out, u32* d_count, Pool& pool, hipStream_t s);

// ----------------------------------------------------------------- context
struct StepTimer;
struct WorkPool;  // host threads for per-system work of a batch (workpool.hpp)

struct DevInfo {
    int device = 0;
    size_t max_lds = 65536;  // dynamic LDS bytes per workgroup usable by a kernel
    int cus = 256;
};

// Per-context state.  All device work of a call goes to `stream`.
struct Ctx {
    DevInfo dev;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;  // stream of the current call
    Pool pool;
    u32 flags = 0;
    u32 stop_deg = 0;  // stop a system after its first step of this degree (0: never)
    std::string last_error;
    // pinned host arena for small uploads / readbacks: uploads take successive
    // regions (no wait while the arena has room); a readback drains the
    // stream, after which the whole arena is free again
    u8* pinned = nullptr;
    size_t pinned_bytes = 0, pinned_used = 0;
    hipEvent_t staging_done = nullptr;  // last async copy out of the arena
    bool staging_pending = false;
    // caches keyed by (n, D): binomial table and dense-rank -> monomial table
    std::map<std::pair<u32, u32>, DBuf<u32>> binom;
    std::map<std::pair<u32, u32>, DBuf<u64>> montab;
    // timing events (F4_OPT_TIMING)
    std::vector<hipEvent_t> events;
    u32 ev_used = 0;
    // autotuner (F4_OPT_AUTOTUNE): the measured choice per (operation, shape
    // bucket); a forced value (nonzero) overrides both the table and the rule
    struct Tuner {
        bool on = false;
        u32 force_rr = 0, force_digit = 0;
        std::map<u64, u32> table;
    } tune;
    WorkPool* cpu = nullptr;  // created on first use, joined by f4_destroy
};

// ------------------------------------------------------------- autotuner
// (tune.hip)  Operations with a tuned schedule; every candidate computes the
// same result, so a choice changes time only.
enum TuneOp : u32 { TUNE_TRSM = 1, TUNE_SORT = 2 };
// Table key of an operation and its shape bucket (three 16-bit fields).
u64 tune_key(TuneOp op, u32 a, u32 b, u32 c);
// ceil(log2(x)) (0 for x <= 1): shape buckets are powers of two.
u32 tune_lg(u64 x);
// The tuned choice for `key`: the table entry when it is one of `cands`, else
// every candidate is run (`prep` then `run`, `prep` outside the timed region)
// twice on the live data, the fastest (by HIP events, best of two) is stored
// and returned.  Waits for the context stream while measuring.
u32 tune_pick(Ctx& c, u64 key, const std::vector<u32>& cands, const std::function<void(u32)>& prep,
              const std::function<void(u32)>& run);
// Radix sort with the context's schedule: a forced digit width, else the
// tuned plan (autotuner on and more than 8 key bits), else the default plan.
void tuned_sort(Ctx& c, u64* keys, u32* vals, u64 n, u32 lo_bit, u32 hi_bit);
// Text form of the tuning table (one line per entry) and its parser, which
// merges well-formed entries into the table and throws on anything else.
std::string tune_text(const Ctx& c);
void tune_parse(Ctx& c, const char* text);

// Block operator application (krylov.hip): Y = A X over F_p for a CSR matrix
// (nrows rows) and a row-major block X of b <= 64 columns; words of the
// matrix values and of X are read modulo p.  Enqueued on c.stream.
// optional epilogues of the block product (Krylov branch): a projection
// PX^T Y added into S64; AY AF added to the output; or the output's
// nonzero-column flags into NZ with the columns of KP flagged in KNZ copied
// into K
struct SpmmEpi {
    const u32* PX = nullptr;
    unsigned long long* S64 = nullptr;
    const u32* AY = nullptr;
    const u32* AF = nullptr;
    u32 ayb = 0;
    u32* NZ = nullptr;
    const u32* KP = nullptr;
    const u32* KNZ = nullptr;
    u32* K = nullptr;
};
void spmm_run(hipStream_t s, u32 p, u32 nrows, u32 b, const u32* ptr, const u32* idx, const u32* val, const u32* X,
              u32* Y, const SpmmEpi& ep = SpmmEpi());
// CSR of the transpose (the CSC of A): column pointers, row indices, values.
void csr_transpose(Ctx& c, u32 nrows, u32 ncols, u64 nnz, const u32* ptr, const u32* idx, const u32* val,
                   DBuf<u32>& tptr, DBuf<u32>& tidx, DBuf<u32>& tval);
// The same into caller memory: tptr (ncols + 1), tidx and tval (nnz), and a
// workspace of csr_transpose_ws_words(ncols) words; allocates nothing.
u64 csr_transpose_ws_words(u32 ncols);
void csr_transpose_into(hipStream_t s, u32 nrows, u32 ncols, u64 nnz, const u32* ptr, const u32* idx,
                        const u32* val, u32* tptr, u32* tidx, u32* tval, u32* ws);
// Block Wiedemann (wiedemann.hip).  The matrix A (r x N) as CSR, its
// transpose's CSR, and the transpose's values times D (the diagonal of the
// operator B = A D A^T).
struct BwCsr {
    u32 r = 0, N = 0;
    u64 nnz = 0;
    const u32 *ptr = nullptr, *idx = nullptr, *val = nullptr;
    const u32 *tptr = nullptr, *tidx = nullptr, *tval = nullptr;
    const u32* tval_d = nullptr;
};
// tval_d = the transpose's values of row j times d[j]
void bw_scale_transpose(Ctx& c, u32 p, const BwCsr& A, const u32* d, u32* tval_d);
// S_t = X^T B^t (B Y), t < L: S (L x b x b, device)
void bw_sequence(Ctx& c, u32 p, const BwCsr& A, u32 b, const u32* X, const u32* Y, u32 L, u32* S);
// M-Basis of [S(x)^T ; -I_b] to order L: P (2b x 2b x (L + 2), device), shifts (2b, device)
void bw_mbasis(Ctx& c, u32 p, u32 b, u32 L, const u32* S, u32* P, u32* shifts);
// For w generator columns (F: (Dmax + 1) x b x w, coefficients of B^m Y):
// K = sum_m B^m Y F_m by Horner, then the iterates B^e K for e < E with their
// nonzero-column flags (nzhist, E x w); K ends as each column's last nonzero
// iterate; nzcheck (w) flags the columns with A^T K != 0.
void bw_kernel_vectors(Ctx& c, u32 p, const BwCsr& A, u32 b, const u32* Y, u32 w, u32 Dmax, const u32* F, u32 E,
                       u32* K, u32* nzhist, u32* nzcheck);

// Allocation-free block products (f4_spmm_noalloc): the device address of
// the file-scope scratch array is looked up once per device (call with that
// device current); spmm_noalloc_words gives the scratch a product needs (the
// transpose for trans = 1, nothing for trans = 0); spmm_noalloc_run enqueues
// the product on `s`, the transpose built in the device's scratch.
void noalloc_scratch_init(int device);
u64 spmm_noalloc_words(u32 ncols, u64 nnz, int trans);
void spmm_noalloc_run(hipStream_t s, int device, u32 p, u32 nrows, u32 ncols, u64 nnz, const u32* ptr,
                      const u32* idx, const u32* val, int trans, u32 b, const u32* X, u32* Y);

// Modular inner-loop microbenchmark (micro.hip): uploads the chains' start
// values, times one launch of `iters` updates per chain with HIP events and
// reads the final values back.  Arguments are checked by the caller.
struct ModloopResult {
    double updates_per_s = 0, kernel_ms = 0;
    u32 regs = 0, private_bytes = 0;
};
void modloop_run(Ctx& c, u32 p, u32 form, u32 nchains, u32 iters, const u32* x0, const u32* a0, const u32* b0, u32* out,
                 ModloopResult& res);

// Next free region (>= bytes) of the pinned arena; waits for the copies in
// flight only when the arena has to wrap around.
u8* staging(Ctx& c, size_t bytes);
// Enqueue an H2D copy of host data through the staging buffer (small arrays).
void upload(Ctx& c, void* dst, const void* src, size_t bytes);
// Synchronous readback of a small device array through the staging buffer.
void readback(Ctx& c, void* dst, const void* src, size_t bytes);
// Event for stage timing (nullptr when timing is off).
hipEvent_t stage_event(Ctx& c);
// Whether the context records timings (the timing option).
bool timing_on(const Ctx& c);
// Per-launch events and product counters of the elimination kernels (the
// kernel-timing option); nullptr / false when it is off.
hipEvent_t kernel_event(Ctx& c);
bool kernel_timing_on(const Ctx& c);
float event_ms(hipEvent_t a, hipEvent_t b);

// Binomial table C(x, y), x <= n+D+1, y <= min(n, 15), on the device.
const u32* rank_table(Ctx& c, u32 n, u32 D);
// P word of every dense rank q < N(n, D).
const u64* unrank_table(Ctx& c, u32 n, u32 D);
u64 binom_host(u32 x, u32 y);

// ------------------------------------------------------------- basis view
struct DevBasis {
    u32 n = 0, w = 0, npolys = 0;
    const u64* mon = nullptr;
    const u32* coeff = nullptr;
    const u64* off = nullptr;
    const u64* lm = nullptr;   // leading monomial per polynomial
    const u32* len = nullptr;  // term count per polynomial
};

// --------------------------------------------------------------- matrix
// A batch of independent Macaulay matrices in one set of buffers.  System i
// owns rows [row_base, row_base + r), entries [nnz_base, nnz_base + nnz) and
// dictionary entries [dict_base, dict_base + N); column indices are local to
// the system.  A single matrix is the batch of one.
struct SysPart {
    u32 n = 0, deg = 0, r = 0, N = 0;
    u32 npiv = 0xffffffffu;  // distinct leading columns of the rows (unknown: all ones)
    u64 nnz = 0;
    u32 row_base = 0;
    u64 nnz_base = 0;
    u32 dict_base = 0;
};

struct Matrix {
    u32 S = 0, R = 0;
    u32 key_words = 1;  // words per monomial in dict_keys / row_t (2: two-word keys)
    u32 built_p = 0;  // prime the values were checked against (0: a caller CSR, not checked)
    u64 nnz = 0;
    std::vector<SysPart> sys;
    DBuf<u32> row_ptr, col_ind, val, row_k, row_sys;  // row_ptr holds batch-global offsets
    DBuf<u64> dict_keys, row_t;
    u32 closure_rounds = 0, dict_path = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // stage boundaries (timing on)
    float t_dict = 0, t_assemble = 0;
    void read_times() {  // once the stream has passed ev[2]
        if (!ev[0]) return;
        (void)hipEventSynchronize(ev[2]);
        t_dict = event_ms(ev[0], ev[1]);
        t_assemble = event_ms(ev[1], ev[2]);
    }
};

struct BuildArgs {
    DevBasis G;
    const u64* rows_t_host = nullptr;  // r0 initial rows (distinct (t, k)), host
    const u32* rows_k_host = nullptr;
    // or on the device: one buffer for the whole batch (every system passes
    // the same base), system i's rows at the sum of the r0 of the systems
    // before it
    const u64* rows_t_dev = nullptr;
    const u32* rows_k_dev = nullptr;
    u32 r0 = 0;                        // rows (with r0_dev: the room for them)
    const u32* r0_dev = nullptr;       // device rows only: the actual count, on the device
    const u32* active_host = nullptr;  // active basis indices in descending order, host
    const u32* active_dev = nullptr;   // or on the device (this system's own list)
    const struct SigDev* sig_dev = nullptr;  // device descriptor: closure over admissible reducers only
    u32 nactive = 0;
    u32 D = 0;                         // largest degree of any row
    bool closure = true;
    int dict_path = -1;                // -1 auto, 0 dense rank, 1 radix sort
};
// SP for every system of the batch (one launch per kernel for the batch).
void build_batch(Ctx& c, const std::vector<BuildArgs>& args, Matrix& out);

// ------------------------------------------------------ pair set (device)
// The pair set of one system on the device (Gebauer-Moeller update, normal
// selection): pairs (i, j, lcm) in one of two buffers (the selection moves the
// pairs it leaves into the other), and the summary of the last update.
struct DevPairs {
    DBuf<u64> lcm[2];
    DBuf<u32> ij[2];  // i, j of each pair
    DBuf<u32> born;   // element of the current step that created the pair
    DBuf<u32> alist;  // active elements, descending index (written by each update)
    u32 cur = 0;
    u64 cap = 0, acap = 0;
    u32 count = 0;                               // pairs in the current buffer
    u32 kept = 0, dmin = 0, nsel = 0, nact = 0;  // pairs, least lcm degree, pairs of it, active elements
};

// Insertion of basis elements h0 .. h0+rho-1 (their leading monomials already
// in lm) into a system's pair set, with the removals they cause and the
// retirement of the active elements they divide (act: one flag per element).
struct GmInsert {
    DevPairs* P;
    const u64* lm;
    u32* act;
    u32 n, h0, rho;
    // the selection of this step (its 4 output words) and the halves it had
    // to find: checked on the device, reported by the readback (sel_out
    // nullptr: nothing to check)
    const u32* sel_out = nullptr;
    u32 sel_halves = 0;
};
// Every system's insertion in one launch sequence, then one readback of the
// summaries into the DevPairs (count, kept, dmin, nsel, nact).
void gm_insert_batch(Ctx& c, const std::vector<GmInsert>& v);

// Normal selection of a system whose least lcm degree is d: the pairs of
// degree d leave the set and their halves (lcm / LM(k), k), deduplicated, go
// to rows at row_base (at most 2 * nsel of them; the active list for the
// reducer search is DevPairs::alist).  Returns the output words, 4 per
// system, written on the device: rows (what the build reads as the system's
// row count), unused, unused, halves; they live in `keep`, which the caller
// holds until the build has run.
struct GmSelect {
    DevPairs* P;
    const u64* lm;
    u32 n, npolys, d;
    u32 row_base;
};
u32* gm_select_batch(Ctx& c, const std::vector<GmSelect>& v, u64* rows_t, u32* rows_k, DBuf<u64>& keep);

// ------------------------------------------------------- block schedule
// The block schedule of a matrix (column panels of width W, the rows grouped
// by the panel of their leading column, SELL-C-sigma windows and slices) and
// its padded slice storage, all on the device.
struct SchedBufs {
    bool has = false;
    u32 W = 0, C = 0, sigma = 0, r = 0, npanels = 0, nslices = 0;
    u64 padded = 0;
    DBuf<u32> perm, panel_ptr, slice_start, slice_panel, slice_width, sell_col, sell_val;
    DBuf<u64> slice_off;
};
void sched_build(Ctx& c, u32 r, u32 N, u64 nnz, const u32* ptr, const u32* col, const u32* val, u32 W, u32 C, u32 sigma,
                 SchedBufs& S);
// Y = A X (b <= 8) through the slices.
void spmm_sell_run(hipStream_t s, u32 p, const SchedBufs& S, u32 b, const u32* X, u32* Y);

// ------------------------------------------------- two-word monomial keys
// The matrix of an explicit row list with two-word monomials (records of
// f4_rowspec_mw), basis as host SoA arrays already checked; out: key_words 2.
void build_rows_mw(Ctx& c, u32 n, u32 npolys, const u64* mon_h, const u32* coeff_h, const u64* off_h,
                   const void* rows_h, u32 r, Matrix& out);

// ----------------------------------------------------------- signatures
// Signatures of a basis on the device (one block: the descriptor and its
// arrays); dev points at the descriptor.
struct SigBufs {
    DBuf<u8> blob;
    const struct SigDev* dev = nullptr;
    const u32* sidx = nullptr;  // signature index of each element (in blob)
    size_t lds_bytes = 0;       // the tables' size (copied to LDS by the filter when small)
    u32 nindex = 0;
};
// Checks and uploads signatures (element k: mon[k] e_index[k]; index i's
// syzygy monomials syz_mon[syz_off[i] .. syz_off[i+1])).
void sig_upload(Ctx& c, u32 n, u32 npolys, const u32* index, const u64* mon, u32 nindex, const u32* syz_off,
                const u64* syz_mon, SigBufs& out);
// Flags of r rows (t[q*ts], k[q*ks]) (flags may be nullptr), the admissible
// ones compacted in input order into t2 / k2 with their count on the device;
// info_out (read back): overflow, kept, syzygy, rewritten.
void sig_filter_dev(Ctx& c, const SigBufs& S, const u64* t, u32 ts, const u32* k, u32 ks, u32 r, u8* flags,
                    DBuf<u64>& t2, DBuf<u32>& k2, DBuf<u32>& count, u32 info_out[4]);
// Schedule of the nkept survivors: positions sorted by (row degree, length of
// g_k, signature index), ties in input order; max_deg / max_len bound the
// row degrees and lengths (the key is as wide as they need).
void sig_schedule_dev(Ctx& c, const SigBufs& S, const u64* t2, const u32* k2, const u32* count, u32 nkept,
                      u32 max_deg, u32 max_len, const u64* lm, const u32* len, DBuf<u32>& order);

// ----------------------------------------------------------- elimination
struct RedPart {
    u32 N = 0, npivot = 0, lower = 0, rho = 0, rank = 0;
    u64 nnz = 0;
    u32 row_base = 0;   // first echelon row of the system
    u64 nnz_base = 0;   // first echelon entry
    u32 piv_base = 0;   // first pivot column entry
};

struct Reduced {
    u32 S = 0;
    std::vector<RedPart> sys;
    // leading monomial of every echelon row (row order), when the matrix
    // carries its dictionary: read back with the echelon's sizes
    std::vector<u64> newlm;
    DBuf<u32> pivot_cols, row_ptr, col_ind, val;  // row_ptr holds batch-global offsets
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float t_split = 0, t_trsm = 0, t_echelon = 0, t_emit = 0;
    // per-kernel timing (timing option): event pairs around each launch of the
    // triangular-solve and echelon block-step kernels, and their product counts
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_trsm, ev_block;
    DBuf<u64> ops;  // [0] triangular solve, [1] block step
    float t_k_trsm = 0, t_k_block = 0;
    u64 trsm_ops = 0, block_ops = 0;
    void read_times() {
        if (!ev[0]) return;
        (void)hipEventSynchronize(ev[4]);
        t_split = event_ms(ev[0], ev[1]);
        t_trsm = event_ms(ev[1], ev[2]);
        t_echelon = event_ms(ev[2], ev[3]);
        t_emit = event_ms(ev[3], ev[4]);
        t_k_trsm = t_k_block = 0;
        for (auto& e : ev_trsm) t_k_trsm += event_ms(e.first, e.second);
        for (auto& e : ev_block) t_k_block += event_ms(e.first, e.second);
        u64 h[2] = {0, 0};
        if (ops.ptr) (void)hipMemcpy(h, ops.ptr, sizeof(h), hipMemcpyDeviceToHost);
        trsm_ops = h[0];
        block_ops = h[1];
    }
};
// Elimination of every system of a batched matrix (p[i] for system i).
void reduce_batch(Ctx& c, const std::vector<u32>& p, const Matrix& A, Reduced& out);
// Inter-reduction: in every system all rows are pivot rows (distinct leading
// columns); returns each row's tail reduced by the other rows, as CSR over the
// system's columns (leading entry excluded), row order of A.
void tail_reduce_batch(Ctx& c, const std::vector<u32>& p, const Matrix& A, DBuf<u32>& tptr, DBuf<u32>& tcol,
                       DBuf<u32>& tval);
