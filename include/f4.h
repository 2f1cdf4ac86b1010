/*
 * f4.h - C-ABI of the MI355X (gfx950) F4 reduction-step library.
 *
 * One F4 step over F_p, as the paper states the problem:
 *   symbolic preprocessing SP : B -> (T, R, Pi)   (Definition "Symbolic
 *     preprocessing operator"; Algorithm "FBSP", two-pass count -> scan -> fill
 *     -> sort/unique -> join), producing the Macaulay matrix of Definition
 *     "Sparse Macaulay matrix for a batch" in CSR form with columns in
 *     descending grevlex order;
 *   elimination mod p of that matrix (section "PSGE: panel-structured Gaussian
 *     elimination"; two panels: pivot / non-pivot columns), with the modular
 *     multiply-add of equation "mod-fma" and Barrett reduction (section
 *     "Barrett reduction as reciprocal multiplication");
 *   and the F4 loop around it (section "F4 as batched module reduction").
 *
 * Conventions (fixed where the paper is silent):
 *   - Term order: grevlex with x_1 > x_2 > ... > x_n.
 *   - Monomials are packed exponent words ("P words"), see f4_pack(): the
 *     total degree in bits 56..63 and exponent a_i in a lane of w(n) bits at
 *     bit offset w(n)*(i-1), w(n) = min(8, floor(56/n)).  Monomial product is
 *     the integer sum of P words while no lane overflows.
 *   - Column 0 of a matrix is the largest monomial; dictionary keys are P words.
 *   - Reducer choice: among active basis elements whose leading monomial
 *     divides m, the one with the largest index.
 *   - Row order: leading monomial descending, then basis index ascending;
 *     duplicate (t, k) rows collapse to one.
 *   - Pivot row of a pivot column: fewest nonzeros, then lowest row index.
 *   - Echelon form: the reduced row echelon form (monic) of the trailing block.
 *
 * All functions return an int status (F4_OK on success).  No C++ exception
 * crosses this boundary.  Device work is asynchronous on the given stream
 * (a hipStream_t passed as void*; NULL = the context's own stream); outputs are
 * valid after that stream is synchronized.  The library never frees caller
 * memory.  A context is used by one host thread at a time; its cached device
 * memory is reused in stream order, so when a caller switches streams between
 * calls the context first synchronizes the stream it used before.
 */
#ifndef F4_H
#define F4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    F4_OK = 0,
    F4_E_ARG = 1,     /* bad argument: n = 0 or n > 14, p not an odd prime < 2^31,
                         unsorted / repeated terms, coefficient >= p, NULL pointer */
    F4_E_RANGE = 2,   /* an exponent lane or the degree field would overflow, or a
                         size exceeds 32-bit offsets */
    F4_E_NOMEM = 3,   /* device or host allocation failed; the context stays usable */
    F4_E_BUSY = 4,    /* request not admissible now (serving); retry later */
    F4_E_DEVICE = 5,  /* HIP runtime error; destroy the context */
    F4_E_STATE = 6    /* call not valid in the current state (e.g. unknown handle) */
};

typedef struct f4_ctx f4_ctx;
typedef struct f4_matrix f4_matrix;
typedef struct f4_reduced f4_reduced;
typedef struct f4_basis f4_basis;

/* Options for f4_create.  flags: bitwise OR of the F4_OPT_* values. */
enum {
    F4_OPT_TIMING = 1u << 0,     /* record per-stage HIP-event timings in f4_step_stats */
    F4_OPT_DICT_RANK = 1u << 1,  /* force the dense-rank dictionary (bitmap sort/unique) */
    F4_OPT_DICT_RADIX = 1u << 2, /* force the radix-sort dictionary (sort + unique + join) */
    F4_OPT_AUTOTUNE = 1u << 3,   /* pick schedules by measurement (see f4_tune_export) */
    F4_OPT_KERNEL_TIMING = 1u << 4, /* also HIP events around every launch of the triangular-solve
                                      and echelon block-step kernels, and their product counts */
    F4_OPT_HOST_PAIRS = 1u << 5   /* keep pair sets and activity flags on the host (the
                                      Gebauer-Moeller update and the normal selection in host
                                      code) instead of on the device; same results */
};
typedef struct f4_opts {
    uint32_t flags;
    /* 0: run F4 to the end.  d > 0: f4_groebner / f4_groebner_batch stop each
     * system after its first step of degree d (the step statistics are kept;
     * the returned basis of such a system is empty) - for timing one step of
     * a system at its real shape. */
    uint32_t stop_deg;
    /* 0: tuned or default.  1..4: rows of D' per workgroup tile of the sparse
     * triangular solve (capped by what the LDS holds).  Schedules never change
     * results. */
    uint32_t trsm_rows;
    /* 0: tuned or default (8).  1..8: bits per digit pass of the radix sorts. */
    uint32_t radix_bits;
    /* Device memory of the context (all of it: the block cache, matrices,
     * bases, scratch).  NULL: hipMalloc / hipFree.  Otherwise alloc(user,
     * bytes, stream) returns `bytes` of device memory on the context's device,
     * 256-byte aligned, or NULL when it cannot (the call then fails with
     * F4_E_NOMEM and the context stays usable); `stream` is the stream the
     * context works on at that moment (the memory may be used on it at once).
     * free(user, ptr, stream) returns a block; the context calls it only after
     * the work that used the block has finished (it synchronizes its stream
     * first), at the latest in f4_destroy.  The context caches blocks, so the
     * callbacks see few, large requests.  Both or neither must be set. */
    void* (*alloc)(void* user, size_t bytes, void* stream);
    void (*free)(void* user, void* ptr, void* stream);
    void* alloc_user;
} f4_opts;

/* Create a context on HIP device `device` (opts may be NULL).  The context owns
 * a device memory cache, a stream, events and host staging buffers. */
int f4_create(f4_ctx** out, int device, const f4_opts* opts);
int f4_destroy(f4_ctx* ctx);
/* Text of the last error on this context (static storage owned by the context). */
const char* f4_last_error(const f4_ctx* ctx);
/* Autotuner (F4_OPT_AUTOTUNE).  The paper leaves the schedule of its bulk
 * primitives open (section "Batching, scheduling, and GPU/accelerator
 * considerations": tile sizes and radix passes are tuning choices); with the
 * option set, the first call that meets an (operation, shape bucket) times
 * every candidate schedule on its live data with HIP events (best of two runs)
 * and keeps the fastest in the context's table; later calls reuse it.  Tuned
 * operations: the sparse triangular solve (rows per tile, 1..4) and the radix
 * sorts of more than 8 key bits (digit width 5..8, keys per thread 8 or 16).
 * All candidates compute identical outputs.
 *
 * f4_tune_export writes the table as text, one entry per line:
 *   "trsm <small p> <lg2 rows> <lg2 N> <rows per tile>"
 *   "sort <with values> <lg2 n> <key bits> <digit bits> <keys per thread>"
 * *len receives the text length (without the terminating NUL).  buf == NULL
 * is a size query; otherwise the text and a NUL are copied when cap > *len,
 * and F4_E_RANGE is returned (nothing copied) when the buffer is too small.
 * f4_tune_import merges such text into the table (entries are used by later
 * calls when they are valid for the shape at hand, otherwise re-tuned); a
 * malformed line gives F4_E_ARG and leaves the table unchanged. */
int f4_tune_export(f4_ctx* ctx, char* buf, size_t cap, size_t* len);
int f4_tune_import(f4_ctx* ctx, const char* text);
/* Copy `bytes` from device memory (e.g. a view pointer) to host memory `dst`
 * on the context's current stream and wait for it. */
int f4_download(f4_ctx* ctx, void* dst, const void* src, size_t bytes);

/* ------------------------------------------------------------- monomials */
/* Lane width w(n) in bits for n variables (0 if n is 0 or > 14). */
uint32_t f4_lane_bits(uint32_t n);
/* Pack n exponents into a P word (section "Monomial keys: order-refining
 * encodings"; key (deg, tie) in one machine word).  F4_E_RANGE if an exponent
 * exceeds 2^w(n)-1 or the degree exceeds 255; F4_E_ARG for a bad n. */
int f4_pack(uint32_t n, const uint32_t* exps, uint64_t* out);
/* Unpack a P word into n exponents. */
int f4_unpack(uint32_t n, uint64_t word, uint32_t* exps);
/* Two-word monomial keys for 1 <= n <= 30 variables (section "Monomial keys:
 * order-refining encodings that make sorting feasible", multiword keys): a
 * monomial is two words read as one 128-bit number, word 0 the high half.
 * Bits 120..127 hold the degree; below it come the exponents of x_n, x_{n-1},
 * ..., x_1 in lanes of w = f4_mw_lane_bits(n) bits, floor(56/w) lanes in
 * word 0 (from bit 56 down) and the rest in word 1 (from bit 64 down), no
 * lane split between the words, unused bits zero.  Complementing the lanes
 * (not the degree) gives the order key: comparing keys as 128-bit numbers is
 * grevlex (x_1 > ... > x_n), the key refines the order (no two monomials
 * share one), and a product is the word-wise sum while no lane overflows. */
/* w(n): 8 for n <= 15, 7 for n <= 17, 6 for n <= 19, 5 for n <= 23, 4 for
 * n <= 30, 0 otherwise. */
uint32_t f4_mw_lane_bits(uint32_t n);
/* Pack n exponents into two words (out[0] high).  F4_E_RANGE if an exponent
 * exceeds 2^w-1 or the degree 255; F4_E_ARG for a bad n. */
int f4_pack_mw(uint32_t n, const uint32_t* exps, uint64_t* out);
/* Unpack two words (in[0] high) into n exponents. */
int f4_unpack_mw(uint32_t n, const uint64_t* in, uint32_t* exps);
/* Dense grevlex rank of a monomial of degree <= D among the N(n, D) =
 * C(n+D, n) monomials of degree <= D (equation "monomial-count"): rank 0 is the
 * largest monomial x_1^D, and ranks increase as monomials decrease, so sorting
 * by rank is sorting by descending grevlex.  Host-side, for checking. */
int f4_grevlex_rank(uint32_t n, uint32_t D, uint64_t word, uint32_t* rank);
/* Inverse of f4_grevlex_rank. */
int f4_grevlex_unrank(uint32_t n, uint32_t D, uint32_t rank, uint64_t* word);

/* ------------------------------------------------------------ polynomials */
/* A list of polynomials in structure-of-arrays form (section "Coalesced sparse
 * polynomial storage: SoA support vectors"): the terms of polynomial k are
 * mon[offset[k] .. offset[k+1]) and coeff[...].  Terms are sorted by monomial,
 * largest first, with no repeated monomial and coefficients in [1, p).
 * on_device = 1: mon/coeff/offset are device pointers; 0: host pointers. */
typedef struct f4_polys {
    uint32_t n;
    uint32_t npolys;
    const uint64_t* mon;
    const uint32_t* coeff;
    const uint64_t* offset; /* npolys + 1 entries */
    int on_device;
} f4_polys;

/* Checks host polynomials against the form above (the input contract of
 * f4_build_matrix and f4_build_matrix_rows): P words of n variables, terms in
 * strictly decreasing grevlex order (unsorted or repeated terms fail),
 * coefficients in [1, p), no zero polynomial, and with monic != 0 leading
 * coefficients 1.  Host-side, no context needed.  Returns F4_OK or F4_E_ARG;
 * *bits (may be NULL) receives the failed rules: 1 a word that is not a
 * monomial of n variables, 2 order, 4 coefficient range, 8 not monic, 16 a
 * zero polynomial. */
int f4_check_polys(uint32_t p, const f4_polys* G, int monic, uint32_t* bits);
/* Brings host polynomials into the form above: each polynomial's terms are
 * sorted by decreasing grevlex, repeated monomials merged (coefficients added
 * mod p), coefficients reduced mod p and zero terms dropped; monic != 0 also
 * divides each polynomial by its leading coefficient.  mon_out / coeff_out
 * have room for in->offset[in->npolys] terms, off_out for npolys + 1 offsets
 * (a polynomial that cancels to zero keeps an empty range).  Host-side, no
 * context.  F4_E_ARG: bad p or n, a word that is not a monomial of n
 * variables, decreasing offsets, null arrays. */
int f4_normalize_polys(uint32_t p, const f4_polys* in, int monic, uint64_t* mon_out, uint32_t* coeff_out,
                       uint64_t* off_out);

/* A critical pair of basis indices (i < j). */
typedef struct f4_pair {
    uint32_t i, j;
} f4_pair;

/* A shifted reducer t * g_k: t a P word, k a basis index. */
typedef struct f4_rowspec {
    uint64_t t;
    uint32_t k;
    uint32_t pad;
} f4_rowspec;

/* ------------------------------------------------------- matrix (SP output) */
typedef struct f4_matrix_view {
    uint32_t n;        /* variables */
    uint32_t r;        /* rows */
    uint32_t N;        /* columns = dictionary size |T| */
    uint32_t deg;      /* largest degree in the dictionary */
    uint64_t nnz;      /* = M, the total row length */
    const uint32_t* row_ptr;   /* device, r + 1: exclusive scan of row lengths */
    const uint32_t* col_ind;   /* device, nnz: column of each entry, ascending per row */
    const uint32_t* val;       /* device, nnz: coefficient in [1, p) */
    const uint64_t* dict_keys; /* device, N * key_words: monomial of each column, descending grevlex */
    const uint64_t* row_t;     /* device, r * key_words: shift monomial t_i */
    const uint32_t* row_k;     /* device, r: basis index k_i */
    uint32_t key_words;        /* words per monomial: 1 (P words) or 2 (f4_build_matrix_rows_mw) */
    uint32_t pad;
} f4_matrix_view;

/* Symbolic preprocessing of one F4 step (Definition "Symbolic preprocessing
 * operator"; Algorithm "FBSP"): the rows are the two halves
 * (lcm/LM(g_i), i), (lcm/LM(g_j), j) of every selected pair, closed under
 * one-step reduction (Remark "Truncation and why symbolic preprocessing
 * matters", Definition "Support-closure for correctness") by the reducer rule
 * above; the dictionary is the sorted, deduplicated union of the row supports
 * and the CSR is written by a two-pass count -> prefix-sum -> fill plan.
 *   p       : odd prime < 2^31.
 *   G       : basis (host or device SoA); all elements monic.
 *   active  : host array of G->npolys bytes, nonzero = usable as a reducer.
 *   sel     : host array of nsel pairs, all with the same lcm degree.
 *   A       : out, a context-owned matrix handle (free with f4_matrix_free).
 * Errors: F4_E_ARG (bad p, n, indices, empty selection; a basis that breaks
 * the f4_polys form - see f4_check_polys - or is not monic: host input is
 * checked on the host, device input by a kernel before any use), F4_E_RANGE
 * (lane overflow), F4_E_NOMEM, F4_E_DEVICE. */
int f4_build_matrix(f4_ctx* ctx, uint32_t p, const f4_polys* G, const uint8_t* active,
                    const f4_pair* sel, uint32_t nsel, f4_matrix** A, void* stream);

/* The same map for an explicit row list R (host, r entries) with no closure:
 * the matrix of Definition "Sparse Macaulay matrix for a batch" for
 * (T = union of supports, R).  Theorem "Matrix materialization correctness"
 * is stated for exactly this object.  G must have the f4_polys form (checked
 * as for f4_build_matrix; it need not be monic); F4_E_ARG otherwise. */
int f4_build_matrix_rows(f4_ctx* ctx, uint32_t p, const f4_polys* G, const f4_rowspec* R, uint32_t r,
                         f4_matrix** A, void* stream);

/* ------------------------------------------------------------ signatures */
/* Signatures of a basis (section "Signature regime: correctness under
 * admissibility predicates"; section "Discussion: Integrating Signatures,
 * Admissibility, and GPU Scheduling"; the paper leaves the order and the
 * rewrite rule open, the readings taken are these): element k carries the
 * signature mon[k] e_{index[k]}, and the shifted reducer t * g_k the signature
 * (t mon[k]) e_{index[k]}, ordered position over term.  For each index i,
 * syz_mon[syz_off[i] .. syz_off[i+1]) are monomials u with u e_i the
 * signature of a known syzygy (for instance LM(f_j), j < i, for the principal
 * syzygies).  A row is admissible unless
 *   - a syzygy monomial of its index divides its signature monomial
 *     (F4_ADM_SYZYGY, tested first), or
 *   - a newer element k' > k with index[k'] = index[k] has mon[k'] dividing
 *     it (F4_ADM_REWRITTEN: the newest element whose signature divides a
 *     signature is the one allowed to produce it).
 * All arrays are host arrays, P words of the basis's n variables. */
typedef struct f4_sigs {
    uint32_t npolys;          /* the basis size */
    const uint32_t* index;    /* npolys, each < nindex */
    const uint64_t* mon;      /* npolys */
    uint32_t nindex;          /* 1 .. 2^20 */
    const uint32_t* syz_off;  /* nindex + 1, nondecreasing, syz_off[0] = 0 */
    const uint64_t* syz_mon;  /* syz_off[nindex] */
} f4_sigs;

enum { F4_ADM_OK = 0, F4_ADM_SYZYGY = 1, F4_ADM_REWRITTEN = 2 };

typedef struct f4_sig_stats {
    uint32_t kept, syzygy, rewritten; /* rows admissible / rejected by each test */
    uint32_t pad;
    double t_device_ms;  /* HIP events around the device work of the call (predicate, scan,
                            compaction, schedule; for f4_build_matrix_sig also the build) */
} f4_sig_stats;

/* The admissibility predicate over a row list, in bulk: the flag of every row
 * (F4_ADM_*), the admissible rows compacted in input order, and a schedule
 * of them bucketed by (degree of t * LM(g_k), number of terms of g_k,
 * signature index), ties in input order.
 *   p, G   : as for f4_build_matrix_rows (G host or device, f4_polys form).
 *   S      : signatures of G (S->npolys = G->npolys).
 *   R, r   : host rows, r >= 1.
 *   flags  : host, r bytes out (may be NULL).
 *   kept   : host, room for r rows out (may be NULL); *nkept = their count.
 *   order  : host, room for r entries out (may be NULL): positions in kept,
 *            scheduled (r < 2^28; the key saturates lengths at 2^16 - 1 and
 *            indices at 2^12 - 1, ties then fall back to input order).
 *   st     : out (may be NULL).
 * Errors: F4_E_ARG (bad p, G, S, a row's k out of range or t not a
 * monomial), F4_E_RANGE (t * LM(g_k) or a signature t mon[k] overflows an
 * exponent lane), F4_E_NOMEM, F4_E_DEVICE. */
int f4_sig_filter(f4_ctx* ctx, uint32_t p, const f4_polys* G, const f4_sigs* S, const f4_rowspec* R,
                  uint32_t r, uint8_t* flags, f4_rowspec* kept, uint32_t* nkept, uint32_t* order,
                  f4_sig_stats* st, void* stream);

/* Symbolic preprocessing over the admissible reducers (Theorem
 * "Signature-sound compilation"; the fixed point "propose rows, filter by
 * signatures, close the dictionary for the filtered set, recheck coverage"):
 * the rows R are deduplicated and filtered, then closed as in
 * f4_build_matrix, except that a dictionary monomial m gets as reducer the
 * active element g of largest index with LM(g) | m whose row (m / LM(g), g)
 * is admissible, and no row when there is none.  Every row of the result is
 * admissible.  G monic (as for f4_build_matrix), active: host bytes,
 * S: signatures of G, R: host rows (r >= 1), A: out handle, st: out (may be
 * NULL).  Errors as for f4_build_matrix and f4_sig_filter; F4_E_ARG also when
 * no row of R is admissible. */
int f4_build_matrix_sig(f4_ctx* ctx, uint32_t p, const f4_polys* G, const uint8_t* active, const f4_sigs* S,
                        const f4_rowspec* R, uint32_t r, f4_matrix** A, f4_sig_stats* st, void* stream);

/* ------------------------------------------------ multiword monomial keys */
/* Host SoA polynomials with two-word monomials (f4_pack_mw): mon holds
 * 2 words per term (high word first), terms of each polynomial in strictly
 * decreasing grevlex, coefficients in [1, p), no zero polynomial. */
typedef struct f4_polys_mw {
    uint32_t n;               /* 1 .. 30 */
    uint32_t npolys;
    const uint64_t* mon;      /* 2 * offset[npolys] words */
    const uint32_t* coeff;
    const uint64_t* offset;   /* npolys + 1 entries */
} f4_polys_mw;

/* f4_normalize_polys for two-word monomials: terms sorted by decreasing
 * grevlex (order keys as 128-bit numbers), repeats merged, coefficients
 * reduced mod p, zero terms dropped.  mon_out has room for 2 words per input
 * term, coeff_out for one, off_out for npolys + 1 offsets.  Host-side.
 * F4_E_ARG: bad p or n, a word pair that is not a monomial, decreasing
 * offsets, null arrays. */
int f4_normalize_polys_mw(uint32_t p, const f4_polys_mw* in, uint64_t* mon_out, uint32_t* coeff_out,
                          uint64_t* off_out);

/* A shifted reducer t * g_k with a two-word shift (t[0] high). */
typedef struct f4_rowspec_mw {
    uint64_t t[2];
    uint32_t k;
    uint32_t pad;
} f4_rowspec_mw;

/* f4_build_matrix_rows for n up to 30 variables with two-word keys: the
 * matrix of the explicit row list R (Definition "Sparse Macaulay matrix for a
 * batch" for T = union of supports, R; no closure): every row's terms are
 * shifted (word-wise sums), their order keys sorted as 128-bit numbers by two
 * stable 64-bit radix sorts (low word, then high word), repeats dropped, and
 * each term joined to its key's rank; rows in the usual order (leading
 * monomial descending, then k; repeated (t, k) collapse).  The view has
 * key_words = 2 (dict_keys and row_t two words per entry).  The matrix works
 * with f4_reduce, f4_spmm and f4_block_wiedemann like any other.  G and R are
 * host arrays checked on the host (G) and the device (R: k in range, t a
 * monomial, t * LM(g_k) without lane overflow).  Errors: F4_E_ARG (bad p, G,
 * a row), F4_E_RANGE (lane overflow, 2^32 or more nonzeros), F4_E_NOMEM,
 * F4_E_DEVICE. */
int f4_build_matrix_rows_mw(f4_ctx* ctx, uint32_t p, const f4_polys_mw* G, const f4_rowspec_mw* R, uint32_t r,
                            f4_matrix** A, void* stream);

/* A matrix from caller CSR arrays (host): r rows, N columns, entries sorted by
 * column within each row, values in [1, p).  Used to run f4_reduce on given
 * matrices.  dict_keys/row_t/row_k of the view are NULL for such a matrix. */
int f4_matrix_from_csr(f4_ctx* ctx, uint32_t r, uint32_t N, const uint32_t* row_ptr, const uint32_t* col_ind,
                       const uint32_t* val, f4_matrix** A, void* stream);

int f4_matrix_get(const f4_matrix* A, f4_matrix_view* out);
int f4_matrix_free(f4_matrix* A);

/* Block operator application for Krylov solvers (section "Block Wiedemann
 * and Block Lanczos"): Y = A X (trans = 0) or Y = A^T X (trans = 1) over F_p,
 * A the r x N matrix of a handle of one system (f4_build_matrix,
 * f4_build_matrix_rows or f4_matrix_from_csr), X and Y device arrays owned by
 * the caller, row-major with b columns (1 <= b <= 64): X is N x b and Y is
 * r x b for A X; X is r x b and Y is N x b for A^T X.  Stored values and the
 * words of X are read modulo p; Y receives canonical residues.  The first
 * transposed call on a handle builds the transpose's CSR on the device (kept
 * with the handle, freed with it).  Asynchronous on `stream` (NULL: the
 * context's stream); Y must not overlap X.  X and Y need 4-byte alignment
 * only (8-byte aligned blocks with an even b take a faster layout).
 * F4_E_ARG: p not an odd prime
 * < 2^31, b out of range, trans not 0/1, a null block with a nonempty side,
 * or a handle of a batch; F4_E_STATE: a handle not of this context. */
int f4_spmm(f4_ctx* ctx, uint32_t p, f4_matrix* A, int trans, uint32_t b, const uint32_t* X, uint32_t* Y,
            void* stream);
/* f4_spmm repeated `reps` times on the context's stream between one pair of
 * HIP events; *ms_per_call receives the mean time of one call (a transposed
 * call on a handle without its transpose builds it first, outside the timed
 * pair).  Same arguments and errors as f4_spmm, plus F4_E_ARG for reps = 0
 * or a null ms_per_call. */
int f4_spmm_timed(f4_ctx* ctx, uint32_t p, f4_matrix* A, int trans, uint32_t b, const uint32_t* X, uint32_t* Y,
                  uint32_t reps, double* ms_per_call);
/* ------------------------------------------------------ block schedule */
/* The block schedule that enriches the plan Pi (section "PSGE:
 * panel-structured Gaussian elimination", "Why Pi must be enriched": panel
 * boundaries and the row-to-panel incidence; section "Row assembly as a
 * dictionary join; divergence control via SELL-C-sigma bucketing"), built on
 * the device and kept with the handle: panels are the column segments
 * [l W, (l+1) W), l < npanels = max(1, ceil(N / W)); a row belongs to the
 * panel of its leading column, empty rows to a last group npanels; perm lists
 * the rows panel by panel, each panel's rows (in row order) cut into windows
 * of sigma rows sorted longest first (ties by row index); slices are runs of
 * C rows inside one group, padded to their longest row; the slice storage is
 * column-major (entry k of the slice's row j at slice_off[s] + k C + j,
 * padding column 0 and value 0).  All arrays device, owned by the handle
 * (until the next f4_matrix_schedule or f4_matrix_free). */
typedef struct f4_schedule_view {
    uint32_t W, C, sigma;
    uint32_t npanels;
    uint32_t nslices;
    uint32_t pad;
    uint64_t padded;                /* slots of the slice storage */
    const uint32_t* perm;           /* r */
    const uint32_t* panel_ptr;      /* npanels + 2: positions in perm, the last group empty rows */
    const uint32_t* slice_start;    /* nslices: positions in perm */
    const uint32_t* slice_panel;    /* nslices */
    const uint32_t* slice_width;    /* nslices */
    const uint64_t* slice_off;      /* nslices + 1 */
    const uint32_t* sell_col;       /* padded */
    const uint32_t* sell_val;       /* padded */
} f4_schedule_view;
/* Build (or rebuild) the schedule of a handle of one system.  W >= 1,
 * 1 <= C <= 64, sigma >= 1; out may be NULL.  F4_E_ARG: bad parameters or a
 * batch handle; F4_E_STATE: unknown handle; F4_E_RANGE: key widths exceeded
 * (2^30 panels or more, or a sort key of the rows past 64 bits); F4_E_NOMEM. */
int f4_matrix_schedule(f4_ctx* ctx, f4_matrix* A, uint32_t W, uint32_t C, uint32_t sigma, f4_schedule_view* out,
                       void* stream);
/* Y = A X over F_p through the schedule's slices (one wave per slice, each
 * row of the slice on a few lanes that split the b vectors; b <= 8 device
 * vectors, row-major as for f4_spmm, any 4-byte alignment; the same result
 * as f4_spmm).  F4_E_STATE: no schedule built; F4_E_ARG: bad p, b, blocks. */
int f4_spmm_sell(f4_ctx* ctx, uint32_t p, const f4_matrix* A, uint32_t b, const uint32_t* X, uint32_t* Y,
                 void* stream);
/* f4_spmm_sell repeated `reps` times between one pair of HIP events (mean
 * time per call in *ms_per_call), as f4_spmm_timed. */
int f4_spmm_sell_timed(f4_ctx* ctx, uint32_t p, const f4_matrix* A, uint32_t b, const uint32_t* X, uint32_t* Y,
                       uint32_t reps, double* ms_per_call);

/* Block Wiedemann over F_p (section "Block Wiedemann and Block Lanczos":
 * kernel vectors by black-box linear algebra, the block form of Wiedemann's
 * method; Remark "Syzygies, revisited"): left-kernel vectors v != 0,
 * v^T A = 0, of the r x N matrix of a handle of one system - by Proposition
 * "Kernel equals syzygies under dictionary closure" the syzygies among the
 * shifted reducers - using only products with A and A^T on blocks of b
 * vectors.  The square operator is B = A D A^T (r x r) for a caller diagonal
 * d of N nonzero elements (device array); ker A^T is contained in ker B, and
 * every vector returned is checked against A^T v = 0.  X and Y are device
 * blocks (r x b, row-major) of random elements: projection and start.
 * 1 <= b <= F4_BW_MAX_B.  Words of d, X and Y are read modulo p. */
#define F4_BW_MAX_B 16
/* The projected block Krylov sequence S_t = X^T B^t (B Y), t = 0 .. L-1, into
 * S (device, L x b x b, S[t][k][l] at (t b + k) b + l, canonical residues). */
int f4_bw_sequence(f4_ctx* ctx, uint32_t p, f4_matrix* A, uint32_t b, const uint32_t* d, const uint32_t* X,
                   const uint32_t* Y, uint32_t L, uint32_t* S, void* stream);
/* The generator step: an M-Basis sigma-basis, to order L, of the matrix power
 * series [S(x)^T ; -I_b] (2b x b) with shifts (0^b, 1^b).  At each order the
 * residual coefficient of every row is eliminated in the order of (shift,
 * row index): a row whose residual is nonzero pivots on its first nonzero
 * column and clears it from the later rows fraction-free
 * (row_j <- piv row_j - r_j row_i); the pivot rows are then multiplied by x
 * and their shifts raised by one.  Output P (device, 2b x 2b x (L + 2):
 * coefficient l of entry (i, j) at (i 2b + j)(L + 2) + l) and shifts (device,
 * 2b).  A row (g, h) with shift s has deg g <= s, deg h < s, and
 * f_m = g_{s-m} is a right generator of the sequence for t <= L - 1 - s. */
int f4_bw_mbasis(f4_ctx* ctx, uint32_t p, uint32_t b, uint32_t L, const uint32_t* S, uint32_t* P,
                 uint32_t* shifts, void* stream);
typedef struct f4_bw_stats {
    uint32_t L;            /* sequence length 2 ceil(r / b) + 4 */
    uint32_t generators;   /* sigma-basis rows used as generators */
    double t_sequence_ms;  /* host wall time of each phase (device work waited for) */
    double t_mbasis_ms;
    double t_vectors_ms;
} f4_bw_stats;
/* The whole method on the context's stream: the sequence with
 * L = 2 ceil(r / b) + 4; the sigma-basis; as generators the rows with g != 0
 * and 2 s + 2 <= L, in the order of (shift, index); for each, with m0 its
 * lowest nonzero coefficient, u = sum_{m >= m0} B^(m - m0) Y f_m (Horner, all
 * generators at once) and the first iterate B^e u (e <= s + 1) that B sends
 * to zero; kept when A^T v = 0.  V (host, cap x r) receives the vectors found
 * (vector i at V + i r, canonical residues), *nvec their number (which may
 * exceed cap; only cap are written).  st may be NULL.  F4_E_ARG: bad p, b,
 * null arguments, a handle of a batch; F4_E_STATE: a handle not of this
 * context. */
int f4_block_wiedemann(f4_ctx* ctx, uint32_t p, f4_matrix* A, uint32_t b, const uint32_t* d, const uint32_t* X,
                       const uint32_t* Y, uint32_t* V, uint32_t cap, uint32_t* nvec, f4_bw_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): f4_spmm on
 * caller CSR arrays, allocating nothing.  A is r x N with row_ptr (r + 1
 * entries), col_ind and val (nnz entries, nnz = row_ptr[r] < 2^32), all
 * device arrays owned by the caller; X, Y, b, trans and the results are as
 * for f4_spmm (bit-identical to f4_spmm on a handle of the same CSR).
 * trans = 1 builds the transpose in a scratch array of
 * F4_NOALLOC_SCRATCH_BYTES that the library keeps on each GPU (set up by
 * f4_create, held until the process ends): it needs
 * 4 * (N + 1 rounded up to 64 + 2 nnz + workspace) bytes, about
 * 8 nnz + 8 N, and larger products fail with F4_E_RANGE before any work is
 * enqueued.  trans = 0 uses no scratch.  Every call on one GPU shares that
 * GPU's scratch and the last call's contents stay in it: calls that overlap
 * on one GPU (two streams, two contexts or two threads) race, so callers
 * order them (one stream, or events).  Asynchronous on `stream` (NULL: the
 * context's stream).  F4_E_ARG: as for f4_spmm, plus a null row_ptr, null
 * col_ind / val with nnz > 0, nnz >= 2^32. */
#define F4_NOALLOC_SCRATCH_BYTES (64u << 20)
int f4_spmm_noalloc(f4_ctx* ctx, uint32_t p, uint32_t r, uint32_t N, uint64_t nnz, const uint32_t* row_ptr,
                    const uint32_t* col_ind, const uint32_t* val, int trans, uint32_t b, const uint32_t* X,
                    uint32_t* Y, void* stream);
/* Device memory from the context's cache (freed with the context at the
 * latest), for blocks passed to f4_spmm; f4_upload copies host bytes to it
 * and waits (f4_download copies back). */
int f4_device_alloc(f4_ctx* ctx, size_t bytes, void** ptr);
int f4_device_free(f4_ctx* ctx, void* ptr);
int f4_upload(f4_ctx* ctx, void* dst, const void* src, size_t bytes);

/* ------------------------------------------------- reduce (elimination) */
typedef struct f4_reduced_view {
    uint32_t N;          /* columns of A */
    uint32_t npivot;     /* |Pc|: distinct leading columns of the rows of A */
    uint32_t rho;        /* rank of the reduced trailing block */
    uint32_t rank;       /* rank(A) = npivot + rho */
    uint64_t nnz;        /* entries of the echelon rows */
    const uint32_t* pivot_cols; /* device, npivot, ascending */
    const uint32_t* row_ptr;    /* device, rho + 1 */
    const uint32_t* col_ind;    /* device: columns of A, ascending per row */
    const uint32_t* val;        /* device: first entry of each row is 1 */
} f4_reduced_view;

/* Elimination of A mod p (section "PSGE"): pivot columns = leading columns of
 * the rows; one pivot row per pivot column; the other rows are reduced by the
 * pivot rows on the pivot columns (sparse triangular solve), and the reduced
 * row echelon form of the remaining trailing block is returned as CSR over the
 * columns of A, rows ordered by leading column.  A is not modified.
 * F4_E_ARG: bad p, or stored values outside [1, p) (checked on the device for
 * a matrix from f4_matrix_from_csr or built for another prime); F4_E_STATE: a
 * handle not of this context. */
int f4_reduce(f4_ctx* ctx, uint32_t p, const f4_matrix* A, f4_reduced** out, void* stream);
int f4_reduced_get(const f4_reduced* R, f4_reduced_view* out);
int f4_reduced_free(f4_reduced* R);

/* ----------------------------------------------------------- full F4 */
typedef struct f4_step_stats {
    uint32_t deg, nsel, r, N;
    uint64_t nnz;
    uint32_t npivot, lower, rho, rank;
    uint32_t closure_rounds, dict_path; /* dict_path: 0 dense rank, 1 radix sort */
    float t_dict_ms;      /* DictBuild: row emission, closure, sort + unique (HIP events) */
    float t_assemble_ms;  /* RowAssemble: count, scan, fill + join */
    float t_numeric_ms;   /* NumericCore: split, triangular solve, echelon, emit */
    float t_trsm_ms;      /* of which the sparse triangular solve */
    float t_echelon_ms;   /* of which the trailing-block echelon */
    float t_step_ms;      /* host wall time of the whole step */
    float t_pairs_ms;     /* pair selection and Gebauer-Moeller update of the step: device
                             pair sets - HIP events with F4_OPT_TIMING (for a batch, the
                             batch's launches), else host wall time of the calls including
                             the wait for the summary; host pair sets - host time */
    /* per kernel (F4_OPT_KERNEL_TIMING only; for a batch, the batch's launches):
     * the triangular-solve kernel and the echelon block-step kernel, summed
     * over their launches (HIP events around each launch on the call's
     * stream), their launch counts, and the modular products they performed
     * (triangular solve: panel products and trailing-entry updates; block
     * step: the transform products and the row-operation products). */
    float t_k_trsm_ms;
    uint32_t n_k_trsm;
    uint64_t trsm_ops;
    float t_k_block_ms;
    uint32_t n_k_block;
    uint64_t block_ops;
} f4_step_stats;

/* Reduced Groebner basis of <F> under grevlex (unique: monic, minimal,
 * inter-reduced), computed by F4 with the Gebauer-Moeller pair update and the
 * normal selection strategy (section "Pair management and the normal
 * strategy"; both on the device unless F4_OPT_HOST_PAIRS is set: the pair set
 * and the activity flags then never leave the device between steps, and the
 * halves of the selected pairs go to the symbolic preprocessing as device
 * arrays).  F: host SoA polynomials (any coefficients < p,
 * terms sorted as above; zero polynomials allowed).  gb: out handle. */
int f4_groebner(f4_ctx* ctx, uint32_t p, const f4_polys* F, f4_basis** gb, void* stream);
/* The same for nsys independent systems (prime p[i], input F[i]) processed
 * together: every F4 iteration advances all unfinished systems by one step
 * with one batched launch sequence (symbolic preprocessing and elimination of
 * all their matrices at once), and the finished ones are inter-reduced
 * together.  gb: array of nsys out handles.  Each result equals what
 * f4_groebner returns for that system alone. */
int f4_groebner_batch(f4_ctx* ctx, uint32_t nsys, const uint32_t* p, const f4_polys* F, f4_basis** gb,
                      void* stream);
/* Host view of a basis: polynomials sorted by leading monomial, largest first. */
int f4_basis_view(const f4_basis* B, f4_polys* out);
int f4_basis_stats(const f4_basis* B, const f4_step_stats** steps, uint32_t* nsteps);
int f4_basis_free(f4_basis* B);

/* ------------------------------------------------------------- serving */
typedef struct f4_server f4_server;

/* Estimated device footprint of one system with n variables and m quadratic
 * generators: 8 * N(n, D) * N(n, D - 1) bytes + 64 MiB, where D is the
 * degree of regularity of a semi-regular sequence of m quadratics (first
 * non-positive coefficient of (1 - t^2)^m / (1 - t)^n) and N(n, d) = C(n+d, d)
 * (equation "monomial-count"): the size of a dense trailing block of the
 * widest step.  Host-side only. */
int f4_server_footprint(uint32_t n, uint32_t m, uint64_t* bytes);

/* A serving engine on a context.  Systems are admitted while their estimated
 * footprint fits in hbm_budget bytes and fewer than max_slots are resident;
 * their bases, pair sets and activity flags stay on the device between steps
 * (the Gebauer-Moeller update and the normal selection run on the device; a
 * few summary words per system come back each step; with F4_OPT_HOST_PAIRS
 * the pair sets are host state instead).  Each f4_server_step advances
 * every resident unfinished system by one F4 iteration with one batched
 * launch sequence (continuous batching: systems admitted between steps join
 * the next one), and systems whose pairs are exhausted get their reduced
 * basis in the same step.  One host thread at a time. */
int f4_server_create(f4_ctx* ctx, uint64_t hbm_budget, uint32_t max_slots, f4_server** out);
/* Admit a system (host SoA input, as for f4_groebner).  F4_E_BUSY when its
 * footprint or a slot is not available now (nothing is kept; retry after a
 * step).  ticket: out id, also when the system finishes at once. */
int f4_server_submit(f4_server* srv, uint32_t p, const f4_polys* F, uint64_t* ticket);
/* One engine iteration; *completed (may be NULL) = systems it finished. */
int f4_server_step(f4_server* srv, uint32_t* completed);
/* *done = 1 and *gb = the reduced basis (caller frees it with f4_basis_free)
 * when the ticket's system is finished; its slot and footprint are released.
 * *done = 0 otherwise.  F4_E_STATE for an unknown ticket. */
int f4_server_poll(f4_server* srv, uint64_t ticket, f4_basis** gb, int* done);
/* Resident systems, unfinished systems, footprint in use. */
int f4_server_load(const f4_server* srv, uint32_t* resident, uint32_t* running, uint64_t* used);
int f4_server_destroy(f4_server* srv);

/* ---------------------------------------------- modular inner loop */
/* The modular-arithmetic microbenchmark of the benchmark protocol
 * ("Microbenchmarks": randomized residues, Barrett against Montgomery update
 * kernels; updates/s, register count, spill rate).  Chain i runs
 *     x <- (b[i] + x * a[i]) mod p,   x = x0[i] at the start,
 * `iters` times (an update of the form of equation "mod-fma" whose product
 * takes the running value), and out[i] receives the final x as a standard
 * residue.  Forms:
 *   F4_MODLOOP_MUL24      p < 2^16: 24-bit product, float quotient estimate,
 *                         then a modular add (the elimination's small-p form);
 *   F4_MODLOOP_BARRETT32  p < 2^16: one-word Barrett of b + x*a < 2^32;
 *   F4_MODLOOP_BARRETT64  two-word Barrett (section "Barrett reduction as
 *                         reciprocal multiplication"), any p;
 *   F4_MODLOOP_MONTGOMERY R = 2^32 (section "Montgomery multiplication and
 *                         domain reuse"), any p; values enter the Montgomery
 *                         domain once and leave it once.
 * x0, a, b and out are host arrays of nchains residues (< p) owned by the
 * caller.  One untimed warm-up launch, then one launch timed with HIP events
 * on the context's stream.  st receives updates/s (nchains * iters / kernel
 * time), the kernel time, and the kernel's registers per lane and private
 * (spill) bytes per lane as the runtime reports them.  F4_E_ARG: p not an odd
 * prime < 2^31, an unknown form, p >= 2^16 for the 16-bit forms, nchains 0
 * or above 2^26, iters 0, a null pointer, or an input value >= p. */
enum {
    F4_MODLOOP_MUL24 = 0,
    F4_MODLOOP_BARRETT32 = 1,
    F4_MODLOOP_BARRETT64 = 2,
    F4_MODLOOP_MONTGOMERY = 3
};
typedef struct {
    double updates_per_s;
    double kernel_ms;
    uint32_t regs;
    uint32_t private_bytes;
} f4_modloop_stats;
int f4_modloop(f4_ctx* ctx, uint32_t p, uint32_t form, uint32_t nchains, uint32_t iters, const uint32_t* x0,
               const uint32_t* a, const uint32_t* b, uint32_t* out, f4_modloop_stats* st);

#ifdef __cplusplus
}
#endif

#endif /* F4_H */
