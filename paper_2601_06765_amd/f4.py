"""Thin ctypes binding of libf4.so (include/f4.h): argument marshalling only.

Every step of the F4 path runs in the HIP library; this module packs
exponent tuples into P words, lays polynomials out as host arrays or takes
device tensors (torch, for device memory and streams), and copies results
back.  There is no fallback: if the library is missing, importing fails.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libf4.so")

F4_OK, F4_E_ARG, F4_E_RANGE, F4_E_NOMEM, F4_E_BUSY, F4_E_DEVICE, F4_E_STATE = range(7)
F4_OPT_TIMING, F4_OPT_DICT_RANK, F4_OPT_DICT_RADIX, F4_OPT_AUTOTUNE, F4_OPT_KERNEL_TIMING = 1, 2, 4, 8, 16
F4_OPT_HOST_PAIRS = 32

if not os.path.exists(LIB_PATH):
    raise ImportError("libf4.so is not built: run `python -m paper_2601_06765_amd.build` "
                      "(or __graft_entry__.build()) first")
_lib = ctypes.CDLL(LIB_PATH)

c_u32, c_u64, c_int, c_vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
P = ctypes.POINTER


ALLOC_FN = ctypes.CFUNCTYPE(c_vp, c_vp, ctypes.c_size_t, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp, c_vp)


class Opts(ctypes.Structure):
    _fields_ = [("flags", c_u32), ("stop_deg", c_u32), ("trsm_rows", c_u32), ("radix_bits", c_u32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", c_vp)]


class Polys(ctypes.Structure):
    _fields_ = [("n", c_u32), ("npolys", c_u32), ("mon", c_vp), ("coeff", c_vp), ("offset", c_vp),
                ("on_device", c_int)]


class Pair(ctypes.Structure):
    _fields_ = [("i", c_u32), ("j", c_u32)]


class RowSpec(ctypes.Structure):
    _fields_ = [("t", c_u64), ("k", c_u32), ("pad", c_u32)]


class Sigs(ctypes.Structure):
    _fields_ = [("npolys", c_u32), ("index", c_vp), ("mon", c_vp), ("nindex", c_u32), ("syz_off", c_vp),
                ("syz_mon", c_vp)]


class SigStats(ctypes.Structure):
    _fields_ = [("kept", c_u32), ("syzygy", c_u32), ("rewritten", c_u32), ("pad", c_u32),
                ("t_device_ms", ctypes.c_double)]


F4_ADM_OK, F4_ADM_SYZYGY, F4_ADM_REWRITTEN = 0, 1, 2


class MatrixView(ctypes.Structure):
    _fields_ = [("n", c_u32), ("r", c_u32), ("N", c_u32), ("deg", c_u32), ("nnz", c_u64),
                ("row_ptr", c_vp), ("col_ind", c_vp), ("val", c_vp), ("dict_keys", c_vp),
                ("row_t", c_vp), ("row_k", c_vp), ("key_words", c_u32), ("pad", c_u32)]


class ScheduleView(ctypes.Structure):
    _fields_ = [("W", c_u32), ("C", c_u32), ("sigma", c_u32), ("npanels", c_u32), ("nslices", c_u32),
                ("pad", c_u32), ("padded", c_u64), ("perm", c_vp), ("panel_ptr", c_vp), ("slice_start", c_vp),
                ("slice_panel", c_vp), ("slice_width", c_vp), ("slice_off", c_vp), ("sell_col", c_vp),
                ("sell_val", c_vp)]


class PolysMW(ctypes.Structure):
    _fields_ = [("n", c_u32), ("npolys", c_u32), ("mon", c_vp), ("coeff", c_vp), ("offset", c_vp)]


class RowSpecMW(ctypes.Structure):
    _fields_ = [("t0", c_u64), ("t1", c_u64), ("k", c_u32), ("pad", c_u32)]


class ReducedView(ctypes.Structure):
    _fields_ = [("N", c_u32), ("npivot", c_u32), ("rho", c_u32), ("rank", c_u32), ("nnz", c_u64),
                ("pivot_cols", c_vp), ("row_ptr", c_vp), ("col_ind", c_vp), ("val", c_vp)]


class StepStats(ctypes.Structure):
    _fields_ = [("deg", c_u32), ("nsel", c_u32), ("r", c_u32), ("N", c_u32), ("nnz", c_u64),
                ("npivot", c_u32), ("lower", c_u32), ("rho", c_u32), ("rank", c_u32),
                ("closure_rounds", c_u32), ("dict_path", c_u32),
                ("t_dict_ms", ctypes.c_float), ("t_assemble_ms", ctypes.c_float),
                ("t_numeric_ms", ctypes.c_float), ("t_trsm_ms", ctypes.c_float),
                ("t_echelon_ms", ctypes.c_float), ("t_step_ms", ctypes.c_float),
                ("t_pairs_ms", ctypes.c_float),
                ("t_k_trsm_ms", ctypes.c_float), ("n_k_trsm", c_u32), ("trsm_ops", c_u64),
                ("t_k_block_ms", ctypes.c_float), ("n_k_block", c_u32), ("block_ops", c_u64)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("f4_create", c_int, [P(c_vp), c_int, P(Opts)])
_sig("f4_destroy", c_int, [c_vp])
_sig("f4_last_error", ctypes.c_char_p, [c_vp])
_sig("f4_download", c_int, [c_vp, c_vp, c_vp, ctypes.c_size_t])
_sig("f4_tune_export", c_int, [c_vp, ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_size_t)])
_sig("f4_tune_import", c_int, [c_vp, ctypes.c_char_p])
_sig("f4_lane_bits", c_u32, [c_u32])
_sig("f4_pack", c_int, [c_u32, P(c_u32), P(c_u64)])
_sig("f4_unpack", c_int, [c_u32, c_u64, P(c_u32)])
_sig("f4_mw_lane_bits", c_u32, [c_u32])
_sig("f4_pack_mw", c_int, [c_u32, P(c_u32), P(c_u64)])
_sig("f4_unpack_mw", c_int, [c_u32, P(c_u64), P(c_u32)])
_sig("f4_build_matrix_rows_mw", c_int, [c_vp, c_u32, P(PolysMW), P(RowSpecMW), c_u32, P(c_vp), c_vp])
_sig("f4_normalize_polys_mw", c_int, [c_u32, P(PolysMW), P(c_u64), P(c_u32), P(c_u64)])
_sig("f4_matrix_schedule", c_int, [c_vp, c_vp, c_u32, c_u32, c_u32, P(ScheduleView), c_vp])
_sig("f4_spmm_sell", c_int, [c_vp, c_u32, c_vp, c_u32, c_vp, c_vp, c_vp])
_sig("f4_spmm_sell_timed", c_int, [c_vp, c_u32, c_vp, c_u32, c_vp, c_vp, c_u32, P(ctypes.c_double)])
_sig("f4_check_polys", c_int, [c_u32, P(Polys), c_int, P(c_u32)])
_sig("f4_normalize_polys", c_int, [c_u32, P(Polys), c_int, P(c_u64), P(c_u32), P(c_u64)])
_sig("f4_grevlex_rank", c_int, [c_u32, c_u32, c_u64, P(c_u32)])
_sig("f4_grevlex_unrank", c_int, [c_u32, c_u32, c_u32, P(c_u64)])
_sig("f4_build_matrix", c_int, [c_vp, c_u32, P(Polys), P(ctypes.c_uint8), P(Pair), c_u32, P(c_vp), c_vp])
_sig("f4_build_matrix_rows", c_int, [c_vp, c_u32, P(Polys), P(RowSpec), c_u32, P(c_vp), c_vp])
_sig("f4_sig_filter", c_int, [c_vp, c_u32, P(Polys), P(Sigs), P(RowSpec), c_u32, c_vp, P(RowSpec), P(c_u32),
                              P(c_u32), P(SigStats), c_vp])
_sig("f4_build_matrix_sig", c_int, [c_vp, c_u32, P(Polys), c_vp, P(Sigs), P(RowSpec), c_u32, P(c_vp),
                                    P(SigStats), c_vp])
_sig("f4_matrix_from_csr", c_int, [c_vp, c_u32, c_u32, P(c_u32), P(c_u32), P(c_u32), P(c_vp), c_vp])
_sig("f4_matrix_get", c_int, [c_vp, P(MatrixView)])
_sig("f4_matrix_free", c_int, [c_vp])
_sig("f4_reduce", c_int, [c_vp, c_u32, c_vp, P(c_vp), c_vp])
_sig("f4_reduced_get", c_int, [c_vp, P(ReducedView)])
_sig("f4_reduced_free", c_int, [c_vp])
_sig("f4_groebner", c_int, [c_vp, c_u32, P(Polys), P(c_vp), c_vp])
_sig("f4_groebner_batch", c_int, [c_vp, c_u32, P(c_u32), P(Polys), P(c_vp), c_vp])
_sig("f4_basis_view", c_int, [c_vp, P(Polys)])
_sig("f4_basis_stats", c_int, [c_vp, P(P(StepStats)), P(c_u32)])
_sig("f4_basis_free", c_int, [c_vp])
_sig("f4_server_footprint", c_int, [c_u32, c_u32, P(c_u64)])
_sig("f4_server_create", c_int, [c_vp, c_u64, c_u32, P(c_vp)])
_sig("f4_server_submit", c_int, [c_vp, c_u32, P(Polys), P(c_u64)])
_sig("f4_server_step", c_int, [c_vp, P(c_u32)])
_sig("f4_server_poll", c_int, [c_vp, c_u64, P(c_vp), P(c_int)])
_sig("f4_server_load", c_int, [c_vp, P(c_u32), P(c_u32), P(c_u64)])
_sig("f4_server_destroy", c_int, [c_vp])


class ModloopStats(ctypes.Structure):
    _fields_ = [("updates_per_s", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("regs", c_u32), ("private_bytes", c_u32)]


_sig("f4_spmm", c_int, [c_vp, c_u32, c_vp, c_int, c_u32, c_vp, c_vp, c_vp])
_sig("f4_spmm_noalloc", c_int, [c_vp, c_u32, c_u32, c_u32, c_u64, c_vp, c_vp, c_vp, c_int, c_u32, c_vp, c_vp,
                               c_vp])
_sig("f4_spmm_timed", c_int, [c_vp, c_u32, c_vp, c_int, c_u32, c_vp, c_vp, c_u32, P(ctypes.c_double)])
_sig("f4_device_alloc", c_int, [c_vp, ctypes.c_size_t, P(c_vp)])
_sig("f4_device_free", c_int, [c_vp, c_vp])
_sig("f4_upload", c_int, [c_vp, c_vp, c_vp, ctypes.c_size_t])
_sig("f4_modloop", c_int, [c_vp, c_u32, c_u32, c_u32, c_u32, P(c_u32), P(c_u32), P(c_u32), P(c_u32),
                           P(ModloopStats)])

class BwStats(ctypes.Structure):
    _fields_ = [("L", c_u32), ("generators", c_u32), ("t_sequence_ms", ctypes.c_double),
                ("t_mbasis_ms", ctypes.c_double), ("t_vectors_ms", ctypes.c_double)]


_sig("f4_bw_sequence", c_int, [c_vp, c_u32, c_vp, c_u32, c_vp, c_vp, c_vp, c_u32, c_vp, c_vp])
_sig("f4_bw_mbasis", c_int, [c_vp, c_u32, c_u32, c_u32, c_vp, c_vp, c_vp, c_vp])
_sig("f4_block_wiedemann", c_int, [c_vp, c_u32, c_vp, c_u32, c_vp, c_vp, c_vp, P(c_u32), c_u32, P(c_u32),
                                   P(BwStats)])

MODLOOP_FORMS = {"mul24": 0, "barrett32": 1, "barrett64": 2, "montgomery": 3}


class F4Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("f4 error %d: %s" % (code, msg))
        self.code = code


# ------------------------------------------------------------- monomials
def lane_bits(n):
    return _lib.f4_lane_bits(n)


def pack(n, exps):
    arr = (c_u32 * n)(*exps)
    out = c_u64()
    rc = _lib.f4_pack(n, arr, ctypes.byref(out))
    if rc:
        raise F4Error(rc, "cannot pack %r" % (tuple(exps),))
    return out.value


def unpack(n, word):
    arr = (c_u32 * n)()
    rc = _lib.f4_unpack(n, word, arr)
    if rc:
        raise F4Error(rc, "cannot unpack")
    return tuple(arr)


def pack_mw(n, exps):
    """Two-word monomial (high word first) of n <= 30 exponents (f4_pack_mw)."""
    arr = (c_u32 * n)(*[int(x) for x in exps])
    out = (c_u64 * 2)()
    rc = _lib.f4_pack_mw(n, arr, out)
    if rc:
        raise F4Error(rc, "cannot pack %r in two words" % (tuple(exps),))
    return int(out[0]), int(out[1])


def unpack_mw(n, words):
    arr = (c_u32 * n)()
    w = (c_u64 * 2)(int(words[0]), int(words[1]))
    rc = _lib.f4_unpack_mw(n, w, arr)
    if rc:
        raise F4Error(rc, "cannot unpack")
    return tuple(arr)


def _mw_positions(n):
    """Bit position (in the 128-bit number) of each variable's lane, from
    f4_pack_mw of the unit vectors."""
    pos = []
    for v in range(n):
        e = [0] * n
        e[v] = 1
        hi, lo = pack_mw(n, e)
        x = ((hi << 64) | lo) - (1 << 120)
        pos.append(x.bit_length() - 1)
    return pos


def pack_many_mw(n, exps):
    """Two-word monomials of many exponent vectors (rows of an integer array
    of width n) as an (m, 2) uint64 array, the same words as pack_mw."""
    e = np.asarray(exps, dtype=np.uint64).reshape(-1, n)
    w = _lib.f4_mw_lane_bits(n)
    if w == 0:
        raise F4Error(F4_E_ARG, "bad number of variables %d" % n)
    if e.size and (e.max() >= (1 << w) or e.sum(axis=1).max() > 255):
        raise F4Error(F4_E_RANGE, "an exponent or the degree does not fit its field")
    out = np.zeros((e.shape[0], 2), dtype=np.uint64)
    for v, b in enumerate(_mw_positions(n)):
        if b >= 64:
            out[:, 0] |= e[:, v] << np.uint64(b - 64)
        else:
            out[:, 1] |= e[:, v] << np.uint64(b)
    out[:, 0] |= e.sum(axis=1) << np.uint64(56)
    return out


def normalize_mw(p, n, polys):
    """f4_normalize_polys_mw: [(exps, coeff), ...] per polynomial into the
    input form of f4_build_matrix_rows_mw (terms by decreasing grevlex)."""
    off = np.zeros(len(polys) + 1, dtype=np.uint64)
    exps, coeff = [], []
    for i, f in enumerate(polys):
        for e, c in f:
            exps.append(e)
            coeff.append(int(c) % p)
        off[i + 1] = len(coeff)
    mon = np.ascontiguousarray(pack_many_mw(n, exps).reshape(-1))
    coeff = np.ascontiguousarray(np.array(coeff, dtype=np.uint32))
    mo = np.zeros(max(1, len(mon)), dtype=np.uint64)
    co = np.zeros(max(1, len(coeff)), dtype=np.uint32)
    oo = np.zeros(len(off), dtype=np.uint64)
    arg = PolysMW(n, len(polys), mon.ctypes.data, coeff.ctypes.data, off.ctypes.data)
    rc = _lib.f4_normalize_polys_mw(p, ctypes.byref(arg), mo.ctypes.data_as(P(c_u64)), co.ctypes.data_as(P(c_u32)),
                                    oo.ctypes.data_as(P(c_u64)))
    if rc:
        raise F4Error(rc, "f4_normalize_polys_mw")
    out = []
    for i in range(len(polys)):
        a, b = int(oo[i]), int(oo[i + 1])
        out.append([(unpack_mw(n, (int(mo[2 * q]), int(mo[2 * q + 1]))), int(co[q])) for q in range(a, b)])
    return out


def grevlex_rank(n, D, word):
    out = c_u32()
    rc = _lib.f4_grevlex_rank(n, D, word, ctypes.byref(out))
    if rc:
        raise F4Error(rc, "rank")
    return out.value


def grevlex_unrank(n, D, rank):
    out = c_u64()
    rc = _lib.f4_grevlex_unrank(n, D, rank, ctypes.byref(out))
    if rc:
        raise F4Error(rc, "unrank")
    return out.value


def pack_many(n, exps):
    """P words of many exponent vectors at once (rows of an integer array of
    width n), the same words as pack(): degree in the top byte, exponent i in
    lane i of width lane_bits(n)."""
    w = lane_bits(n)
    if not w:
        raise F4Error(F4_E_ARG, "bad number of variables %d" % n)
    e = np.asarray(exps, dtype=np.int64).reshape(-1, n)
    if e.size and (e.min() < 0 or e.max() >= (1 << w) or e.sum(axis=1).max() > 255):
        raise F4Error(F4_E_RANGE, "an exponent or the degree does not fit its field")
    shifts = (np.arange(n, dtype=np.uint64) * np.uint64(w))
    words = (e.astype(np.uint64) << shifts).sum(axis=1, dtype=np.uint64)
    return words | (e.sum(axis=1).astype(np.uint64) << np.uint64(56))


def polys_to_arrays(n, polys):
    """List of polys [(exps, coeff), ...] -> (mon u64, coeff u32, offset u64)
    host arrays, terms in the given order (no sorting: see normalize)."""
    terms = [t for f in polys for t in f]
    offs = np.zeros(len(polys) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(f) for f in polys])
    mons = pack_many(n, [e for e, _ in terms]) if terms else np.zeros(0, dtype=np.uint64)
    cs = [c for _, c in terms]
    if cs and (min(cs) < 0 or max(cs) >= 1 << 32):
        raise F4Error(F4_E_RANGE, "a coefficient does not fit a 32-bit word")
    coeffs = np.array(cs, dtype=np.uint64).astype(np.uint32) if terms else np.zeros(0, dtype=np.uint32)
    return mons, coeffs, offs


def check_arrays(p, n, mon, coeff, off, monic=False):
    """f4_check_polys on host arrays: (status, failed-rule bits)."""
    arg = _PolysArg(n, mon, coeff, off)
    bits = c_u32()
    rc = _lib.f4_check_polys(p, ctypes.byref(arg.s), 1 if monic else 0, ctypes.byref(bits))
    return rc, bits.value


def normalize_arrays(p, n, mon, coeff, off, monic=False):
    """f4_normalize_polys on host arrays: terms sorted by decreasing grevlex,
    repeats merged, coefficients reduced mod p, zero terms dropped (and each
    polynomial made monic with monic=True)."""
    mon = np.ascontiguousarray(mon, dtype=np.uint64)
    coeff = np.ascontiguousarray(coeff, dtype=np.uint32)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    arg = _PolysArg(n, mon, coeff, off)
    mo = np.zeros(max(1, len(mon)), dtype=np.uint64)
    co = np.zeros(max(1, len(mon)), dtype=np.uint32)
    oo = np.zeros(len(off), dtype=np.uint64)
    rc = _lib.f4_normalize_polys(p, ctypes.byref(arg.s), 1 if monic else 0, mo.ctypes.data_as(P(c_u64)),
                                 co.ctypes.data_as(P(c_u32)), oo.ctypes.data_as(P(c_u64)))
    if rc:
        raise F4Error(rc, "f4_normalize_polys")
    return mo[:int(oo[-1])], co[:int(oo[-1])], oo


def normalize(p, n, polys, monic=False):
    """Polynomials [(exps, coeff), ...] in the library's input form (see
    normalize_arrays); polynomials that cancel to zero are dropped."""
    mo, co, oo = normalize_arrays(p, n, *polys_to_arrays(n, polys), monic=monic)
    out = []
    for a in range(len(oo) - 1):
        f = [(unpack(n, int(mo[q])), int(co[q])) for q in range(int(oo[a]), int(oo[a + 1]))]
        if f:
            out.append(f)
    return out


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, DeviceArray):
        return c_vp(a.ptr)
    if hasattr(a, "data_ptr"):  # torch tensor (device or host)
        return c_vp(a.data_ptr())
    return a.ctypes.data_as(c_vp)


class _PolysArg:
    """Keeps the arrays alive while the struct is in use."""

    def __init__(self, n, mon, coeff, off, on_device=False, npolys=None):
        self.keep = (mon, coeff, off)
        k = len(off) - 1 if npolys is None else npolys
        self.s = Polys(n, k, _ptr(mon), _ptr(coeff), _ptr(off), 1 if on_device else 0)


def _sigstats(st):
    return {"kept": st.kept, "syzygy": st.syzygy, "rewritten": st.rewritten, "t_device_ms": st.t_device_ms}


# --------------------------------------------------------------- context
class Context:
    def __init__(self, device=0, timing=False, dict_path=None, stop_deg=0, autotune=False, trsm_rows=0,
                 radix_bits=0, kernel_timing=False, alloc=None, free=None, host_pairs=False):
        """alloc(bytes, stream) -> device pointer or 0, free(ptr, stream):
        optional device allocator of the context (f4_opts.alloc / .free).
        host_pairs: pair sets on the host (F4_OPT_HOST_PAIRS)."""
        flags = F4_OPT_TIMING if timing else 0
        if host_pairs:
            flags |= F4_OPT_HOST_PAIRS
        if kernel_timing:
            flags |= F4_OPT_TIMING | F4_OPT_KERNEL_TIMING
        if dict_path == "rank":
            flags |= F4_OPT_DICT_RANK
        elif dict_path == "radix":
            flags |= F4_OPT_DICT_RADIX
        if autotune:
            flags |= F4_OPT_AUTOTUNE
        self._h = c_vp()
        opts = Opts(flags, stop_deg, trsm_rows, radix_bits)
        if alloc is not None:
            # the callbacks must outlive the context: keep them on it
            self._cb = (ALLOC_FN(lambda user, nbytes, stream: alloc(nbytes, stream) or None),
                        FREE_FN(lambda user, ptr, stream: free(ptr, stream)))
            opts.alloc, opts.free = self._cb
        rc = _lib.f4_create(ctypes.byref(self._h), device, ctypes.byref(opts))
        if rc:
            raise F4Error(rc, "f4_create failed")

    def tune_table(self):
        """The autotuner's table as text (f4_tune_export)."""
        n = ctypes.c_size_t(0)
        self._check(_lib.f4_tune_export(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        self._check(_lib.f4_tune_export(self._h, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def load_tune_table(self, text):
        """Merge a table in the text form of tune_table() (f4_tune_import)."""
        self._check(_lib.f4_tune_import(self._h, text.encode()))

    def modloop(self, p, form, x0, a, b, iters):
        """Modular inner-loop microbenchmark (f4_modloop): chain i runs
        x <- (b[i] + x * a[i]) mod p `iters` times from x0[i] in the named
        form; returns (final values, stats dict)."""
        x0, a, b = (np.ascontiguousarray(v, dtype=np.uint32) for v in (x0, a, b))
        if not (len(x0) == len(a) == len(b)):
            raise ValueError("x0, a and b differ in length")
        out = np.empty(len(x0), dtype=np.uint32)
        st = ModloopStats()
        u = P(c_u32)
        self._check(_lib.f4_modloop(self._h, p, MODLOOP_FORMS[form], len(x0), iters, x0.ctypes.data_as(u),
                                    a.ctypes.data_as(u), b.ctypes.data_as(u), out.ctypes.data_as(u),
                                    ctypes.byref(st)))
        return out, {"updates_per_s": st.updates_per_s, "kernel_ms": st.kernel_ms, "regs": st.regs,
                     "private_bytes": st.private_bytes}

    def close(self):
        if self._h:
            _lib.f4_destroy(self._h)
            self._h = c_vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise F4Error(rc, (_lib.f4_last_error(self._h) or b"").decode())

    def download(self, ptr, count, dtype):
        out = np.empty(count, dtype=dtype)
        if count:
            self._check(_lib.f4_download(self._h, out.ctypes.data_as(c_vp), c_vp(ptr), out.nbytes))
        return out

    # -- full F4
    def _basis(self, h, n):
        v = Polys()
        _lib.f4_basis_view(h, ctypes.byref(v))
        k = v.npolys
        offs = np.ctypeslib.as_array(ctypes.cast(v.offset, P(c_u64)), (k + 1,)).copy() if k else [0]
        nt = int(offs[-1])
        mons = np.ctypeslib.as_array(ctypes.cast(v.mon, P(c_u64)), (nt,)).copy() if nt else []
        cfs = np.ctypeslib.as_array(ctypes.cast(v.coeff, P(c_u32)), (nt,)).copy() if nt else []
        basis = []
        for a in range(k):
            basis.append([(unpack(n, int(mons[q])), int(cfs[q])) for q in range(int(offs[a]), int(offs[a + 1]))])
        sp = P(StepStats)()
        ns = c_u32()
        _lib.f4_basis_stats(h, ctypes.byref(sp), ctypes.byref(ns))
        steps = []
        for i in range(ns.value):
            s = sp[i]
            steps.append({name: getattr(s, name) for name, _ in StepStats._fields_})
        return basis, steps

    def prepare(self, p, n, polys):
        """Marshal one system once; the result feeds groebner_prepared."""
        mon, coeff, off = polys_to_arrays(n, [[(e, c % p) for e, c in f] for f in polys])
        return (p, n, _PolysArg(n, mon, coeff, off))

    def groebner(self, p, n, polys, stream=None):
        """Reduced Groebner basis of a system given as lists of (exps, coeff).
        Returns (basis, steps): basis as lists of (exps, coeff), leading term
        first, sorted by leading monomial (largest first); steps as dicts."""
        return self.groebner_prepared(self.prepare(p, n, polys), stream)

    def groebner_prepared(self, prep, stream=None):
        p, n, arg = prep
        h = c_vp()
        self._check(_lib.f4_groebner(self._h, p, ctypes.byref(arg.s), ctypes.byref(h), c_vp(stream)))
        try:
            return self._basis(h, n)
        finally:
            _lib.f4_basis_free(h)

    def prepare_batch(self, systems):
        """Marshal [(p, n, polys), ...] once; the result feeds groebner_batch_prepared."""
        args = [_PolysArg(n, *polys_to_arrays(n, [[(e, c % p) for e, c in f] for f in polys]))
                for p, n, polys in systems]
        arr = (Polys * len(args))(*[a.s for a in args])
        ps = (c_u32 * len(args))(*[p for p, _, _ in systems])
        ns = [n for _, n, _ in systems]
        return (args, arr, ps, ns)

    def groebner_batch_prepared(self, prep, stream=None):
        args, arr, ps, ns = prep
        hs = (c_vp * len(args))()
        self._check(_lib.f4_groebner_batch(self._h, len(args), ps, arr, hs, c_vp(stream)))
        out = []
        try:
            for i, n in enumerate(ns):
                out.append(self._basis(hs[i], n))
        finally:
            for i in range(len(args)):
                if hs[i]:
                    _lib.f4_basis_free(hs[i])
        return out

    def groebner_batch(self, systems, stream=None):
        """Reduced Groebner bases of independent systems [(p, n, polys), ...],
        computed together (one batched launch sequence per F4 iteration)."""
        return self.groebner_batch_prepared(self.prepare_batch(systems), stream)

    # -- one step
    def build_matrix(self, p, n, G, active, sel, stream=None, device_arrays=None):
        """Symbolic preprocessing for the selected pairs.  G: list of polys in
        the library's input form (monic, terms by decreasing grevlex; see
        normalize) or, with device_arrays=(mon, coeff, off, npolys) (three
        DeviceArray blocks holding the u64 / u32 / u64 arrays), a
        device-resident basis."""
        if device_arrays is not None:
            mon, coeff, off, k = device_arrays
            arg = _PolysArg(n, mon, coeff, off, on_device=True, npolys=k)
        else:
            arg = _PolysArg(n, *polys_to_arrays(n, G))
        act = np.array([1 if a else 0 for a in active], dtype=np.uint8)
        pairs = (Pair * len(sel))(*[Pair(i, j) for i, j in sel])
        h = c_vp()
        self._check(_lib.f4_build_matrix(self._h, p, ctypes.byref(arg.s),
                                         act.ctypes.data_as(P(ctypes.c_uint8)), pairs, len(sel),
                                         ctypes.byref(h), c_vp(stream)))
        return Matrix(self, h, n)

    def build_matrix_rows(self, p, n, G, rows, stream=None):
        """Matrix of an explicit row list [(t exps, k), ...]; G in the
        library's input form (see normalize)."""
        arg = _PolysArg(n, *polys_to_arrays(n, G))
        rs = (RowSpec * len(rows))(*[RowSpec(pack(n, t), k, 0) for t, k in rows])
        h = c_vp()
        self._check(_lib.f4_build_matrix_rows(self._h, p, ctypes.byref(arg.s), rs, len(rows), ctypes.byref(h),
                                              c_vp(stream)))
        return Matrix(self, h, n)

    def build_matrix_rows_packed(self, p, n, G, t_words, ks, stream=None):
        """build_matrix_rows with the shifts given as arrays: t_words (P words,
        e.g. from pack_many) and ks (basis indices), marshalled in bulk."""
        arg = _PolysArg(n, *polys_to_arrays(n, G))
        t_words = np.asarray(t_words, dtype=np.uint64)
        rs = np.zeros(len(t_words), dtype=np.dtype([("t", "<u8"), ("k", "<u4"), ("pad", "<u4")]))
        rs["t"] = t_words
        rs["k"] = np.asarray(ks, dtype=np.uint32)
        h = c_vp()
        self._check(_lib.f4_build_matrix_rows(self._h, p, ctypes.byref(arg.s), rs.ctypes.data_as(P(RowSpec)),
                                              len(rs), ctypes.byref(h), c_vp(stream)))
        return Matrix(self, h, n)

    # -- signatures
    @staticmethod
    def _sigs(n, sig_index, sig_mon, syz):
        """Marshal signatures: sig_index[k], sig_mon[k] (exps) per element and
        syz[i] (list of exps) per index.  Returns (Sigs, keep-alive arrays)."""
        idx = np.ascontiguousarray(np.asarray(sig_index, dtype=np.uint32))
        mon = np.ascontiguousarray(pack_many(n, [tuple(e) for e in sig_mon]) if len(sig_mon)
                                   else np.zeros(0, dtype=np.uint64))
        off = np.zeros(len(syz) + 1, dtype=np.uint32)
        flat = []
        for i, lst in enumerate(syz):
            flat += [tuple(e) for e in lst]
            off[i + 1] = len(flat)
        smon = np.ascontiguousarray(pack_many(n, flat) if flat else np.zeros(1, dtype=np.uint64))
        sg = Sigs(len(idx), idx.ctypes.data, mon.ctypes.data, len(syz), off.ctypes.data, smon.ctypes.data)
        return sg, (idx, mon, off, smon)

    @staticmethod
    def _rows(n, rows):
        rs = np.zeros(len(rows), dtype=np.dtype([("t", "<u8"), ("k", "<u4"), ("pad", "<u4")]))
        if len(rows):
            rs["t"] = pack_many(n, [tuple(t) for t, _ in rows])
            rs["k"] = np.asarray([k for _, k in rows], dtype=np.uint32)
        return rs

    def sig_filter(self, p, n, G, sig_index, sig_mon, syz, rows, stream=None):
        """f4_sig_filter: (flags, kept rows, schedule, stats) for rows
        [(t exps, k), ...] of the basis G (library input form)."""
        arg = _PolysArg(n, *polys_to_arrays(n, G))
        sg, keep = self._sigs(n, sig_index, sig_mon, syz)
        rs = self._rows(n, rows)
        r = len(rs)
        flags = np.zeros(r, dtype=np.uint8)
        kept = np.zeros(r, dtype=rs.dtype)
        order = np.zeros(r, dtype=np.uint32)
        nk = c_u32()
        st = SigStats()
        self._check(_lib.f4_sig_filter(self._h, p, ctypes.byref(arg.s), ctypes.byref(sg),
                                       rs.ctypes.data_as(P(RowSpec)), r, flags.ctypes.data_as(c_vp),
                                       kept.ctypes.data_as(P(RowSpec)), ctypes.byref(nk),
                                       order.ctypes.data_as(P(c_u32)), ctypes.byref(st), c_vp(stream)))
        k = nk.value
        kept_rows = [(unpack(n, int(kept["t"][q])), int(kept["k"][q])) for q in range(k)]
        return flags, kept_rows, [int(x) for x in order[:k]], _sigstats(st)

    def sig_filter_packed(self, p, n, G, sigs_packed, t_words, ks, schedule=True, stream=None):
        """f4_sig_filter on rows given as arrays (P words, indices), with
        signatures already marshalled by _sigs; returns (flags, nkept, order,
        stats) without unpacking the kept rows (order None without the
        schedule)."""
        arg = _PolysArg(n, *polys_to_arrays(n, G))
        sg, _keep = sigs_packed
        rs = np.zeros(len(t_words), dtype=np.dtype([("t", "<u8"), ("k", "<u4"), ("pad", "<u4")]))
        rs["t"] = np.asarray(t_words, dtype=np.uint64)
        rs["k"] = np.asarray(ks, dtype=np.uint32)
        r = len(rs)
        flags = np.zeros(r, dtype=np.uint8)
        order = np.zeros(r, dtype=np.uint32)
        nk = c_u32()
        st = SigStats()
        self._check(_lib.f4_sig_filter(self._h, p, ctypes.byref(arg.s), ctypes.byref(sg),
                                       rs.ctypes.data_as(P(RowSpec)), r, flags.ctypes.data_as(c_vp), None,
                                       ctypes.byref(nk), order.ctypes.data_as(P(c_u32)) if schedule else None,
                                       ctypes.byref(st), c_vp(stream)))
        return flags, nk.value, (order[:nk.value] if schedule else None), _sigstats(st)

    def build_matrix_sig(self, p, n, G, active, sig_index, sig_mon, syz, rows, stream=None):
        """f4_build_matrix_sig: (Matrix, stats)."""
        arg = _PolysArg(n, *polys_to_arrays(n, G))
        sg, keep = self._sigs(n, sig_index, sig_mon, syz)
        rs = self._rows(n, rows)
        act = np.array([1 if a else 0 for a in active], dtype=np.uint8)
        h = c_vp()
        st = SigStats()
        self._check(_lib.f4_build_matrix_sig(self._h, p, ctypes.byref(arg.s), act.ctypes.data_as(c_vp),
                                             ctypes.byref(sg), rs.ctypes.data_as(P(RowSpec)), len(rs),
                                             ctypes.byref(h), ctypes.byref(st), c_vp(stream)))
        return Matrix(self, h, n), _sigstats(st)

    # -- two-word monomial keys
    def build_matrix_rows_mw_packed(self, p, n, G, t_words, ks, stream=None):
        """build_matrix_rows_mw with the shifts as an (r, 2) array of two-word
        monomials (pack_many_mw) and ks the basis indices."""
        off = np.zeros(len(G) + 1, dtype=np.uint64)
        exps, coeff = [], []
        for i, g in enumerate(G):
            for e, c in g:
                exps.append(e)
                coeff.append(int(c) % p)
            off[i + 1] = len(coeff)
        mon = np.ascontiguousarray(pack_many_mw(n, exps).reshape(-1))
        coeff = np.ascontiguousarray(np.array(coeff, dtype=np.uint32))
        pg = PolysMW(n, len(G), mon.ctypes.data, coeff.ctypes.data, off.ctypes.data)
        t_words = np.asarray(t_words, dtype=np.uint64).reshape(-1, 2)
        rs = np.zeros(len(t_words), dtype=np.dtype([("t0", "<u8"), ("t1", "<u8"), ("k", "<u4"), ("pad", "<u4")]))
        rs["t0"] = t_words[:, 0]
        rs["t1"] = t_words[:, 1]
        rs["k"] = np.asarray(ks, dtype=np.uint32)
        h = c_vp()
        self._check(_lib.f4_build_matrix_rows_mw(self._h, p, ctypes.byref(pg), rs.ctypes.data_as(P(RowSpecMW)),
                                                 len(rs), ctypes.byref(h), c_vp(stream)))
        return Matrix(self, h, n)

    def build_matrix_rows_mw(self, p, n, G, rows, stream=None):
        """f4_build_matrix_rows_mw: the matrix of rows [(t exps, k), ...] of a
        basis G (polys [(exps, coeff), ...], terms by decreasing grevlex,
        coefficients in [1, p)) for n <= 30 variables."""
        off = np.zeros(len(G) + 1, dtype=np.uint64)
        mon, coeff = [], []
        for i, g in enumerate(G):
            for e, c in g:
                mon.extend(pack_mw(n, e))
                coeff.append(int(c) % p)
            off[i + 1] = len(coeff)
        mon = np.ascontiguousarray(np.array(mon, dtype=np.uint64))
        coeff = np.ascontiguousarray(np.array(coeff, dtype=np.uint32))
        pg = PolysMW(n, len(G), mon.ctypes.data, coeff.ctypes.data, off.ctypes.data)
        rs = (RowSpecMW * len(rows))()
        for q, (t, k) in enumerate(rows):
            t0, t1 = pack_mw(n, t)
            rs[q] = RowSpecMW(t0, t1, k, 0)
        h = c_vp()
        self._check(_lib.f4_build_matrix_rows_mw(self._h, p, ctypes.byref(pg), rs, len(rows), ctypes.byref(h),
                                                 c_vp(stream)))
        return Matrix(self, h, n)

    def device_array(self, shape):
        """A block of u32 words in device memory from this context's cache."""
        return DeviceArray(self, shape)

    def to_device(self, arr):
        """Upload a host array of words (taken modulo 2^32) as a DeviceArray."""
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint64).astype(np.uint32))
        d = DeviceArray(self, a.shape)
        if a.size:
            self._check(_lib.f4_upload(self._h, c_vp(d.ptr), a.ctypes.data_as(c_vp), a.nbytes))
        return d

    def _spmm_args(self, A, X, trans, out):
        b = 1 if len(X.shape) == 1 else X.shape[1]
        nin, nout = (A.view.r, A.view.N) if trans else (A.view.N, A.view.r)
        if X.shape[0] != nin:
            raise ValueError("block rows do not match the matrix")
        if out is None:
            out = DeviceArray(self, (nout, b) if len(X.shape) == 2 else (nout,))
        elif out.size != nout * b:
            raise ValueError("output block does not match")
        return b, out

    def spmm(self, p, A, X, trans=False, out=None, stream=None):
        """Y = A X (or A^T X) over F_p on the device (f4_spmm); X a DeviceArray
        of shape (rows, b) or (rows,); returns Y as a DeviceArray."""
        b, out = self._spmm_args(A, X, trans, out)
        self._check(_lib.f4_spmm(self._h, p, A._h, 1 if trans else 0, b, c_vp(X.ptr), c_vp(out.ptr), c_vp(stream)))
        return out

    def spmm_noalloc(self, p, r, N, nnz, row_ptr, col_ind, val, X, out, trans=False, stream=None):
        """Y = A X (or A^T X) over F_p for a CSR matrix in caller DeviceArrays
        (f4_spmm_noalloc: allocates nothing; the transpose goes to the
        library's per-GPU scratch array).  X and out are DeviceArrays."""
        b = 1 if len(X.shape) == 1 else X.shape[1]
        nin, nout = (r, N) if trans else (N, r)
        if X.shape[0] != nin or out.size != nout * b:
            raise ValueError("blocks do not match the matrix")
        self._check(_lib.f4_spmm_noalloc(self._h, p, r, N, nnz, c_vp(row_ptr.ptr), c_vp(col_ind.ptr),
                                         c_vp(val.ptr), 1 if trans else 0, b, c_vp(X.ptr), c_vp(out.ptr),
                                         c_vp(stream)))
        return out

    def schedule(self, A, W, C, sigma, stream=None):
        """f4_matrix_schedule: build the block schedule of A; returns its
        arrays downloaded to the host (perm, panel_ptr, slices, storage)."""
        v = ScheduleView()
        self._check(_lib.f4_matrix_schedule(self._h, A._h, W, C, sigma, ctypes.byref(v), c_vp(stream)))
        d = self.download
        r = A.view.r
        return {"W": v.W, "C": v.C, "sigma": v.sigma, "npanels": v.npanels, "nslices": v.nslices,
                "padded": v.padded, "perm": d(v.perm, r, np.uint32),
                "panel_ptr": d(v.panel_ptr, v.npanels + 2, np.uint32),
                "slice_start": d(v.slice_start, v.nslices, np.uint32),
                "slice_panel": d(v.slice_panel, v.nslices, np.uint32),
                "slice_width": d(v.slice_width, v.nslices, np.uint32),
                "slice_off": d(v.slice_off, v.nslices + 1, np.uint64),
                "sell_col": d(v.sell_col, v.padded, np.uint32), "sell_val": d(v.sell_val, v.padded, np.uint32)}

    def schedule_build(self, A, W, C, sigma, stream=None):
        """f4_matrix_schedule without downloading any array; returns the
        schedule's sizes (npanels, nslices, padded)."""
        v = ScheduleView()
        self._check(_lib.f4_matrix_schedule(self._h, A._h, W, C, sigma, ctypes.byref(v), c_vp(stream)))
        return {"npanels": v.npanels, "nslices": v.nslices, "padded": v.padded}

    def spmm_sell(self, p, A, X, out=None, stream=None):
        """Y = A X through the block schedule's slices (f4_spmm_sell)."""
        b, out = self._spmm_args(A, X, False, out)
        self._check(_lib.f4_spmm_sell(self._h, p, A._h, b, c_vp(X.ptr), c_vp(out.ptr), c_vp(stream)))
        return out

    def spmm_sell_timed(self, p, A, X, out=None, reps=10):
        b, out = self._spmm_args(A, X, False, out)
        ms = ctypes.c_double(0.0)
        self._check(_lib.f4_spmm_sell_timed(self._h, p, A._h, b, c_vp(X.ptr), c_vp(out.ptr), reps,
                                            ctypes.byref(ms)))
        return out, ms.value

    def spmm_timed(self, p, A, X, trans=False, out=None, reps=10):
        """spmm repeated `reps` times between HIP events on the context's
        stream (f4_spmm_timed); returns (Y, mean milliseconds per call)."""
        b, out = self._spmm_args(A, X, trans, out)
        ms = ctypes.c_double(0.0)
        self._check(_lib.f4_spmm_timed(self._h, p, A._h, 1 if trans else 0, b, c_vp(X.ptr), c_vp(out.ptr), reps,
                                       ctypes.byref(ms)))
        return out, ms.value

    def bw_sequence(self, p, A, d, X, Y, L):
        """Projected block Krylov sequence S_t = X^T B^t (B Y), B = A D A^T
        (f4_bw_sequence); d, X, Y are DeviceArrays.  Returns an L x b x b array."""
        b = X.shape[1]
        S = DeviceArray(self, (L, b, b))
        try:
            self._check(_lib.f4_bw_sequence(self._h, p, A._h, b, c_vp(d.ptr), c_vp(X.ptr), c_vp(Y.ptr), L,
                                            c_vp(S.ptr), None))
            return S.to_host().astype(np.int64)
        finally:
            S.free()

    def bw_mbasis(self, p, b, S):
        """Sigma-basis of [S(x)^T ; -I_b] to order L = len(S) (f4_bw_mbasis).
        Returns (P, shifts): P[i, j, l] is coefficient l of entry (i, j)."""
        S = np.asarray(S)
        L = S.shape[0]
        Sd = self.to_device(S.reshape(-1))
        Pd = DeviceArray(self, (2 * b, 2 * b, L + 2))
        sd = DeviceArray(self, (2 * b,))
        try:
            self._check(_lib.f4_bw_mbasis(self._h, p, b, L, c_vp(Sd.ptr), c_vp(Pd.ptr), c_vp(sd.ptr), None))
            return Pd.to_host().astype(np.int64), [int(x) for x in sd.to_host()]
        finally:
            for a in (Sd, Pd, sd):
                a.free()

    def block_wiedemann(self, p, A, d, X, Y):
        """Left-kernel vectors of A by block Wiedemann (f4_block_wiedemann);
        returns (list of vectors as int64 arrays of length r, stats dict)."""
        b = X.shape[1]
        r = A.view.r
        cap = 2 * b
        V = np.zeros(max(1, cap * r), dtype=np.uint32)
        n = c_u32(0)
        st = BwStats()
        self._check(_lib.f4_block_wiedemann(self._h, p, A._h, b, c_vp(d.ptr), c_vp(X.ptr), c_vp(Y.ptr),
                                            V.ctypes.data_as(P(c_u32)), cap, ctypes.byref(n), ctypes.byref(st)))
        vecs = [V[i * r:(i + 1) * r].astype(np.int64) for i in range(min(n.value, cap))]
        return vecs, {"L": st.L, "generators": st.generators, "t_sequence_ms": st.t_sequence_ms,
                      "t_mbasis_ms": st.t_mbasis_ms, "t_vectors_ms": st.t_vectors_ms}

    def matrix_from_csr(self, r, N, row_ptr, col_ind, val, stream=None):
        rp = np.ascontiguousarray(row_ptr, dtype=np.uint32)
        ci = np.ascontiguousarray(col_ind, dtype=np.uint32)
        vv = np.ascontiguousarray(val, dtype=np.uint32)
        h = c_vp()
        self._check(_lib.f4_matrix_from_csr(self._h, r, N, rp.ctypes.data_as(P(c_u32)),
                                            ci.ctypes.data_as(P(c_u32)) if len(ci) else None,
                                            vv.ctypes.data_as(P(c_u32)) if len(vv) else None,
                                            ctypes.byref(h), c_vp(stream)))
        return Matrix(self, h, 0)

    def reduce(self, p, A, stream=None):
        h = c_vp()
        self._check(_lib.f4_reduce(self._h, p, A._h, ctypes.byref(h), c_vp(stream)))
        return Reduced(self, h)


class DeviceArray:
    """u32 words in device memory owned by a context (f4_device_alloc)."""

    def __init__(self, ctx, shape):
        self.ctx = ctx
        self.shape = tuple(int(x) for x in (shape if isinstance(shape, (tuple, list)) else (shape,)))
        self.size = int(np.prod(self.shape, dtype=np.int64)) if self.shape else 1
        h = c_vp()
        ctx._check(_lib.f4_device_alloc(ctx._h, max(1, self.size) * 4, ctypes.byref(h)))
        self.ptr = h.value

    def to_host(self):
        return self.ctx.download(self.ptr, self.size, np.uint32).reshape(self.shape)

    def sub(self, offset, shape):
        """A view of `shape` words starting `offset` words in (no copy; the
        block must outlive it)."""
        v = DeviceArray.__new__(DeviceArray)
        v.ctx, v.owner = self.ctx, self
        v.shape = tuple(int(x) for x in (shape if isinstance(shape, (tuple, list)) else (shape,)))
        v.size = int(np.prod(v.shape, dtype=np.int64)) if v.shape else 1
        if offset < 0 or offset + v.size > self.size:
            raise ValueError("view outside the block")
        v.ptr = self.ptr + 4 * offset
        return v

    def free(self):
        if getattr(self, "owner", None) is not None:  # a view frees nothing
            self.ptr = None
            return
        if self.ptr and self.ctx._h:
            _lib.f4_device_free(self.ctx._h, c_vp(self.ptr))
        self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Matrix:
    def __init__(self, ctx, h, n):
        self.ctx, self._h, self.n = ctx, h, n
        self.view = MatrixView()
        _lib.f4_matrix_get(h, ctypes.byref(self.view))

    def free(self):
        if self._h:
            _lib.f4_matrix_free(self._h)
            self._h = c_vp()

    def __del__(self):
        try:
            if self.ctx._h:
                self.free()
        except Exception:
            pass

    def to_host(self):
        v, d = self.view, self.ctx.download
        out = {"r": v.r, "N": v.N, "nnz": v.nnz, "deg": v.deg,
               "row_ptr": d(v.row_ptr, v.r + 1, np.uint32),
               "col_ind": d(v.col_ind, v.nnz, np.uint32),
               "val": d(v.val, v.nnz, np.uint32)}
        if v.dict_keys:
            kw = max(1, v.key_words)
            out["key_words"] = kw
            out["dict_keys"] = d(v.dict_keys, v.N * kw, np.uint64)
            out["row_t"] = d(v.row_t, v.r * kw, np.uint64)
            out["row_k"] = d(v.row_k, v.r, np.uint32)
            if kw == 2:
                out["dict_keys"] = out["dict_keys"].reshape(-1, 2)
                out["row_t"] = out["row_t"].reshape(-1, 2)
        return out


class Reduced:
    def __init__(self, ctx, h):
        self.ctx, self._h = ctx, h
        self.view = ReducedView()
        _lib.f4_reduced_get(h, ctypes.byref(self.view))

    def free(self):
        if self._h:
            _lib.f4_reduced_free(self._h)
            self._h = c_vp()

    def __del__(self):
        try:
            if self.ctx._h:
                self.free()
        except Exception:
            pass

    def to_host(self):
        v, d = self.view, self.ctx.download
        return {"N": v.N, "npivot": v.npivot, "rho": v.rho, "rank": v.rank, "nnz": v.nnz,
                "pivot_cols": d(v.pivot_cols, v.npivot, np.uint32),
                "row_ptr": d(v.row_ptr, v.rho + 1, np.uint32),
                "col_ind": d(v.col_ind, v.nnz, np.uint32),
                "val": d(v.val, v.nnz, np.uint32)}


def server_footprint(n, m):
    out = c_u64()
    rc = _lib.f4_server_footprint(n, m, ctypes.byref(out))
    if rc:
        raise F4Error(rc, "footprint")
    return out.value


class Server:
    """Continuous-batching F4 server on a context (f4_server_* of include/f4.h)."""

    def __init__(self, ctx, hbm_budget, max_slots):
        self.ctx = ctx
        self._h = c_vp()
        ctx._check(_lib.f4_server_create(ctx._h, hbm_budget, max_slots, ctypes.byref(self._h)))
        self._n = {}

    @staticmethod
    def prepare(p, n, polys):
        return (p, n, _PolysArg(n, *polys_to_arrays(n, [[(e, c % p) for e, c in f] for f in polys])))

    def submit_prepared(self, prep):
        """Ticket, or None when the server is busy (retry after a step)."""
        p, n, arg = prep
        t = c_u64()
        rc = _lib.f4_server_submit(self._h, p, ctypes.byref(arg.s), ctypes.byref(t))
        if rc == F4_E_BUSY:
            return None
        self.ctx._check(rc)
        self._n[t.value] = n
        return t.value

    def submit(self, p, n, polys):
        return self.submit_prepared(self.prepare(p, n, polys))

    def step(self):
        k = c_u32()
        self.ctx._check(_lib.f4_server_step(self._h, ctypes.byref(k)))
        return k.value

    def poll(self, ticket):
        """(basis, steps) when finished (the slot is released), else None."""
        h = c_vp()
        d = c_int()
        self.ctx._check(_lib.f4_server_poll(self._h, ticket, ctypes.byref(h), ctypes.byref(d)))
        if not d.value:
            return None
        try:
            return self.ctx._basis(h, self._n.pop(ticket))
        finally:
            _lib.f4_basis_free(h)

    def load(self):
        a, b, u = c_u32(), c_u32(), c_u64()
        _lib.f4_server_load(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(u))
        return a.value, b.value, u.value

    def close(self):
        if self._h and self.ctx._h:
            _lib.f4_server_destroy(self._h)
        self._h = c_vp()
