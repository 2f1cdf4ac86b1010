"""CPU oracle for the F4 step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library:

* O1 ``f4_oracle.cpp``: textbook F4 in plain C++ (exponent vectors, std::map
  dictionary, ``% p`` arithmetic), driven through ctypes by :class:`OracleRun`.
* O2 ``buchberger.py``: Buchberger's algorithm with all pairs, in pure Python.
* O3 ``dense.py``: dense Gaussian elimination over Python integers.
* O4 ``modloop.py``: the iterated modular update of the arithmetic
  microbenchmark, by ``%``.
* O5 ``krylov.py``: the block operator application Y = A X / A^T X over F_p.
* O6 ``wiedemann.py``: block Wiedemann left-kernel vectors (projected Krylov
  sequence, sigma-basis generator, kernel-vector evaluation).
* O7 ``signatures.py``: signature admissibility of shifted reducers (syzygy
  and rewrite tests), the filtered and bucketed row lists, and symbolic
  preprocessing closed over the admissible reducers only.
* O8 ``schedule.py``: the block schedule of the plan (column panels, the
  row-to-panel incidence, SELL-C-sigma windows and slices) and the padded
  slice storage.

Each is pinned in ``tests/test_oracle_*.py`` against facts fixed by the paper
and by mathematics (uniqueness of the reduced Groebner basis, closed forms,
the theorems on dictionary and matrix correctness, an independent library
routine), not against itself.
"""

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(HERE, "liborf4.so")
SRC = os.path.join(HERE, "f4_oracle.cpp")


def build(force=False):
    """Compile O1 with the host compiler (no GPU code involved)."""
    if os.environ.get("ORACLE_LIB_OVERRIDE"):
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        lib.or_create.restype = ctypes.c_void_p
        lib.or_create.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.or_destroy.argtypes = [ctypes.c_void_p]
        lib.or_add_poly.argtypes = [ctypes.c_void_p, ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)]
        lib.or_add_poly.restype = ctypes.c_int
        lib.or_set_record.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        lib.or_set_stop.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        lib.or_set_stop_deg.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        lib.or_run.argtypes = [ctypes.c_void_p]
        lib.or_run.restype = ctypes.c_int
        lib.or_len.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
        lib.or_len.restype = ctypes.c_int64
        lib.or_get.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint64)]
        lib.or_get.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleRun:
    """One O1 run of F4 on a system given as lists of (exps, coeff) terms.

    ``record``: -1 records nothing per step, -2 every step, k only step k.
    ``stop_after``: stop after step k (the basis is then left incomplete).
    ``stop_deg``: stop after the first step whose degree is ``stop_deg``.
    """

    def __init__(self, n, p, polys, record=-1, stop_after=-1, stop_deg=-1):
        lib = _load()
        self.n, self.p = n, p
        self._h = lib.or_create(n, p)
        if not self._h:
            raise ValueError("bad oracle parameters")
        for f in polys:
            k = len(f)
            ex = (ctypes.c_uint32 * max(1, k * n))()
            co = (ctypes.c_uint64 * max(1, k))()
            for t, (e, c) in enumerate(f):
                for i in range(n):
                    ex[t * n + i] = e[i]
                co[t] = c % p
            if lib.or_add_poly(self._h, k, ex, co) != 0:
                raise ValueError("exponent out of the oracle's range")
        lib.or_set_record(self._h, record)
        lib.or_set_stop(self._h, stop_after)
        lib.or_set_stop_deg(self._h, stop_deg)
        if lib.or_run(self._h) != 0:
            raise RuntimeError("oracle run failed")

    def __del__(self):
        if getattr(self, "_h", None):
            _load().or_destroy(self._h)
            self._h = None

    def array(self, name):
        lib = _load()
        k = lib.or_len(self._h, name.encode())
        if k < 0:
            raise KeyError(name)
        buf = (ctypes.c_uint64 * max(1, k))()
        lib.or_get(self._h, name.encode(), buf)
        return [int(buf[i]) for i in range(k)]

    def has(self, name):
        return _load().or_len(self._h, name.encode()) >= 0

    # ---- convenience views -------------------------------------------------
    def _polys(self, ptr, exp, coeff):
        n = self.n
        out = []
        for a in range(len(ptr) - 1):
            f = []
            for q in range(ptr[a], ptr[a + 1]):
                f.append((tuple(exp[q * n:(q + 1) * n]), coeff[q]))
            out.append(f)
        return out

    def basis(self):
        """Reduced Groebner basis: monic polys, leading monomial first, sorted
        by leading monomial, largest first."""
        return self._polys(self.array("gb.ptr"), self.array("gb.exp"), self.array("gb.coeff"))

    def steps(self):
        """Per-step shapes: list of dicts (d, r, N, M, npiv, rank, rho)."""
        s = self.array("steps")
        keys = ("d", "r", "N", "M", "npiv", "rank", "rho")
        return [dict(zip(keys, s[i:i + 7])) for i in range(0, len(s), 7)]

    def times_ns(self):
        """Per-step (build, reduce) wall times in nanoseconds."""
        t = self.array("time")
        return [(t[i], t[i + 1]) for i in range(0, len(t), 2)]

    def step_record(self, k):
        """All recorded arrays of step k as a dict (monomials as tuples)."""
        n = self.n
        pre = "s%d." % k
        if not self.has(pre + "d"):
            raise KeyError("step %d not recorded" % k)
        rec = {}
        rec["d"] = self.array(pre + "d")[0]
        rec["G"] = self._polys(self.array(pre + "G.ptr"), self.array(pre + "G.exp"),
                               self.array(pre + "G.coeff"))
        rec["active"] = self.array(pre + "G.active")
        sel = self.array(pre + "sel")
        rec["sel"] = [(sel[i], sel[i + 1]) for i in range(0, len(sel), 2)]
        for name in ("row_ptr", "col_ind", "val", "pivot_cols", "pivot_rows",
                     "rref_ptr", "rref_col", "rref_val"):
            rec[name] = self.array(pre + name)
        te = self.array(pre + "T")
        rec["T"] = [tuple(te[i * n:(i + 1) * n]) for i in range(len(te) // n)]
        rt = self.array(pre + "rows.t")
        rec["rows_t"] = [tuple(rt[i * n:(i + 1) * n]) for i in range(len(rt) // n)]
        rec["rows_k"] = self.array(pre + "rows.k")
        return rec


def groebner(n, p, polys):
    """Reduced Groebner basis by O1."""
    return OracleRun(n, p, polys).basis()
