"""Error paths of the C-ABI on the device (each returns its status and leaves
the context usable): malformed basis input to the matrix builders (host and
device arrays), matrix values that are not residues mod p, handles of another
context, and device allocation failures through the context's allocator
callbacks (F4_E_NOMEM, then a successful call on the same context).

No kernel is made to fault: every bad input here is refused by the host checks
or by the builders' own check kernel, which only reads the arrays.
"""

import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def f4():
    import paper_2601_06765_amd.f4 as mod
    return mod


@pytest.fixture(scope="module")
def ctx(f4):
    c = f4.Context(0)
    yield c
    c.close()


def step_record(n, p, polys, k):
    run = oracle.OracleRun(n, p, polys, record=k)
    return run.step_record(k)


def device_basis(f4, ctx, n, mon, coeff, off):
    """The arrays of a basis as DeviceArray blocks of u32 words."""
    return (ctx.to_device(np.asarray(mon, dtype=np.uint64).view(np.uint32)),
            ctx.to_device(np.asarray(coeff, dtype=np.uint32)),
            ctx.to_device(np.asarray(off, dtype=np.uint64).view(np.uint32)), len(off) - 1)


def test_build_rejects_malformed_basis(f4, ctx):
    n, p, polys = synth.system("dense_n6")
    rec = step_record(n, p, polys, 2)
    mon, coeff, off = f4.polys_to_arrays(n, rec["G"])
    say("build_matrix with the recorded basis (host and device arrays)")
    want = ctx.build_matrix(p, n, rec["G"], rec["active"], rec["sel"]).to_host()
    got = ctx.build_matrix(p, n, None, rec["active"], rec["sel"],
                           device_arrays=device_basis(f4, ctx, n, mon, coeff, off)).to_host()
    assert got["col_ind"].tolist() == want["col_ind"].tolist() and got["val"].tolist() == want["val"].tolist()
    assert want["col_ind"].tolist() == rec["col_ind"]
    cases = {}
    sw = mon.copy()
    a = int(off[0])
    sw[[a + 1, a + 2]] = sw[[a + 2, a + 1]]
    cases["unsorted"] = (sw, coeff)
    rep = mon.copy()
    rep[a + 2] = rep[a + 1]
    cases["repeated"] = (rep, coeff)
    c0 = coeff.copy()
    c0[a + 3] = 0
    cases["zero coefficient"] = (mon, c0)
    cp = coeff.copy()
    cp[a + 3] = p + 1
    cases["coefficient >= p"] = (mon, cp)
    nm = coeff.copy()
    nm[a] = 3
    cases["not monic"] = (mon, nm)
    for name, (m, c) in cases.items():
        for on_dev in (False, True):
            say("build_matrix rejects", name, "device" if on_dev else "host")
            with pytest.raises(f4.F4Error) as e:
                if on_dev:
                    ctx.build_matrix(p, n, None, rec["active"], rec["sel"],
                                     device_arrays=device_basis(f4, ctx, n, m, c, off))
                else:
                    arg_polys = [[(f4.unpack(n, int(m[q])), int(c[q])) for q in range(int(off[k]), int(off[k + 1]))]
                                 for k in range(len(off) - 1)]
                    ctx.build_matrix(p, n, arg_polys, rec["active"], rec["sel"])
            assert e.value.code == f4.F4_E_ARG
    say("context still usable")
    again = ctx.build_matrix(p, n, rec["G"], rec["active"], rec["sel"]).to_host()
    assert again["col_ind"].tolist() == rec["col_ind"] and again["val"].tolist() == rec["val"]


def test_build_rows_rejects_unsorted(f4, ctx):
    n, p = 4, 65521
    G = [[((0, 0, 1, 0), 1), ((1, 0, 0, 0), 5)]]  # x3 before x1: not decreasing grevlex
    say("build_matrix_rows rejects unsorted terms")
    with pytest.raises(f4.F4Error) as e:
        ctx.build_matrix_rows(p, n, G, [((0, 0, 0, 0), 0)])
    assert e.value.code == f4.F4_E_ARG
    A = ctx.build_matrix_rows(p, n, f4.normalize(p, n, G), [((0, 0, 0, 0), 0)]).to_host()
    assert A["nnz"] == 2 and A["val"].tolist() == [5, 1]


def test_build_rows_checks_rows_on_device(f4, ctx):
    import numpy as np
    n, p = 4, 65521
    G = f4.normalize(p, n, [[((0, 1, 0, 0), 1), ((0, 0, 0, 1), 3)], [((1, 0, 0, 0), 1), ((0, 0, 0, 0), 2)]])
    t_ok = f4.pack(n, (0, 0, 1, 0))
    say("build_matrix_rows: basis index out of range")
    with pytest.raises(f4.F4Error) as e:
        ctx.build_matrix_rows_packed(p, n, G, np.array([t_ok, t_ok], dtype=np.uint64), np.array([0, 2]))
    assert e.value.code == f4.F4_E_ARG
    say("build_matrix_rows: a shift word whose lanes do not add up to its degree")
    bad = (1 << 56) | f4.pack(n, (0, 0, 2, 0))  # degree field 1 + 2 = 3, lanes 2
    with pytest.raises(f4.F4Error) as e:
        ctx.build_matrix_rows_packed(p, n, G, np.array([bad], dtype=np.uint64), np.array([0]))
    assert e.value.code == f4.F4_E_ARG
    say("build_matrix_rows: exponent lane overflow")
    w = f4.lane_bits(n)
    big = f4.pack(n, (0, (1 << w) - 1, 0, 0))  # times x2 overflows the lane
    with pytest.raises(f4.F4Error) as e:
        ctx.build_matrix_rows_packed(p, n, G, np.array([big], dtype=np.uint64), np.array([0]))
    assert e.value.code == f4.F4_E_RANGE
    say("build_matrix_rows: repeated rows collapse, context still usable")
    ts = np.array([t_ok, t_ok, f4.pack(n, (0, 0, 0, 0)), t_ok], dtype=np.uint64)
    A = ctx.build_matrix_rows_packed(p, n, G, ts, np.array([1, 1, 0, 0])).to_host()
    assert A["r"] == 3 and A["nnz"] == 6


def test_reduce_rejects_values_not_residues(f4, ctx):
    p = 65521
    rp = [0, 2, 3]
    ci = [0, 1, 1]
    say("reduce rejects a value >= p")
    A = ctx.matrix_from_csr(2, 2, rp, ci, [1, p + 3, 7])
    with pytest.raises(f4.F4Error) as e:
        ctx.reduce(p, A)
    assert e.value.code == f4.F4_E_ARG
    # the same values are residues for a larger prime
    R = ctx.reduce(2147483647, A).to_host()
    assert R["rank"] == 2
    B = ctx.matrix_from_csr(2, 2, rp, ci, [1, 3, 7])
    assert ctx.reduce(p, B).to_host()["rank"] == 2


def test_handle_of_another_context(f4, ctx):
    other = f4.Context(0)
    try:
        A = other.matrix_from_csr(1, 1, [0, 1], [0], [1])
        say("reduce with a handle of another context")
        with pytest.raises(f4.F4Error) as e:
            ctx.reduce(65521, A)
        assert e.value.code == f4.F4_E_STATE
        A.free()
    finally:
        other.close()


class HipBudget:
    """Device allocator callbacks over hipMalloc / hipFree with a byte budget;
    requests beyond it return NULL."""

    def __init__(self, budget):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipMalloc.restype = ctypes.c_int
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.hip.hipFree.restype = ctypes.c_int
        self.budget = budget
        self.live = {}
        self.calls = 0
        self.refused = 0

    def alloc(self, nbytes, stream):
        self.calls += 1
        if sum(self.live.values()) + nbytes > self.budget:
            self.refused += 1
            return 0
        ptr = ctypes.c_void_p()
        if self.hip.hipMalloc(ctypes.byref(ptr), nbytes) != 0 or not ptr.value:
            return 0
        self.live[ptr.value] = nbytes
        return ptr.value

    def free(self, ptr, stream):
        if ptr in self.live:
            del self.live[ptr]
            self.hip.hipFree(ctypes.c_void_p(ptr))


def test_nomem_through_allocator_callbacks(f4):
    # the n = 10 system: its largest step alone holds about 5 MB of CSR
    n, p, polys = synth.system("dense_n10")
    want = oracle.OracleRun(n, p, polys).basis()
    hb = HipBudget(1 << 20)  # 1 MiB: far too little for the run
    c = f4.Context(0, alloc=hb.alloc, free=hb.free)
    try:
        say("groebner with a 1 MiB device budget")
        with pytest.raises(f4.F4Error) as e:
            c.groebner(p, n, polys)
        assert e.value.code == f4.F4_E_NOMEM and hb.refused > 0
        hb.budget = 4 << 30
        say("groebner on the same context with enough memory")
        basis, _ = c.groebner(p, n, polys)
        assert [[(tuple(e), v) for e, v in f] for f in basis] == want
        assert hb.calls > 0 and hb.live
    finally:
        c.close()
    assert not hb.live, "the context returned every block through the free callback"
