"""The block schedule of the plan on the device (f4_matrix_schedule) and the
block product through its SELL-C-sigma slices (f4_spmm_sell) against O8 and
O5, exactly: perm, panel offsets, slices (start, panel, width, offsets) and
the padded storage, on the hand-worked example, random matrices with empty
rows, every step matrix of the n=6 workload, and the n=14 degree-5 Macaulay
operator; the product equal to O5 and to f4_spmm.  Every test prints its
case first."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import krylov as o5
from oracle import schedule as o8

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


def check(ctx, A, rp, ci, vv, N, W, C, sigma):
    got = ctx.schedule(A, W, C, sigma)
    want = o8.block_schedule(rp, ci, N, W, C, sigma)
    assert got["npanels"] == want["npanels"]
    for key in ("perm", "panel_ptr", "slice_start", "slice_panel", "slice_width", "slice_off"):
        assert list(map(int, got[key])) == list(want[key]), key
    cols, vals = o8.sell_storage(rp, ci, vv, want, C)
    assert list(map(int, got["sell_col"])) == cols and list(map(int, got["sell_val"])) == vals
    return got


def check_product(ctx, A, rp, ci, vv, N, p, b, seed):
    X = np.random.default_rng(seed).integers(0, p, size=(N, b))
    Xd = ctx.to_device(X)
    Y = ctx.spmm_sell(p, A, Xd)
    Y2 = ctx.spmm(p, A, Xd)
    want = o5.spmm(rp, ci, vv, N, X, p)
    assert np.array_equal(Y.to_host().reshape(-1, b).astype(np.int64), want)
    assert np.array_equal(Y.to_host(), Y2.to_host())
    for d in (Xd, Y, Y2):
        d.free()


def test_hand_example(f4, ctx):
    from test_oracle_schedule import load_golden
    rp, ci, vv, want = load_golden()
    say("block schedule, hand-worked example")
    A = ctx.matrix_from_csr(len(rp) - 1, 10, rp, ci, vv)
    got = check(ctx, A, rp, ci, vv, 10, 4, 2, 2)
    assert list(map(int, got["perm"])) == want["perm"]
    check_product(ctx, A, rp, ci, vv, 10, 65521, 3, 1)
    A.free()


@pytest.mark.parametrize("r,N,W,C,sigma,seed", [(300, 200, 16, 64, 64, 1), (1000, 50, 7, 32, 100, 2),
                                                (77, 500, 1000, 5, 3, 3), (2048, 4096, 256, 64, 1, 4)])
def test_random(f4, ctx, r, N, W, C, sigma, seed):
    from test_oracle_schedule import random_csr
    rp, ci, vv = random_csr(r, N, seed)
    say("block schedule, random", r, N, W, C, sigma)
    A = ctx.matrix_from_csr(r, N, rp, ci, vv)
    check(ctx, A, rp, ci, vv, N, W, C, sigma)
    for b in (1, 2, 5, 8):
        check_product(ctx, A, rp, ci, vv, N, 2147483647, b, seed + b)
    # an even b with X and Y at odd word offsets (one word per lane)
    X = np.random.default_rng(seed).integers(0, 65521, size=(N, 4))
    Xb = ctx.to_device(np.concatenate([[7], X.ravel()]))
    Yb = ctx.device_array(r * 4 + 1)
    Y = ctx.spmm_sell(65521, A, Xb.sub(1, (N, 4)), out=Yb.sub(1, (r, 4)))
    assert np.array_equal(Y.to_host().astype(np.int64), o5.spmm(rp, ci, vv, N, X, 65521))
    Xb.free()
    Yb.free()
    A.free()


def test_every_step_of_n6(f4, ctx):
    n, p, polys = synth.system("dense_n6")
    run = oracle.OracleRun(n, p, polys, record=-2)
    for k in range(len(run.steps())):
        rec = run.step_record(k)
        say("block schedule, n=6 step", k)
        A = ctx.build_matrix(p, n, rec["G"], rec["active"], rec["sel"])
        h = A.to_host()
        rp, ci, vv = [list(map(int, h[x])) for x in ("row_ptr", "col_ind", "val")]
        check(ctx, A, rp, ci, vv, h["N"], 32, 64, 128)
        check_product(ctx, A, rp, ci, vv, h["N"], p, 4, k)
        A.free()


def test_macaulay_n14(f4, ctx):
    n, p, polys = synth.system("sparse_n14")
    G = f4.normalize(p, n, polys)
    t = f4.pack_many(n, synth.monomials_upto(n, 3))
    A = ctx.build_matrix_rows_packed(p, n, G, np.repeat(t, len(G)), np.tile(np.arange(len(G), dtype=np.uint32), len(t)))
    h = A.to_host()
    rp, ci, vv = [list(map(int, h[x])) for x in ("row_ptr", "col_ind", "val")]
    say("block schedule, n=14 degree-5 Macaulay rows", h["r"], h["N"], h["nnz"])
    check(ctx, A, rp, ci, vv, h["N"], 512, 64, 256)
    check_product(ctx, A, rp, ci, vv, h["N"], p, 8, 9)
    A.free()


def test_errors(f4, ctx):
    A = ctx.matrix_from_csr(2, 3, [0, 1, 2], [0, 2], [1, 1])
    X = ctx.to_device(np.ones((3, 1), dtype=np.int64))
    say("block schedule errors")
    with pytest.raises(f4.F4Error) as e:
        ctx.spmm_sell(65521, A, X)
    assert e.value.code == f4.F4_E_STATE
    with pytest.raises(f4.F4Error) as e:
        ctx.schedule(A, 4, 65, 2)
    assert e.value.code == f4.F4_E_ARG
    X.free()
    A.free()
