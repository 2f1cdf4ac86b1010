"""Block Wiedemann on the device (f4_bw_sequence, f4_bw_mbasis,
f4_block_wiedemann) against O6, through the C-ABI: the projected Krylov
sequence and the sigma-basis (P and shifts) bit for bit, the kernel vectors
bit for bit (same generators, same evaluation) and checked as syzygies
(v^T A = 0, and on Macaulay matrices the polynomial identity of Proposition
"Kernel equals syzygies under dictionary closure"); at the size of the
degree-4 step of the n=14 workload, where the oracle's sigma-basis is too
slow, the vectors are checked by v^T A = 0 with O5 and by their rank.
Every test prints its case first."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import krylov as o5
from oracle import wiedemann as w6

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import paper_2601_06765_amd.f4 as f4
    c = f4.Context(0)
    yield f4, c
    c.close()


def rank_mod(M, p):
    M = [[int(x) % p for x in row] for row in M]
    rk = 0
    ncols = len(M[0]) if M else 0
    for col in range(ncols):
        piv = next((i for i in range(rk, len(M)) if M[i][col]), None)
        if piv is None:
            continue
        M[rk], M[piv] = M[piv], M[rk]
        inv = pow(M[rk][col], p - 2, p)
        M[rk] = [x * inv % p for x in M[rk]]
        for i in range(len(M)):
            if i != rk and M[i][col]:
                f = M[i][col]
                M[i] = [(x - f * y) % p for x, y in zip(M[i], M[rk])]
        rk += 1
    return rk


def planted_csr(r0, ncols, k, p, seed, maxlen=8, zero_rows=0):
    """r0 sparse random independent rows, k random combinations of them and
    zero_rows empty rows, shuffled (left kernel of dimension k + zero_rows)."""
    rng = np.random.default_rng(seed)
    rows = []
    while len(rows) < r0:
        idx = rng.choice(ncols, size=int(rng.integers(2, maxlen + 1)), replace=False)
        row = [0] * ncols
        for j in idx:
            row[int(j)] = int(rng.integers(1, p))
        if rank_mod(rows + [row], p) == len(rows) + 1:
            rows.append(row)
    for _ in range(k):
        c = [int(x) for x in rng.integers(0, p, size=r0)]
        rows.append([sum(ci * row[j] for ci, row in zip(c, rows[:r0])) % p for j in range(ncols)])
    rows += [[0] * ncols for _ in range(zero_rows)]
    order = rng.permutation(len(rows))
    rows = [rows[i] for i in order]
    rp, ci, vv = [0], [], []
    for row in rows:
        for j, v in enumerate(row):
            if v:
                ci.append(j)
                vv.append(v)
        rp.append(len(ci))
    return rp, ci, vv


def inputs(r, ncols, b, p, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(1, p, size=ncols), rng.integers(0, p, size=(r, b)), rng.integers(0, p, size=(r, b)))


def dev(c, d, X, Y):
    return c.to_device(d), c.to_device(X), c.to_device(Y)


CASES = [  # p, b, r0, ncols, k, zero rows, seed
    (65521, 4, 30, 44, 3, 0, 1),
    (synth.P31, 3, 26, 40, 2, 1, 2),
    (synth.P31, 1, 18, 25, 1, 0, 3),
    (65521, 8, 40, 60, 5, 0, 4),
    (7, 2, 10, 16, 2, 0, 5),
    (2147483629, 5, 33, 50, 4, 2, 6),
    (65521, 16, 36, 70, 6, 0, 7),
]


@pytest.mark.parametrize("case", CASES)
def test_sequence_mbasis_and_vectors_match_o6(env, case):
    f4, c = env
    p, b, r0, ncols, k, z, seed = case
    rp, ci, vv = planted_csr(r0, ncols, k, p, seed, zero_rows=z)
    r = len(rp) - 1
    d, X, Y = inputs(r, ncols, b, p, seed + 100)
    say("block Wiedemann planted", "p", p, "b", b, "r", r, "N", ncols, "kernel", k + z)
    A = c.matrix_from_csr(r, ncols, rp, ci, vv)
    dd, Xd, Yd = dev(c, d, X, Y)
    L = w6.block_len(r, b)
    want = w6.left_kernel_block_wiedemann(rp, ci, vv, ncols, d, X, Y, p)
    S = c.bw_sequence(p, A, dd, Xd, Yd, L)
    assert np.array_equal(S, want["S"]), "Krylov sequence differs"
    P, s = c.bw_mbasis(p, b, S)
    assert s == want["shifts"], "sigma-basis shifts differ"
    assert np.array_equal(P, np.array(want["P"], dtype=np.int64)), "sigma-basis differs"
    vecs, st = c.block_wiedemann(p, A, dd, Xd, Yd)
    assert st["L"] == L and st["generators"] == len(want["gens"])
    assert len(vecs) == len(want["vectors"])
    for v, wv in zip(vecs, want["vectors"]):
        assert np.array_equal(v, wv), "kernel vector differs"
        assert not o5.spmm(rp, ci, vv, ncols, v[:, None], p, trans=True).any()
    assert rank_mod([list(v) for v in vecs], p) == min(b, k + z)
    A.free()


def test_full_row_rank_has_no_vectors(env):
    f4, c = env
    p, b = 65521, 4
    rp, ci, vv = planted_csr(20, 30, 0, p, 31)
    d, X, Y = inputs(20, 30, b, p, 32)
    say("block Wiedemann full row rank")
    A = c.matrix_from_csr(20, 30, rp, ci, vv)
    vecs, st = c.block_wiedemann(p, A, *dev(c, d, X, Y))
    want = w6.left_kernel_block_wiedemann(rp, ci, vv, 30, d, X, Y, p)
    assert vecs == [] and want["vectors"] == []
    A.free()


def mono_mul(a, b):
    return tuple(x + y for x, y in zip(a, b))


@pytest.mark.parametrize("n,p,seed,b", [(4, 65521, 21, 4), (5, synth.P31, 23, 8)])
def test_macaulay_syzygies(env, n, p, seed, b):
    f4, c = env
    polys, _ = synth.planted_system(n, n + 1, p, seed)
    run = oracle.OracleRun(n, p, polys, record=-2)
    tested = 0
    for k in range(len(run.steps())):
        rec = run.step_record(k)
        rp = [int(x) for x in rec["row_ptr"]]
        ci = [int(x) for x in rec["col_ind"]]
        vv = [int(x) for x in rec["val"]]
        r, N = len(rp) - 1, len(rec["T"])
        kdim = r - (len(rec["pivot_cols"]) + len(rec["rref_ptr"]) - 1)
        if kdim == 0 or r > 150:
            continue
        d, X, Y = inputs(r, N, b, p, seed + k)
        say("block Wiedemann Macaulay step", k, "n", n, "r", r, "N", N, "kernel dim", kdim)
        A = c.matrix_from_csr(r, N, rp, ci, vv)
        vecs, _ = c.block_wiedemann(p, A, *dev(c, d, X, Y))
        want = w6.left_kernel_block_wiedemann(rp, ci, vv, N, d, X, Y, p)
        assert len(vecs) == len(want["vectors"]) and all(np.array_equal(a, w) for a, w in zip(vecs, want["vectors"]))
        assert rank_mod([list(v) for v in vecs], p) == min(b, kdim)
        for v in vecs:
            acc = {}
            for vi, t, kk in zip(v, rec["rows_t"], rec["rows_k"]):
                if vi:
                    for e, cf in rec["G"][kk]:
                        m = mono_mul(t, e)
                        acc[m] = (acc.get(m, 0) + int(vi) * cf) % p
            assert all(x == 0 for x in acc.values())
        A.free()
        tested += 1
    assert tested >= 1


def test_large_macaulay_step(env):
    """The first degree-4 step of the n=14 sparse system over F_(2^31-1)
    (r = 1 522, N = 2 734, 303 895 nonzeros, rank 1 377), its matrix built by
    the device's symbolic preprocessing from the oracle's recorded selection:
    b = 8 vectors, checked by v^T A = 0 (O5) and by their rank (min(b, r - rank))."""
    f4, c = env
    n, p, polys = synth.system("sparse_n14")
    run = oracle.OracleRun(n, p, polys, stop_deg=4)
    k = len(run.steps()) - 1
    st = run.steps()[k]
    assert st["d"] == 4
    rec = oracle.OracleRun(n, p, polys, record=k, stop_deg=4).step_record(k)
    A = c.build_matrix(p, n, rec["G"], rec["active"], rec["sel"])
    h = A.to_host()
    r, N = A.view.r, A.view.N
    assert (r, N) == (st["r"], st["N"])
    b = 8
    d, X, Y = inputs(r, N, b, p, 77)
    say("block Wiedemann n=14 degree-4 step", "r", r, "N", N, "kernel dim", r - st["rank"], "b", b)
    vecs, stats = c.block_wiedemann(p, A, *dev(c, d, X, Y))
    say("found", len(vecs), "vectors", stats)
    assert vecs
    rp, ci, vv = h["row_ptr"], h["col_ind"], h["val"]
    for v in vecs:
        assert not o5.spmm(rp, ci, vv, N, v[:, None], p, trans=True).any()
    assert rank_mod([list(v) for v in vecs], p) == min(b, r - st["rank"])
    A.free()
