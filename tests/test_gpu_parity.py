"""Parity of the HIP path with the CPU oracle, element by element.

Every test prints the case it runs before the device call.  All comparisons
are exact (arithmetic is exact mod p): the tolerance is zero.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import buchberger as bb
from oracle import dense

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


@pytest.fixture(scope="module")
def ctx_radix(f4):
    c = f4.Context(0, dict_path="radix")
    yield c
    c.close()


def canon(basis):
    out = []
    for f in basis:
        d = {tuple(e): c for e, c in f}
        out.append(tuple((e, d[e]) for e in sorted(d, key=bb.grevlex_key, reverse=True)))
    return tuple(out)


def check_build(f4, ctx, n, p, rec, label):
    say("build", label, "rows", len(rec["rows_k"]), "N", len(rec["T"]), "M", len(rec["col_ind"]))
    A = ctx.build_matrix(p, n, rec["G"], rec["active"], rec["sel"])
    h = A.to_host()
    assert h["r"] == len(rec["rows_k"]) and h["N"] == len(rec["T"]) and h["nnz"] == len(rec["col_ind"])
    assert [f4.unpack(n, int(x)) for x in h["dict_keys"]] == rec["T"]
    assert [f4.unpack(n, int(x)) for x in h["row_t"]] == rec["rows_t"]
    assert h["row_k"].tolist() == rec["rows_k"]
    assert h["row_ptr"].tolist() == rec["row_ptr"]
    assert np.array_equal(h["col_ind"], np.array(rec["col_ind"], dtype=np.uint32))
    assert np.array_equal(h["val"], np.array(rec["val"], dtype=np.uint32))
    return A


def check_reduce(ctx, p, A, rec, label):
    say("reduce", label)
    R = ctx.reduce(p, A).to_host()
    assert R["pivot_cols"].tolist() == rec["pivot_cols"]
    assert R["row_ptr"].tolist() == rec["rref_ptr"]
    assert np.array_equal(R["col_ind"], np.array(rec["rref_col"], dtype=np.uint32))
    assert np.array_equal(R["val"], np.array(rec["rref_val"], dtype=np.uint32))
    assert R["rank"] == len(rec["pivot_cols"]) + len(rec["rref_ptr"]) - 1


def run_steps(f4, ctx, n, p, polys, label, stop_deg=-1, only=None):
    run = oracle.OracleRun(n, p, polys, record=-2 if only is None else only, stop_deg=stop_deg)
    steps = run.steps()
    ks = range(len(steps)) if only is None else [only]
    for k in ks:
        rec = run.step_record(k)
        A = check_build(f4, ctx, n, p, rec, "%s step %d (d=%d)" % (label, k, rec["d"]))
        check_reduce(ctx, p, A, rec, "%s step %d" % (label, k))
        A.free()
    return run


# ----------------------------------------------------------- step parity
def test_steps_dense_n6(f4, ctx):
    n, p, polys = synth.system("dense_n6")
    run_steps(f4, ctx, n, p, polys, "dense_n6")


def test_steps_dense_n6_radix_dictionary(f4, ctx_radix):
    n, p, polys = synth.system("dense_n6")
    run_steps(f4, ctx_radix, n, p, polys, "dense_n6/radix")


def test_steps_dense_n10(f4, ctx):
    n, p, polys = synth.system("dense_n10")
    run_steps(f4, ctx, n, p, polys, "dense_n10")


def test_steps_dense_n10_radix_dictionary_large_steps(f4, ctx_radix):
    n, p, polys = synth.system("dense_n10")
    run = oracle.OracleRun(n, p, polys, record=4)
    rec = run.step_record(4)
    A = check_build(f4, ctx_radix, n, p, rec, "dense_n10 step 4 radix")
    check_reduce(ctx_radix, p, A, rec, "dense_n10 step 4 radix")


@pytest.mark.parametrize("n,p,seed", [(3, 7, 1), (4, 31, 2), (5, 65521, 3), (4, 2147483647, 4),
                                      (6, 2147483629, 5)])
def test_steps_planted(f4, ctx, n, p, seed):
    polys, _ = synth.planted_system(n, n + 1, p, seed)
    run_steps(f4, ctx, n, p, polys, "planted n=%d p=%d" % (n, p))


def test_steps_sparse_p31(f4, ctx):
    polys = synth.sparse_quadratics(8, 9, 77, synth.P31 - 1, 12)
    run_steps(f4, ctx, 8, synth.P31, polys, "sparse n=8 p31")


def test_step_sparse_n14_degree5_full_size(f4, ctx):
    # the single degree-5 step of the sparse n=14 system over F_(2^31-1)
    n, p, polys = synth.system("sparse_n14")
    say("oracle sparse_n14 up to d=5 (about 20 s)")
    run = oracle.OracleRun(n, p, polys, record=3, stop_deg=5)
    rec = run.step_record(3)
    assert rec["d"] == 5
    A = check_build(f4, ctx, n, p, rec, "sparse_n14 d=5")
    check_reduce(ctx, p, A, rec, "sparse_n14 d=5")


# --------------------------------------------------- reduce on given matrices
def random_csr(r, N, p, density, seed):
    rng = synth.SplitMix64(seed)
    rows = []
    for _ in range(r):
        row = [(c, 1 + rng.below(p - 1)) for c in range(N) if rng.uniform01() < density]
        rows.append(row)
    rp, ci, vv = [0], [], []
    for row in rows:
        for c, v in row:
            ci.append(c)
            vv.append(v)
        rp.append(len(ci))
    return rp, ci, vv


@pytest.mark.parametrize("r,N,p,density,seed", [
    (40, 30, 65521, 0.2, 1), (70, 150, 65521, 0.08, 2), (90, 200, 2147483647, 0.06, 3),
    (130, 70, 7, 0.3, 4), (200, 300, 65521, 0.02, 5), (3, 5, 31, 0.9, 6), (1, 1, 31, 1.0, 7),
    (64, 64, 65521, 0.5, 8), (150, 520, 2147483629, 0.03, 9),
    # more than 1 024 trailing columns: the echelon's tiled update on the fp64
    # matrix cores (one tile per 32 rows x 256 columns, a ragged last tile),
    # for the small-prime and the large-prime instance
    (60, 1300, 65521, 0.05, 10), (60, 1250, 2147483647, 0.05, 11)])
def test_reduce_random_matrices_vs_dense_rref(f4, ctx, r, N, p, density, seed):
    rp, ci, vv = random_csr(r, N, p, density, seed)
    say("reduce random", r, N, p, density, "nnz", len(ci))
    A = ctx.matrix_from_csr(r, N, rp, ci, vv)
    R = ctx.reduce(p, A).to_host()
    Ad = dense.csr_to_dense(rp, ci, vv, N)
    full, pc = dense.rref(Ad, N, p)
    leads = sorted({ci[rp[i]] for i in range(r) if rp[i + 1] > rp[i]})
    assert R["pivot_cols"].tolist() == leads
    want = [row for row, c in zip(full, pc) if c not in set(leads)]
    got = dense.csr_to_dense(R["row_ptr"].tolist(), R["col_ind"].tolist(), R["val"].tolist(), N)
    assert got == want
    assert R["rank"] == len(full)


def test_reduce_edge_cases(f4, ctx):
    p = 65521
    say("reduce: all rows pivots")
    A = ctx.matrix_from_csr(3, 4, [0, 2, 3, 4], [0, 3, 1, 2], [5, 6, 7, 8])
    R = ctx.reduce(p, A).to_host()
    assert R["rho"] == 0 and R["pivot_cols"].tolist() == [0, 1, 2] and R["rank"] == 3
    say("reduce: duplicate rows reduce to zero")
    A = ctx.matrix_from_csr(3, 3, [0, 2, 4, 6], [0, 2, 0, 2, 0, 2], [1, 2, 3, 6, 5, 10])
    R = ctx.reduce(p, A).to_host()
    assert R["rho"] == 0 and R["rank"] == 1
    say("reduce: empty rows")
    A = ctx.matrix_from_csr(3, 3, [0, 0, 1, 1], [1], [9])
    R = ctx.reduce(p, A).to_host()
    assert R["rho"] == 0 and R["rank"] == 1
    say("reduce: trailing block of full rank across several panels")
    # 70 pivot rows x 2 each, 130 lower rows: exercises partial last panel
    rp, ci, vv = random_csr(200, 140, p, 0.25, 11)
    A = ctx.matrix_from_csr(200, 140, rp, ci, vv)
    R = ctx.reduce(p, A).to_host()
    full, pc = dense.rref(dense.csr_to_dense(rp, ci, vv, 140), 140, p)
    assert R["rank"] == len(full)


# ------------------------------------------------------------- rows, no closure
def test_build_rows_matrix_correctness(f4, ctx):
    # Theorem "Matrix materialization correctness" on explicit rows
    n, p = 5, 65521
    G = [bb.as_sorted_terms(bb.monic(bb.from_terms(f, p), p)) for f in synth.random_system(n, 4, p, 21, 0.5)]
    rows = [((1, 0, 0, 0, 0), 0), ((0, 0, 0, 0, 0), 1), ((0, 1, 1, 0, 0), 2), ((0, 0, 0, 0, 2), 3),
            ((1, 0, 0, 0, 0), 0), ((0, 0, 1, 0, 0), 3)]
    say("build_rows n=5")
    h = ctx.build_matrix_rows(p, n, G, rows).to_host()
    T = [f4.unpack(n, int(x)) for x in h["dict_keys"]]
    keys = [bb.grevlex_key(e) for e in T]
    assert all(keys[i] > keys[i + 1] for i in range(len(T) - 1))
    uniq = set(rows)
    assert h["r"] == len(uniq)
    supp = set()
    for t, k in uniq:
        for e, _ in G[k]:
            supp.add(tuple(a + b for a, b in zip(t, e)))
    assert set(T) == supp
    for i in range(h["r"]):
        t = f4.unpack(n, int(h["row_t"][i]))
        k = int(h["row_k"][i])
        got = {T[h["col_ind"][q]]: int(h["val"][q]) for q in range(h["row_ptr"][i], h["row_ptr"][i + 1])}
        assert got == {tuple(a + b for a, b in zip(t, e)): c for e, c in G[k]}


# ------------------------------------------------------------ full F4
def shapes_of(steps):
    return [(s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"], s["rho"]) for s in steps]


def oracle_shapes(run):
    return [(s["d"], s["r"], s["N"], s["M"], s["npiv"], s["rank"], s["rho"]) for s in run.steps()]


@pytest.mark.parametrize("cfg", ["dense_n6", "dense_n10"])
def test_groebner_configs(f4, ctx, cfg):
    n, p, polys = synth.system(cfg)
    say("groebner cfg", cfg)
    B, steps = ctx.groebner(p, n, polys)
    run = oracle.OracleRun(n, p, polys)
    assert canon(B) == canon(run.basis())
    assert shapes_of(steps) == oracle_shapes(run)


@pytest.mark.parametrize("n,p,seed", [(3, 31, 1), (4, 65521, 2), (5, 65521, 3), (4, 2147483647, 4),
                                      (6, 2147483543, 6)])
def test_groebner_planted(f4, ctx, n, p, seed):
    polys, s = synth.planted_system(n, n + 1, p, seed)
    say("groebner planted", n, p)
    B, steps = ctx.groebner(p, n, polys)
    run = oracle.OracleRun(n, p, polys)
    assert canon(B) == canon(run.basis())
    assert shapes_of(steps) == oracle_shapes(run)
    assert len(B) == n  # linear basis x_i - s_i


@pytest.mark.parametrize("n,p,seed", [(3, 65521, 2), (4, 65521, 3), (4, 31, 5), (5, 2147483647, 7)])
def test_groebner_square_nontrivial(f4, ctx, n, p, seed):
    polys = synth.random_system(n, n, p, seed)
    say("groebner square", n, p)
    B, steps = ctx.groebner(p, n, polys)
    run = oracle.OracleRun(n, p, polys)
    assert canon(B) == canon(run.basis())
    assert shapes_of(steps) == oracle_shapes(run)


def test_groebner_tiny_vs_buchberger(f4, ctx):
    for (n, m, p, seed, dens) in [(2, 2, 7, 1, 1.0), (3, 3, 31, 3, 0.6), (3, 4, 65521, 5, 0.5), (4, 3, 31, 7, 0.35)]:
        polys = synth.random_system(n, m, p, seed, density=dens)
        say("groebner tiny", n, m, p, seed)
        B, _ = ctx.groebner(p, n, polys)
        want = canon([bb.as_sorted_terms(f) for f in bb.groebner(n, p, polys)])
        assert canon(B) == want


def test_groebner_degenerate_inputs(f4, ctx):
    p = 65521
    say("groebner: zero polynomials only")
    B, _ = ctx.groebner(p, 3, [[((1, 0, 0), p)], []])
    assert B == []
    say("groebner: a constant")
    B, _ = ctx.groebner(p, 3, [[((1, 1, 0), 3)], [((0, 0, 0), 5)]])
    assert B == [[((0, 0, 0), 1)]]
    say("groebner: single polynomial")
    B, steps = ctx.groebner(p, 3, [[((2, 0, 0), 2), ((0, 1, 1), 4), ((0, 0, 0), 6)]])
    assert steps == [] and B == [[((2, 0, 0), 1), ((0, 1, 1), 2), ((0, 0, 0), 3)]]


def test_crt_primes_same_system(f4, ctx):
    n, polys = synth.crt_system()
    for p in synth.CRT_PRIMES[:2]:
        sysp = synth.reduce_coeffs(polys, p)
        say("crt prime", p)
        B, steps = ctx.groebner(p, n, sysp)
        run = oracle.OracleRun(n, p, sysp)
        assert canon(B) == canon(run.basis())
        assert shapes_of(steps) == oracle_shapes(run)


def test_determinism_repeated_runs(f4, ctx):
    n, p, polys = synth.system("dense_n10")
    run = oracle.OracleRun(n, p, polys, record=3)
    rec = run.step_record(3)
    say("determinism dense_n10 step 3 x3")
    outs = []
    for _ in range(3):
        A = ctx.build_matrix(p, n, rec["G"], rec["active"], rec["sel"])
        h = A.to_host()
        R = ctx.reduce(p, A).to_host()
        outs.append((h["col_ind"].tobytes(), h["val"].tobytes(), R["col_ind"].tobytes(), R["val"].tobytes()))
    assert outs[0] == outs[1] == outs[2]


@pytest.mark.gpu
def test_stop_degree_keeps_leading_steps(f4):
    """A context with a stop degree runs the same steps as a full run up to
    and including the first step of that degree, then stops (empty basis)."""
    n, p, polys = synth.system("dense_n6")
    full = f4.Context(0)
    B, steps = full.groebner(p, n, polys)
    full.close()
    stop = f4.Context(0, stop_deg=3)
    B3, steps3 = stop.groebner(p, n, polys)
    stop.close()
    first3 = next(i for i, s in enumerate(steps) if s["deg"] == 3)
    key = lambda s: (s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"], s["rho"])
    assert [key(s) for s in steps3] == [key(s) for s in steps[:first3 + 1]]
    assert B3 == []
