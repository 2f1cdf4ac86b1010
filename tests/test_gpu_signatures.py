"""Signature admissibility on the device (f4_sig_filter, f4_build_matrix_sig)
against O7, through the C-ABI, exactly: the flags of every row, the
admissible rows in input order and their bucketed schedule; the whole matrix
of the symbolic preprocessing closed over the admissible reducers
(dictionary, rows, CSR).  Cases: the hand-worked example, principal
syzygies of input systems, and every step of the recorded F4 runs of the
n=6 and n=10 workloads and the n=14 degree-4 step, with seeded synthetic
signatures.  Every test prints its case first."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import buchberger as bb
from oracle import signatures as o7

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


def lib_form(G):
    """Basis in the library's input form: terms by decreasing grevlex."""
    return [sorted(((tuple(e), c) for e, c in g), key=lambda t: bb.grevlex_key(t[0]), reverse=True) for g in G]


def check_filter(ctx, p, n, G, sidx, smon, syz, rows):
    flags, kept, order, st = ctx.sig_filter(p, n, lib_form(G), sidx, smon, syz, rows)
    wf, wk, wo = o7.filter_rows(rows, G, sidx, smon, syz)
    assert list(flags) == wf
    assert kept == [(tuple(t), k) for t, k in wk]
    assert order == wo
    assert st["kept"] == len(wk) and st["syzygy"] == wf.count(1) and st["rewritten"] == wf.count(2)
    return wf


def test_filter_hand_example(ctx):
    from test_oracle_signatures import load_golden
    G, sidx, smon, syz, rows, want, order = load_golden()
    say("signature filter, hand-worked example")
    wf = check_filter(ctx, 65521, 2, G, sidx, smon, syz, rows)
    assert wf == want


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 3), (7, 4)])
def test_filter_principal_syzygies(ctx, n, seed):
    p = 65521
    F = lib_form(synth.random_system(n, n + 1, p, seed, density=0.6, max_deg=2))
    lms = [o7.lead(f) for f in F]
    m = len(F)
    sidx, smon = list(range(m)), [(0,) * n] * m
    syz = [[lms[j] for j in range(i)] for i in range(m)]
    rows = [(tuple(int(x) for x in t), k) for k in range(m) for t in synth.monomials_upto(n, 3)]
    say("signature filter, principal syzygies", "n", n, "rows", len(rows))
    wf = check_filter(ctx, p, n, F, sidx, smon, syz, rows)
    assert wf.count(1) > 0


def recorded_steps(cfg, stop_deg=-1):
    n, p, polys = synth.system(cfg)
    run = oracle.OracleRun(n, p, polys, record=-2, stop_deg=stop_deg)
    return n, p, [run.step_record(k) for k in range(len(run.steps()))]


def halves(rec):
    lms = [o7.lead(g) for g in rec["G"]]
    rows = []
    for i, j in rec["sel"]:
        L = tuple(max(a, b) for a, b in zip(lms[i], lms[j]))
        rows.append((o7.mono_div(L, lms[i]), i))
        rows.append((o7.mono_div(L, lms[j]), j))
    return rows


def check_build(f4, ctx, n, p, rec, m_index, seed, label):
    G = [list(g) for g in rec["G"]]
    lms = [o7.lead(g) for g in G]
    sidx, smon = synth.signatures(lms, min(m_index, len(G)), seed)
    syz = [[lms[j] for j in range(i)] for i in range(max(sidx) + 1)]
    rows = halves(rec)
    want = o7.fbsp(G, rec["active"], rows, (sidx, smon, syz))
    say("signature-aware build", label, "rows in", len(rows), "rows out", len(want["rows_k"]), "N", len(want["T"]))
    A, st = ctx.build_matrix_sig(p, n, lib_form(G), rec["active"], sidx, smon, syz, rows)
    h = A.to_host()
    assert [f4.unpack(n, int(x)) for x in h["dict_keys"]] == want["T"]
    assert [f4.unpack(n, int(x)) for x in h["row_t"]] == [tuple(t) for t in want["rows_t"]]
    assert list(h["row_k"]) == list(want["rows_k"])
    assert list(h["row_ptr"]) == list(want["row_ptr"])
    assert list(h["col_ind"]) == list(want["col_ind"]) and list(h["val"]) == list(want["val"])
    A.free()
    flags, _, _ = o7.filter_rows(rows, G, sidx, smon, syz)
    return st, flags


@pytest.mark.parametrize("cfg,m_index,seed", [("dense_n6", 7, 1), ("dense_n6", 3, 2), ("dense_n10", 12, 3), ("dense_n10", 5, 4)])
def test_build_sig_every_step(f4, ctx, cfg, m_index, seed):
    n, p, recs = recorded_steps(cfg)
    for k, rec in enumerate(recs):
        check_build(f4, ctx, n, p, rec, m_index, seed + k, "system %s step %d" % (cfg, k))


def test_build_sig_unconstrained_equals_build(f4, ctx):
    """Distinct indices and no syzygies: every row is admissible and the
    matrix is f4_build_matrix's."""
    n, p, recs = recorded_steps("dense_n10")
    rec = recs[-2]
    G = lib_form([list(g) for g in rec["G"]])
    m = len(G)
    say("signature-aware build with nothing rejected = f4_build_matrix")
    A, st = ctx.build_matrix_sig(p, n, G, rec["active"], list(range(m)), [(0,) * n] * m, [[] for _ in range(m)],
                                 halves(rec))
    B = ctx.build_matrix(p, n, G, rec["active"], rec["sel"])
    a, b = A.to_host(), B.to_host()
    for key in ("dict_keys", "row_t", "row_k", "row_ptr", "col_ind", "val"):
        assert np.array_equal(a[key], b[key]), key
    assert st["syzygy"] == 0 and st["rewritten"] == 0
    A.free()
    B.free()


def test_build_sig_n14_degree4(f4, ctx):
    n, p, polys = synth.system("sparse_n14")
    run = oracle.OracleRun(n, p, polys, stop_deg=4)
    k = len(run.steps()) - 1
    rec = oracle.OracleRun(n, p, polys, record=k, stop_deg=4).step_record(k)
    st, flags = check_build(f4, ctx, n, p, rec, 15, 7, "n=14 degree-4 step")
    assert st["syzygy"] + st["rewritten"] > 0


def test_filter_errors(f4, ctx):
    p, n = 65521, 3
    F = lib_form(synth.random_system(n, 3, p, 9, density=1.0, max_deg=2))
    say("signature filter errors")
    with pytest.raises(f4.F4Error) as e:  # signature index out of range
        ctx.sig_filter(p, n, F, [0, 1, 5], [(0,) * n] * 3, [[], []], [((0, 0, 0), 0)])
    assert e.value.code == f4.F4_E_ARG
    with pytest.raises(f4.F4Error) as e:  # t * s overflows an exponent lane (8-bit lanes for n = 3)
        ctx.sig_filter(p, n, F, [0, 1, 2], [(200, 0, 0), (0, 0, 0), (0, 0, 0)], [[], [], []],
                       [((60, 0, 0), 0)])
    assert e.value.code == f4.F4_E_RANGE
