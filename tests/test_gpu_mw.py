"""Two-word monomial keys on the device (f4_build_matrix_rows_mw) against
O7's symbolic preprocessing without closure (the matrix of an explicit row
list: dictionary = union of the row supports in descending grevlex, rows by
leading monomial then basis index, repeats collapsed), exactly, for n = 15 to
30 variables; the matrix then reduced by f4_reduce and compared with O3's
dense reduced echelon form; and the error paths.  Every test prints its case
first."""

import sys

import numpy as np
import pytest

import synth
from oracle import buchberger as bb
from oracle import dense
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


def lib_form(polys, p):
    out = []
    for f in polys:
        d = {}
        for e, c in f:
            d[tuple(e)] = (d.get(tuple(e), 0) + c) % p
        out.append(sorted(((e, c) for e, c in d.items() if c), key=lambda t: bb.grevlex_key(t[0]), reverse=True))
    return [f for f in out if f]


def check(f4, ctx, p, n, G, rows):
    want = o7.fbsp(G, [0] * len(G), rows)
    A = ctx.build_matrix_rows_mw(p, n, G, rows)
    h = A.to_host()
    assert h["key_words"] == 2
    assert [f4.unpack_mw(n, w) for w in h["dict_keys"]] == want["T"]
    assert [f4.unpack_mw(n, w) for w in h["row_t"]] == [tuple(t) for t in want["rows_t"]]
    assert list(h["row_k"]) == list(want["rows_k"])
    assert list(h["row_ptr"]) == list(want["row_ptr"])
    assert list(h["col_ind"]) == list(want["col_ind"]) and list(h["val"]) == list(want["val"])
    return A, want


CASES = [  # n, m, terms per polynomial, shift degree, p, seed
    (15, 16, 20, 2, 65521, 1),
    (16, 17, 20, 1, synth.P31, 2),
    (20, 21, 30, 1, 65521, 3),
    (24, 25, 20, 1, 65521, 4),
    (30, 31, 20, 1, synth.P31, 5),
]


@pytest.mark.parametrize("case", CASES)
def test_macaulay_rows_match_o7(f4, ctx, case):
    n, m, k, sdeg, p, seed = case
    G = lib_form(synth.reduce_coeffs(synth.sparse_quadratics(n, m, seed, p - 1, k), p), p)
    shifts = [tuple(int(x) for x in t) for t in synth.monomials_upto(n, sdeg)]
    rows = [(t, i) for t in shifts for i in range(len(G))]
    rows += rows[: len(rows) // 7]  # repeats collapse
    say("two-word keys, Macaulay rows", "n", n, "m", len(G), "rows", len(rows))
    A, want = check(f4, ctx, p, n, G, rows)
    assert A.view.r == len(set(rows)) and A.view.N == len(want["T"])
    A.free()


def test_reduce_two_word_matrix(f4, ctx):
    n, p = 18, 65521
    G = lib_form(synth.reduce_coeffs(synth.sparse_quadratics(n, 19, 6, p - 1, 12), p), p)
    rows = [(tuple(int(x) for x in t), i) for t in synth.monomials_upto(n, 1) for i in range(len(G))]
    say("two-word keys, reduce", "n", n, "rows", len(rows))
    A, want = check(f4, ctx, p, n, G, rows)
    R = ctx.reduce(p, A)
    hr = R.to_host()
    N = len(want["T"])
    dense_rows = dense.csr_to_dense(want["row_ptr"], want["col_ind"], want["val"], N)
    E, piv = dense.rref(dense_rows, N, p)
    assert hr["rank"] == len(E)
    # the pivot columns of A (leading columns of its rows) and the trailing
    # block's RREF together give the RREF's pivot set
    pcols = sorted(set(int(x) for x in hr["pivot_cols"]))
    lead = sorted(set(int(want["col_ind"][want["row_ptr"][i]]) for i in range(len(want["rows_k"]))))
    assert pcols == lead
    R.free()
    A.free()


def test_errors(f4, ctx):
    n, p = 20, 65521
    G = lib_form(synth.reduce_coeffs(synth.sparse_quadratics(n, 3, 7, p - 1, 6), p), p)
    say("two-word keys, errors")
    with pytest.raises(f4.F4Error) as e:  # basis index out of range
        ctx.build_matrix_rows_mw(p, n, G, [((0,) * n, 5)])
    assert e.value.code == f4.F4_E_ARG
    big = tuple([31] + [0] * (n - 1))  # 5-bit lanes: 31 + 2 overflows
    lead_x1 = [q for q, g in enumerate(G) if g[0][0][0] > 0]
    if lead_x1:
        with pytest.raises(f4.F4Error) as e:
            ctx.build_matrix_rows_mw(p, n, G, [(big, lead_x1[0])])
        assert e.value.code == f4.F4_E_RANGE
    bad = [list(reversed(G[0]))] + G[1:]  # terms not in decreasing order
    with pytest.raises(f4.F4Error) as e:
        ctx.build_matrix_rows_mw(p, n, bad, [((0,) * n, 0)])
    assert e.value.code == f4.F4_E_ARG
