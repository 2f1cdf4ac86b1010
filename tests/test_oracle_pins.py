"""Pins of the CPU oracle against facts it does not compute itself.

* the reduced Groebner basis is unique, so O1 (textbook F4, C++), O2
  (Buchberger, Python) and sympy's independent `groebner` must agree exactly;
* closed forms: random m = n+1 quadratics have no common zero (basis {1}); a
  planted root gives the linear basis {x_i - s_i}; n generic quadratics in n
  variables have exactly 2^n standard monomials (Bezout);
* Buchberger's criterion (stated after Definition "S-polynomial") on O1's output;
* the step objects obey Theorems "Dictionary correctness" and "Matrix
  materialization correctness", the two-pass offsets of Theorem "Race-freedom
  by prefix-sum allocation", the monomial bound of equation "monomial-count",
  Proposition "Kernel equals syzygies under dictionary closure", and the dense
  elimination O3 pins the pivot / non-pivot elimination.
"""

import itertools
import math

import pytest
import sympy

import oracle
import synth
from oracle import buchberger as bb
from oracle import dense


def canon(basis):
    """Basis as a tuple of tuples of (exps, coeff), each poly sorted largest first."""
    out = []
    for f in basis:
        d = {}
        for e, c in f:
            d[tuple(e)] = c
        out.append(tuple((e, d[e]) for e in sorted(d, key=bb.grevlex_key, reverse=True)))
    return tuple(out)


def sympy_basis(n, p, polys):
    gens = sympy.symbols("x1:%d" % (n + 1))
    exprs = []
    for f in polys:
        expr = 0
        for e, c in f:
            term = sympy.Integer(c % p)
            for g, a in zip(gens, e):
                term *= g ** a
            expr += term
        exprs.append(expr)
    G = sympy.groebner(exprs, *gens, order="grevlex", modulus=p)
    out = []
    for g in G.exprs:
        P = sympy.Poly(g, *gens, modulus=p)
        terms = [(tuple(m), int(c) % p) for m, c in P.terms()]
        lc = max(terms, key=lambda t: bb.grevlex_key(t[0]))[1]
        inv = pow(lc, p - 2, p)
        out.append([(m, c * inv % p) for m, c in terms])
    out.sort(key=lambda f: bb.grevlex_key(max((m for m, _ in f), key=bb.grevlex_key)), reverse=True)
    return canon(out)


TINY = [
    # (n, m, p, seed, density)
    (2, 2, 7, 1, 1.0), (2, 3, 7, 2, 0.7), (3, 3, 31, 3, 0.6), (3, 2, 31, 4, 1.0),
    (3, 4, 65521, 5, 0.5), (3, 3, 7, 6, 0.8), (4, 3, 31, 7, 0.35), (2, 2, 65521, 8, 1.0),
    (3, 3, 65521, 9, 0.4), (4, 4, 7, 10, 0.3), (2, 1, 31, 11, 1.0), (3, 2, 7, 12, 0.5),
]


@pytest.mark.parametrize("n,m,p,seed,density", TINY)
def test_o1_equals_o2_equals_sympy(n, m, p, seed, density):
    polys = synth.random_system(n, m, p, seed, density=density)
    g1 = canon(oracle.groebner(n, p, polys))
    g2 = canon([bb.as_sorted_terms(f) for f in bb.groebner(n, p, polys)])
    g3 = sympy_basis(n, p, polys)
    assert g1 == g2
    assert g1 == g3


def test_o1_equals_sympy_homogeneous_and_cubic():
    # inputs of degree 3 and pure quadratic forms exercise other degree patterns
    for seed in range(3):
        polys = synth.random_system(3, 3, 31, 100 + seed, density=0.5, max_deg=3)
        assert canon(oracle.groebner(3, 31, polys)) == sympy_basis(3, 31, polys)
    polys = [[(e, c) for e, c in f if sum(e) == 2] for f in synth.random_system(3, 3, 65521, 7)]
    assert canon(oracle.groebner(3, 65521, polys)) == sympy_basis(3, 65521, polys)


def test_unit_ideal_closed_form():
    n, p, polys = synth.system("dense_n6")
    B = oracle.groebner(n, p, polys)
    assert B == [[(tuple([0] * n), 1)]]


@pytest.mark.parametrize("n,p,seed", [(3, 31, 1), (4, 65521, 2), (5, 65521, 3), (4, 2147483647, 4)])
def test_planted_root_closed_form(n, p, seed):
    polys, s = synth.planted_system(n, n + 1, p, seed)
    B = oracle.groebner(n, p, polys)
    want = []
    for i in range(n):
        e = [0] * n
        e[i] = 1
        f = [(tuple(e), 1)]
        if s[i]:
            f.append((tuple([0] * n), (p - s[i]) % p))
        want.append(f)
    assert canon(B) == canon(want)


def standard_monomials(B, n, bound):
    lms = [f[0][0] for f in B]
    count = 0
    for e in itertools.product(range(bound + 1), repeat=n):
        if not any(all(a <= b for a, b in zip(l, e)) for l in lms):
            count += 1
    return count


@pytest.mark.parametrize("n,p,seed", [(2, 31, 1), (3, 65521, 2), (4, 65521, 3)])
def test_square_system_bezout_count(n, p, seed):
    polys = synth.random_system(n, n, p, seed)
    B = oracle.groebner(n, p, polys)
    # zero-dimensional: a pure power of every variable leads some element
    for i in range(n):
        assert any(all(a == 0 for j, a in enumerate(f[0][0]) if j != i) for f in B)
    assert standard_monomials(B, n, 2 ** n) == 2 ** n


def to_dict(f):
    return {tuple(e): c for e, c in f}


@pytest.mark.parametrize("n,p,seed", [(3, 65521, 2), (4, 65521, 3), (4, 31, 5)])
def test_buchberger_criterion_on_o1_output(n, p, seed):
    polys = synth.random_system(n, n, p, seed)
    B = [to_dict(f) for f in oracle.groebner(n, p, polys)]
    for i in range(len(B)):
        for j in range(i + 1, len(B)):
            assert bb.normal_form(bb.spoly(B[i], B[j], p), B, p) == {}
    for f in polys:
        assert bb.normal_form(bb.from_terms(f, p), B, p) == {}
    # reduced: no term of any element is divisible by another element's LM
    for i, f in enumerate(B):
        for j, g in enumerate(B):
            if i != j:
                lg = bb.lead(g)
                assert not any(bb.divides(lg, e) for e in f)


# ----------------------------------------------------------------- per step


def mono_mul(a, b):
    return tuple(x + y for x, y in zip(a, b))


def check_step(n, p, rec):
    G, active, d = rec["G"], rec["active"], rec["d"]
    T, rows_t, rows_k = rec["T"], rec["rows_t"], rec["rows_k"]
    row_ptr, col_ind, val = rec["row_ptr"], rec["col_ind"], rec["val"]
    r, N = len(rows_k), len(T)
    lm = lambda f: f[0][0]
    # two-pass offsets: exclusive scan of the row lengths, disjoint segments
    assert row_ptr[0] == 0 and len(row_ptr) == r + 1
    for i in range(r):
        assert row_ptr[i + 1] - row_ptr[i] == len(G[rows_k[i]])
    assert row_ptr[r] == len(col_ind) == len(val)
    # dictionary correctness: T = union of supports, strictly descending
    supp = set()
    for t, k in zip(rows_t, rows_k):
        for e, _ in G[k]:
            supp.add(mono_mul(t, e))
    assert set(T) == supp and len(T) == len(supp)
    keys = [bb.grevlex_key(e) for e in T]
    assert all(keys[i] > keys[i + 1] for i in range(N - 1))
    assert N <= math.comb(n + d, d)
    assert all(sum(e) <= d for e in T)
    # matrix correctness: every row re-expands to t * g_k
    for i, (t, k) in enumerate(zip(rows_t, rows_k)):
        got = {T[col_ind[q]]: val[q] for q in range(row_ptr[i], row_ptr[i + 1])}
        assert got == {mono_mul(t, e): c for e, c in G[k]}
        cols = col_ind[row_ptr[i]:row_ptr[i + 1]]
        assert cols == sorted(cols) and len(set(cols)) == len(cols)
    # rows: no duplicate (t, k); order = LM desc, k asc, t desc
    ids = list(zip(rows_t, rows_k))
    assert len(set(ids)) == len(ids)
    rk = [(bb.grevlex_key(mono_mul(t, lm(G[k]))), -k, bb.grevlex_key(t)) for t, k in ids]
    assert all(rk[i] > rk[i + 1] for i in range(r - 1))
    # both halves of every selected pair are rows
    lcms = set()
    for i, j in rec["sel"]:
        L = tuple(max(a, b) for a, b in zip(lm(G[i]), lm(G[j])))
        lcms.add(L)
        for k in (i, j):
            assert (tuple(a - b for a, b in zip(L, lm(G[k]))), k) in set(ids)
    # closure: a monomial of T divisible by an active LM leads some row; a row
    # that is not a half uses the most recently inserted active divisor
    leads = {}
    for t, k in ids:
        leads.setdefault(mono_mul(t, lm(G[k])), []).append(k)
    for m in T:
        divs = [g for g in range(len(G)) if active[g] and bb.divides(lm(G[g]), m)]
        if divs:
            assert m in leads
            if m not in lcms:
                assert leads[m] == [max(divs)]
    # pivots: leading column of every row; chosen row has fewest entries, then lowest index
    lead_col = [col_ind[row_ptr[i]] for i in range(r)]
    assert rec["pivot_cols"] == sorted(set(lead_col))
    for c, pr in zip(rec["pivot_cols"], rec["pivot_rows"]):
        cand = [i for i in range(r) if lead_col[i] == c]
        best = min(cand, key=lambda i: (row_ptr[i + 1] - row_ptr[i], i))
        assert pr == best
    # O3: rows of RREF(A) led by a non-pivot column are RREF of the trailing block
    A = dense.csr_to_dense(row_ptr, col_ind, val, N)
    R, pc = dense.rref(A, N, p)
    pivset = set(rec["pivot_cols"])
    want = [row for row, c in zip(R, pc) if c not in pivset]
    got = dense.csr_to_dense(rec["rref_ptr"], rec["rref_col"], rec["rref_val"], N)
    assert got == want
    assert len(R) == len(pivset) + len(got)
    return A, ids


@pytest.mark.parametrize("cfg", ["dense_n6"])
def test_step_objects_dense_n6(cfg):
    n, p, polys = synth.system(cfg)
    run = oracle.OracleRun(n, p, polys, record=-2)
    steps = run.steps()
    assert len(steps) >= 4
    for k, s in enumerate(steps):
        rec = run.step_record(k)
        check_step(n, p, rec)
        assert (s["r"], s["N"], s["M"]) == (len(rec["rows_k"]), len(rec["T"]), len(rec["col_ind"]))


@pytest.mark.parametrize("n,p,seed", [(3, 31, 1), (4, 65521, 2), (3, 7, 9)])
def test_step_objects_planted_and_kernel(n, p, seed):
    polys, _ = synth.planted_system(n, n + 1, p, seed)
    run = oracle.OracleRun(n, p, polys, record=-2)
    G0 = None
    for k in range(len(run.steps())):
        rec = run.step_record(k)
        A, ids = check_step(n, p, rec)
        if len(A) <= 60:
            # Proposition: v^T A = 0  <=>  sum v_i t_i g_{k_i} = 0 as polynomials
            K = dense.left_kernel(A, len(rec["T"]), p)
            # dimension of the left kernel: rows minus O1's rank (pivots + rho)
            assert len(K) == len(A) - (len(rec["pivot_cols"]) + len(rec["rref_ptr"]) - 1)
            for v in K[:5]:
                acc = {}
                for vi, (t, kk) in zip(v, ids):
                    if vi:
                        for e, c in rec["G"][kk]:
                            m = mono_mul(t, e)
                            acc[m] = (acc.get(m, 0) + vi * c) % p
                assert all(c == 0 for c in acc.values())
        G0 = rec
    assert G0 is not None


@pytest.mark.parametrize("seed", range(6))
def test_left_kernel_by_brute_force(seed):
    """O3's left kernel on tiny matrices over F_3 and F_5, against brute force:
    the vectors returned satisfy v^T A = 0 (by direct products), there are
    exactly r - rank(A) of them, and they span every solution (the span has
    p^(r - rank) elements, the count of all v with v^T A = 0)."""
    import random
    rnd = random.Random(seed)
    p = (3, 5)[seed % 2]
    r, ncols = rnd.randrange(1, 5), rnd.randrange(1, 4)
    A = [[rnd.randrange(p) if rnd.random() < 0.7 else 0 for _ in range(ncols)] for _ in range(r)]
    if seed == 0:
        A = [[1, 2, 0], [2, 4 % p, 0], [0, 0, 0]]  # repeated and zero rows
        r, ncols = 3, 3
    sols = [v for v in itertools.product(range(p), repeat=r)
            if all(sum(v[i] * A[i][j] for i in range(r)) % p == 0 for j in range(ncols))]
    K = dense.left_kernel(A, ncols, p)
    for v in K:
        assert all(sum(v[i] * A[i][j] for i in range(r)) % p == 0 for j in range(ncols))
    span = {tuple(sum(c * v[i] for c, v in zip(cs, K)) % p for i in range(r))
            for cs in itertools.product(range(p), repeat=len(K))}
    assert span == set(sols)
    assert len(sols) == p ** len(K)  # so the vectors are independent: dim = r - rank(A)
