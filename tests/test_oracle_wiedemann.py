"""Pins of O6 (block Wiedemann left-kernel vectors, oracle/wiedemann.py)
against facts it does not compute itself:

* the projected Krylov sequence equals X^T B^t (B Y) formed from the dense
  matrix B = A D A^T with Python integers (no sparse product involved);
* every row of the sigma-basis satisfies its defining property, P_i F = 0 mod
  x^sigma for F = [S(x)^T ; -I], checked by plain polynomial multiplication,
  with the degree bounds that make its g part a generator;
* for one vector (b = 1) the generator of least degree is the monic minimal
  recurrence of the scalar sequence found by brute force (the smallest order
  whose Hankel system is solvable, by Gaussian elimination over Python
  integers), and its degree is the degree of the minimal polynomial of B
  (the smallest d with B^d in the span of lower powers);
* the kernel vectors satisfy v^T A = 0 by direct products and span exactly
  a planted left kernel, and on Macaulay matrices of F4 steps they are
  polynomial identities sum v_i t_i g_{k_i} = 0 (Proposition "Kernel equals
  syzygies under dictionary closure").
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import dense
from oracle import wiedemann as w6


def dense_of(rp, ci, vv, ncols):
    r = len(rp) - 1
    A = [[0] * ncols for _ in range(r)]
    for i in range(r):
        for e in range(rp[i], rp[i + 1]):
            A[i][ci[e]] = int(vv[e])
    return A


def matmul(X, Y, p):
    return [[sum(a * b for a, b in zip(row, col)) % p for col in zip(*Y)] for row in X]


def transpose(X):
    return [list(c) for c in zip(*X)]


def csr_of(A):
    rp, ci, vv = [0], [], []
    for row in A:
        for j, v in enumerate(row):
            if v:
                ci.append(j)
                vv.append(int(v))
        rp.append(len(ci))
    return rp, ci, vv


def rank_mod(M, p):
    M = [[int(x) % p for x in row] for row in M]
    rk = 0
    ncols = len(M[0]) if M else 0
    for c in range(ncols):
        piv = next((i for i in range(rk, len(M)) if M[i][c]), None)
        if piv is None:
            continue
        M[rk], M[piv] = M[piv], M[rk]
        inv = pow(M[rk][c], p - 2, p)
        M[rk] = [x * inv % p for x in M[rk]]
        for i in range(len(M)):
            if i != rk and M[i][c]:
                f = M[i][c]
                M[i] = [(x - f * y) % p for x, y in zip(M[i], M[rk])]
        rk += 1
    return rk


def planted(r0, ncols, k, p, seed, maxlen=8):
    """r0 sparse random rows and k random combinations of them (left kernel of
    dimension k when the first r0 rows are independent, checked)."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(r0):
        idx = rng.choice(ncols, size=int(rng.integers(2, maxlen + 1)), replace=False)
        row = [0] * ncols
        for j in idx:
            row[int(j)] = int(rng.integers(1, p))
        rows.append(row)
    assert rank_mod(rows, p) == r0
    for _ in range(k):
        c = [int(x) for x in rng.integers(0, p, size=r0)]
        rows.append([sum(ci * row[j] for ci, row in zip(c, rows[:r0])) % p for j in range(ncols)])
    order = rng.permutation(len(rows))
    return [rows[i] for i in order]


def inputs(r, ncols, b, p, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(1, p, size=ncols), rng.integers(0, p, size=(r, b)), rng.integers(0, p, size=(r, b)))


@pytest.mark.parametrize("p,b,seed", [(65521, 3, 1), (synth.P31, 2, 2), (7, 4, 3)])
def test_sequence_is_projected_dense_powers(p, b, seed):
    A = planted(14, 20, 3, p, seed)
    rp, ci, vv = csr_of(A)
    d, X, Y = inputs(len(A), 20, b, p, seed + 10)
    L = 9
    S = w6.sequence(rp, ci, vv, 20, d, X, Y, p, L)
    D = [[int(d[i]) if i == j else 0 for j in range(20)] for i in range(20)]
    B = matmul(matmul(A, D, p), transpose(A), p)
    Z = matmul(B, [[int(x) for x in row] for row in Y], p)
    Xt = transpose([[int(x) for x in row] for row in X])
    for t in range(L):
        assert np.array_equal(S[t], np.array(matmul(Xt, Z, p)))
        Z = matmul(B, Z, p)


def polymul_row(Pi, F, p, order):
    """Coefficients below x^order of the row vector Pi (list of coefficient
    lists) times the matrix F (F[j][c] coefficient lists)."""
    ncol = len(F[0])
    out = [[0] * order for _ in range(ncol)]
    for j, a in enumerate(Pi):
        for c in range(ncol):
            f = F[j][c]
            for u, x in enumerate(a[:order]):
                if x:
                    for v in range(0, order - u):
                        if v < len(f) and f[v]:
                            out[c][u + v] = (out[c][u + v] + x * f[v]) % p
    return out


@pytest.mark.parametrize("p,b,seed", [(65521, 2, 4), (101, 3, 5), (synth.P31, 1, 6)])
def test_sigma_basis_definition(p, b, seed):
    A = planted(16, 22, 2, p, seed)
    rp, ci, vv = csr_of(A)
    d, X, Y = inputs(len(A), 22, b, p, seed)
    L = w6.block_len(len(A), b)
    S = w6.sequence(rp, ci, vv, 22, d, X, Y, p, L)
    P, s = w6.mbasis(S, b, p)
    # F = [S(x)^T ; -I_b] as coefficient lists
    F = [[[int(S[t][c][j]) for t in range(L)] for c in range(b)] for j in range(b)]
    F += [[[(p - 1) if c == j else 0] for c in range(b)] for j in range(b)]
    s0 = [0] * b + [1] * b
    for i in range(2 * b):
        res = polymul_row(P[i], F, p, L)
        assert all(x == 0 for col in res for x in col), "row %d is not an approximant to order %d" % (i, L)
        for j in range(2 * b):
            deg = max((u for u, x in enumerate(P[i][j]) if x), default=-1)
            assert deg <= s[i] - s0[j]
    # the basis generates every approximant: its determinant has degree
    # sum(s - s0) = b * sigma (no approximant is missing a factor of x)
    assert sum(s) - sum(s0) == b * L


def minimal_recurrence(a, p):
    """Smallest d and monic c (c_d = 1) with sum_m c_m a_{t+m} = 0 for all t
    with t + d < len(a), by solving each Hankel system in turn."""
    L = len(a)
    for d in range(0, L // 2 + 1):
        rows = [[a[t + m] % p for m in range(d)] + [(-a[t + d]) % p] for t in range(L - d)]
        # solve sum_{m<d} c_m a_{t+m} = -a_{t+d}
        M = [row[:] for row in rows]
        rk, piv = 0, []
        for c in range(d):
            pr = next((i for i in range(rk, len(M)) if M[i][c]), None)
            if pr is None:
                continue
            M[rk], M[pr] = M[pr], M[rk]
            inv = pow(M[rk][c], p - 2, p)
            M[rk] = [x * inv % p for x in M[rk]]
            for i in range(len(M)):
                if i != rk and M[i][c]:
                    f = M[i][c]
                    M[i] = [(x - f * y) % p for x, y in zip(M[i], M[rk])]
            piv.append(c)
            rk += 1
        if any(M[i][d] for i in range(rk, len(M))):
            continue
        sol = [0] * d
        for i, c in enumerate(piv):
            sol[c] = M[i][d]
        return d, sol + [1]
    return None


def minpoly_degree(B, p):
    """Smallest d with B^d in the span of I, B, ..., B^(d-1) (flattened powers)."""
    n = len(B)
    powers = [[1 if i == j else 0 for j in range(n) for i in range(n)]]
    Bk = [[1 if i == j else 0 for j in range(n)] for i in range(n)]
    for d in range(1, n + 1):
        Bk = matmul(Bk, B, p)
        powers.append([x for row in Bk for x in row])
        if rank_mod(powers, p) < len(powers):
            return d
    return n


@pytest.mark.parametrize("p,seed", [(65521, 7), (synth.P31, 8), (257, 9)])
def test_scalar_generator_is_the_minimal_recurrence(p, seed):
    A = planted(10, 14, 2, p, seed)
    rp, ci, vv = csr_of(A)
    d, X, Y = inputs(len(A), 14, 1, p, seed)
    L = w6.block_len(len(A), 1)
    S = w6.sequence(rp, ci, vv, 14, d, X, Y, p, L)
    P, s = w6.mbasis(S, 1, p)
    gens = w6.generators(P, s, 1, L)
    assert gens, "no generator row"
    deg, f = gens[0]
    a = [int(S[t][0][0]) for t in range(L)]
    dmin, cmin = minimal_recurrence(a, p)
    assert deg == dmin
    lead = f[deg][0]
    assert lead != 0
    inv = pow(lead, p - 2, p)
    assert [x[0] * inv % p for x in f] == cmin
    # and its degree is that of the minimal polynomial of B (the sequence starts
    # at B Y, so the factor x of the kernel is not seen: the minimal polynomial
    # of B restricted away from its kernel, here deg minpoly(B) - 1)
    D = [[int(d[i]) if i == j else 0 for j in range(14)] for i in range(14)]
    B = matmul(matmul(A, D, p), transpose(A), p)
    assert dmin == minpoly_degree(B, p) - 1


@pytest.mark.parametrize("p,b,k,seed", [(65521, 4, 3, 11), (synth.P31, 3, 2, 12), (65521, 2, 1, 13),
                                        (synth.P31, 5, 4, 14)])
def test_planted_left_kernel(p, b, k, seed):
    A = planted(26, 40, k, p, seed)
    rp, ci, vv = csr_of(A)
    d, X, Y = inputs(len(A), 40, b, p, seed)
    res = w6.left_kernel_block_wiedemann(rp, ci, vv, 40, d, X, Y, p)
    for deg, f in res["gens"]:
        assert w6.check_generator(res["S"], f, p)
    assert res["vectors"]
    for v in res["vectors"]:
        assert any(v)
        vA = [sum(int(v[i]) * A[i][j] for i in range(len(A))) % p for j in range(40)]
        assert not any(vA)
    # they span the planted kernel: rank k, and together with O3's basis of
    # the left kernel the rank stays k
    K = dense.left_kernel(A, 40, p)
    assert len(K) == k
    assert rank_mod([list(v) for v in res["vectors"]], p) == k
    assert rank_mod([list(v) for v in res["vectors"]] + K, p) == k


def mono_mul(a, b):
    return tuple(x + y for x, y in zip(a, b))


@pytest.mark.parametrize("cfg_n,p,seed,b", [(4, 65521, 21, 4), (3, synth.P31, 22, 3)])
def test_macaulay_left_kernel_is_syzygies(cfg_n, p, seed, b):
    n = cfg_n
    polys, _ = synth.planted_system(n, n + 1, p, seed)
    run = oracle.OracleRun(n, p, polys, record=-2)
    tested = 0
    for k in range(len(run.steps())):
        rec = run.step_record(k)
        rp = [int(x) for x in rec["row_ptr"]]
        ci = [int(x) for x in rec["col_ind"]]
        vv = [int(x) for x in rec["val"]]
        r, N = len(rp) - 1, len(rec["T"])
        rank = len(rec["pivot_cols"]) + len(rec["rref_ptr"]) - 1
        if r - rank == 0 or r > 80:
            continue
        d, X, Y = inputs(r, N, b, p, seed + k)
        res = w6.left_kernel_block_wiedemann(rp, ci, vv, N, d, X, Y, p)
        assert res["vectors"]
        A = dense_of(rp, ci, vv, N)
        # b independent syzygies (or the whole kernel when it is smaller)
        assert rank_mod([list(v) for v in res["vectors"]], p) == min(b, r - rank)
        for v in res["vectors"]:
            assert not any(sum(int(v[i]) * A[i][j] for i in range(r)) % p for j in range(N))
            acc = {}
            for vi, t, kk in zip(v, rec["rows_t"], rec["rows_k"]):
                if vi:
                    for e, c in rec["G"][kk]:
                        m = mono_mul(t, e)
                        acc[m] = (acc.get(m, 0) + int(vi) * c) % p
            assert all(c == 0 for c in acc.values())
        tested += 1
    assert tested >= 1
