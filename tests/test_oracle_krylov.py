"""Pins of O5, the block operator application (Y = A X and Y = A^T X over
F_p), against things fixed independently of it:

* brute force: the dense matrix product in Python integers, entry by entry;
* the adjoint identity <W, A X> = <A^T W, X> (mod p), which any slip between
  rows and columns breaks;
* the algebra of the Macaulay matrix: its rows are the shifts t*f_i, so the
  vector of column monomials evaluated at a common root s of the f_i is in its
  right kernel (A v = 0), while a point that is not a root is not."""

import itertools

import numpy as np
import pytest

import synth
from oracle import krylov


def random_csr(r, N, p, seed, empty_every=5):
    rng = np.random.default_rng(seed)
    ptr, idx, val = [0], [], []
    for i in range(r):
        k = 0 if (empty_every and i % empty_every == 3) else int(rng.integers(0, min(N, 9) + 1))
        cols = np.sort(rng.choice(N, size=k, replace=False)) if k else np.zeros(0, dtype=np.int64)
        idx.extend(int(c) for c in cols)
        val.extend(int(v) for v in rng.integers(1, p, size=k))
        ptr.append(len(idx))
    return np.array(ptr), np.array(idx, dtype=np.int64), np.array(val, dtype=np.int64)


@pytest.mark.parametrize("p", [3, 65521, synth.P31])
@pytest.mark.parametrize("b", [1, 3])
def test_spmm_brute_force(p, b):
    r, N = 17, 11
    ptr, idx, val = random_csr(r, N, p, p + b)
    rng = np.random.default_rng(b)
    dense = [[0] * N for _ in range(r)]
    for i in range(r):
        for e in range(ptr[i], ptr[i + 1]):
            dense[i][int(idx[e])] = int(val[e])
    X = rng.integers(0, p, size=(N, b))
    W = rng.integers(0, p, size=(r, b))
    got = krylov.spmm(ptr, idx, val, N, X, p)
    gotT = krylov.spmm(ptr, idx, val, N, W, p, trans=True)
    for i in range(r):
        for k in range(b):
            assert got[i, k] == sum(dense[i][j] * int(X[j, k]) for j in range(N)) % p
    for j in range(N):
        for k in range(b):
            assert gotT[j, k] == sum(dense[i][j] * int(W[i, k]) for i in range(r)) % p


def test_spmm_adjoint_identity():
    p = synth.P31
    r, N, b = 300, 200, 4
    ptr, idx, val = random_csr(r, N, p, 7)
    rng = np.random.default_rng(8)
    X = rng.integers(0, p, size=(N, b))
    W = rng.integers(0, p, size=(r, b))
    AX = krylov.spmm(ptr, idx, val, N, X, p)
    ATW = krylov.spmm(ptr, idx, val, N, W, p, trans=True)
    lhs = sum(int(a) * int(w) for a, w in zip(AX.ravel(), W.ravel())) % p
    rhs = sum(int(a) * int(x) for a, x in zip(ATW.ravel(), X.ravel())) % p
    assert lhs == rhs


def macaulay(polys, n, shift_deg):
    """Rows t*f for every monomial t of degree <= shift_deg and every f, over
    the columns of every monomial that occurs (any fixed column order)."""
    shifts = [tuple(int(x) for x in e) for e in synth.monomials_upto(n, shift_deg)]
    rows = []
    for t in shifts:
        for f in polys:
            rows.append({tuple(a + b for a, b in zip(t, e)): c for e, c in f})
    cols = sorted({m for row in rows for m in row})
    where = {m: j for j, m in enumerate(cols)}
    ptr, idx, val = [0], [], []
    for row in rows:
        items = sorted((where[m], c) for m, c in row.items() if c)
        idx.extend(j for j, _ in items)
        val.extend(c for _, c in items)
        ptr.append(len(idx))
    return np.array(ptr), np.array(idx), np.array(val), cols


def test_macaulay_kernel_at_a_root():
    n, p = 4, 65521
    polys, s = synth.planted_system(n, 5, p, 11)
    ptr, idx, val, cols = macaulay(polys, n, 2)
    def at(point):
        out = []
        for m in cols:
            v = 1
            for i, a in enumerate(m):
                v = v * pow(point[i], a, p) % p
            out.append([v])
        return np.array(out, dtype=np.int64)

    assert not krylov.spmm(ptr, idx, val, len(cols), at(s), p).any()
    assert krylov.spmm(ptr, idx, val, len(cols), at([(x + 1) % p for x in s]), p).any()


def test_monomials_upto_counts():
    from math import comb
    for n, d in [(1, 4), (3, 3), (14, 3)]:
        m = synth.monomials_upto(n, d)
        assert len(m) == comb(n + d, d) and len({tuple(r) for r in m}) == len(m)
        assert m.min() >= 0 and m.sum(axis=1).max() == d
