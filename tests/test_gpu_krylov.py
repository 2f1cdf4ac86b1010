"""Block operator application (f4_spmm: Y = A X and Y = A^T X over F_p) on
the device against O5, exactly: random CSR matrices with empty and ragged
rows and block widths across every lane layout, words of X and stored values
at or above p (read modulo p), the Macaulay matrix of a planted system built
by the symbolic preprocessing (its root's monomial vector is in the kernel),
and the full-size Macaulay operator of the sparse n=14 system on sampled rows
and columns plus the adjoint identity.  Every test prints its case first."""

import sys

import numpy as np
import pytest

import synth
from oracle import krylov as o5

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


def host(d):
    return d.to_host().astype(np.int64)


def random_csr(r, N, seed, vmax, empty_every=7, maxlen=40):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, min(N, maxlen) + 1, size=r)
    if empty_every:
        lens[3::empty_every] = 0
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx = np.concatenate([np.sort(rng.choice(N, size=k, replace=False)) for k in lens] or [np.zeros(0)]).astype(np.int64)
    val = rng.integers(1, vmax, size=int(ptr[-1]), dtype=np.int64)
    return ptr, idx, val


@pytest.mark.parametrize("p", [3, 65521, synth.P31])
@pytest.mark.parametrize("b", [1, 2, 3, 4, 5, 6, 8, 12, 13, 17, 32, 33, 63, 64])
def test_spmm_random(env, p, b):
    f4, c = env
    r, N = 1037, 705
    # stored values up to 2^32 - 1: read modulo p, like the words of X
    ptr, idx, val = random_csr(r, N, 100 * b + p % 97, 1 << 32)
    A = c.matrix_from_csr(r, N, ptr, idx, val)
    rng = np.random.default_rng(b)
    X = rng.integers(0, 1 << 32, size=(N, b), dtype=np.int64)
    W = rng.integers(0, 1 << 32, size=(r, b), dtype=np.int64)
    say("spmm random", r, N, "p", p, "b", b)
    Y = c.spmm(p, A, c.to_device(X))
    YT = c.spmm(p, A, c.to_device(W), trans=True)
    assert np.array_equal(host(Y), o5.spmm(ptr, idx, val, N, X, p))
    assert np.array_equal(host(YT), o5.spmm(ptr, idx, val, N, W, p, trans=True))
    A.free()


@pytest.mark.parametrize("b", [2, 6, 12])
def test_spmm_unaligned_blocks(env, b):
    """Even b with X or Y starting 4 bytes past an 8-byte boundary (one word
    per lane then): the same results."""
    f4, c = env
    p = synth.P31
    r, N = 301, 257
    ptr, idx, val = random_csr(r, N, 7 + b, p)
    A = c.matrix_from_csr(r, N, ptr, idx, val)
    rng = np.random.default_rng(50 + b)
    X = rng.integers(0, p, size=(N, b), dtype=np.int64)
    want = o5.spmm(ptr, idx, val, N, X, p)
    Xb = c.to_device(np.concatenate([[0], X.ravel()]))
    Yb = c.device_array(r * b + 1)
    say("spmm unaligned X and Y, b", b)
    Y = c.spmm(p, A, Xb.sub(1, (N, b)), out=Yb.sub(1, (r, b)))
    assert np.array_equal(host(Y), want)
    Y2 = c.spmm(p, A, c.to_device(X), out=Yb.sub(1, (r, b)))
    assert np.array_equal(host(Y2), want)
    A.free()


def test_spmm_edges(env):
    f4, c = env
    p = 65521
    say("spmm all-empty rows and a single entry")
    A = c.matrix_from_csr(5, 4, [0, 0, 0, 0, 0, 0], [], [])
    Y = c.spmm(p, A, c.to_device(np.ones((4, 3))))
    YT = c.spmm(p, A, c.to_device(np.ones((5, 3))), trans=True)
    assert not host(Y).any() and host(Y).shape == (5, 3) and not host(YT).any() and host(YT).shape == (4, 3)
    A.free()
    B = c.matrix_from_csr(1, 1, [0, 1], [0], [p - 1])
    Y = c.spmm(p, B, c.to_device([p - 1]))
    assert host(Y).tolist() == [1]
    with pytest.raises(f4.F4Error) as e:
        c.spmm(65520, B, c.to_device([1]))
    assert e.value.code == f4.F4_E_ARG
    with pytest.raises(ValueError):
        c.spmm(p, B, c.to_device(np.ones((2, 1))))
    Y, ms = c.spmm_timed(p, B, c.to_device([3]), reps=3)
    assert host(Y).tolist() == [(p - 1) * 3 % p] and ms > 0
    with pytest.raises(f4.F4Error) as e:
        c.spmm(p, B, c.to_device(np.ones((1, 65))))
    assert e.value.code == f4.F4_E_ARG
    say("spmm matrix without columns")
    E = c.matrix_from_csr(3, 0, [0, 0, 0, 0], [], [])
    Y = c.spmm(p, E, c.to_device(np.zeros((0, 2))))
    YT = c.spmm(p, E, c.to_device(np.ones((3, 2))), trans=True)
    assert host(Y).shape == (3, 2) and not host(Y).any() and host(YT).shape == (0, 2)
    E.free()
    B.free()


def macaulay_rows(f4, n, shift_deg, m):
    t = f4.pack_many(n, synth.monomials_upto(n, shift_deg))
    return np.repeat(t, m), np.tile(np.arange(m, dtype=np.uint32), len(t))


def test_spmm_macaulay_planted_root(env):
    f4, c = env
    n, p = 6, 65521
    polys, s = synth.planted_system(n, 7, p, 21)
    polys = f4.normalize(p, n, polys)
    tw, ks = macaulay_rows(f4, n, 3, len(polys))
    say("spmm Macaulay planted n=6 shift degree 3, rows", len(tw))
    A = c.build_matrix_rows_packed(p, n, polys, tw, ks)
    h = A.to_host()
    exps = [f4.unpack(n, int(k)) for k in h["dict_keys"]]
    v = np.array([[int(np.prod([1] + [pow(s[i], e[i], p) for i in range(n)], dtype=object) % p)] for e in exps],
                 dtype=np.int64)
    Y = c.spmm(p, A, c.to_device(v))
    X = np.random.default_rng(3).integers(0, p, size=(h["N"], 4))
    Y2 = c.spmm(p, A, c.to_device(X))
    W = np.random.default_rng(4).integers(0, p, size=(h["r"], 4))
    Y3 = c.spmm(p, A, c.to_device(W), trans=True)
    assert not host(Y).any()
    assert np.array_equal(host(Y2), o5.spmm(h["row_ptr"], h["col_ind"], h["val"], h["N"], X, p))
    assert np.array_equal(host(Y3), o5.spmm(h["row_ptr"], h["col_ind"], h["val"], h["N"], W, p, trans=True))
    A.free()


def test_spmm_full_size_macaulay_sampled(env):
    # the operator the benchmark times: degree-10 Macaulay matrix of the
    # sparse n=14 system over F_(2^31-1), b = 8
    f4, c = env
    n, p, polys = synth.system("sparse_n14")
    polys = f4.normalize(p, n, polys)
    tw, ks = macaulay_rows(f4, n, 8, len(polys))
    say("spmm full-size Macaulay n=14 shift degree 8, rows", len(tw))
    A = c.build_matrix_rows_packed(p, n, polys, tw, ks)
    r, N = A.view.r, A.view.N
    b = 8
    rng = np.random.default_rng(6)
    Xh = rng.integers(0, p, size=(N, b), dtype=np.int64)
    Wh = rng.integers(0, p, size=(r, b), dtype=np.int64)
    Y = c.spmm(p, A, c.to_device(Xh))
    YT = c.spmm(p, A, c.to_device(Wh), trans=True)
    h = A.to_host()
    A.free()
    Yh, YTh = host(Y), host(YT)
    # the operator itself (this size takes the symbolic preprocessing's global
    # bitmap path): the dictionary is exactly the set of the products t*m over
    # all rows and terms, and sampled rows re-expand to t * f_k
    words = [f4.pack_many(n, np.array([e for e, _ in f], dtype=np.int64)) for f in polys]
    coefs = [np.array([c0 % p for _, c0 in f], dtype=np.int64) for f in polys]
    dk = h["dict_keys"]
    order = np.argsort(dk)
    sdk = dk[order]
    hits = np.zeros(N, dtype=bool)
    for kk in range(len(polys)):
        rsel = np.nonzero(h["row_k"] == kk)[0]
        prods = (h["row_t"][rsel][:, None] + words[kk][None, :]).ravel()
        pos = np.searchsorted(sdk, prods)
        assert (pos < N).all() and np.array_equal(sdk[np.minimum(pos, N - 1)], prods)
        hits[pos] = True
    assert hits.all()
    ptr0 = h["row_ptr"].astype(np.int64)
    for i in np.random.default_rng(9).choice(r, size=300, replace=False):
        kk, t0 = int(h["row_k"][i]), h["row_t"][i]
        got = {int(dk[j]): int(v) for j, v in zip(h["col_ind"][ptr0[i]:ptr0[i + 1]], h["val"][ptr0[i]:ptr0[i + 1]])}
        want = {int(t0 + w0): int(c0) for w0, c0 in zip(words[kk], coefs[kk]) if c0}
        assert got == want
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(r, size=2000, replace=False))
    ptr = h["row_ptr"].astype(np.int64)
    sub_ptr = np.concatenate([[0], np.cumsum(ptr[rows + 1] - ptr[rows])])
    take = np.concatenate([np.arange(ptr[i], ptr[i + 1]) for i in rows])
    want = o5.spmm(sub_ptr, h["col_ind"][take], h["val"][take], N, Xh, p)
    assert np.array_equal(Yh[rows], want)
    cols = np.sort(rng.choice(N, size=300, replace=False))
    ci = h["col_ind"].astype(np.int64)
    sel = np.nonzero(np.isin(ci, cols))[0]
    rid = np.searchsorted(ptr, sel, side="right") - 1
    pos = np.searchsorted(cols, ci[sel])
    wantT = np.zeros((len(cols), b), dtype=np.int64)
    np.add.at(wantT, pos, (h["val"][sel].astype(np.int64)[:, None] % p) * Wh[rid] % p)
    assert np.array_equal(YTh[cols], wantT % p)
    lhs = int(((Wh * Yh) % p).sum() % p)
    rhs = int(((YTh * Xh) % p).sum() % p)
    assert lhs == rhs
