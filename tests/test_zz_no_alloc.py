"""Allocation-free block product (f4_spmm_noalloc) against the allocating
f4_spmm on a handle of the same CSR, bit for bit: two calls in a row, the
second on a smaller matrix (the per-GPU scratch keeps the first call's
transpose, which must not leak into the second), both orientations and two
block widths; and the size limit, refused before any work.  Every case is
printed first."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def random_csr(r, N, seed, vmax, maxlen):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, min(N, maxlen) + 1, size=r)
    lens[5::11] = 0  # empty rows
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx = np.concatenate([np.sort(rng.choice(N, size=k, replace=False)) for k in lens]).astype(np.int64)
    val = rng.integers(1, vmax, size=int(ptr[-1]), dtype=np.int64)
    return ptr, idx, val


@pytest.fixture(scope="module")
def env():
    import paper_2601_06765_amd.f4 as f4
    c = f4.Context(0)
    yield f4, c
    c.close()


@pytest.mark.parametrize("p,b", [(synth.P31, 8), (65521, 5)])
def test_noalloc_matches_spmm_twice_second_smaller(env, p, b):
    f4, c = env
    # first call: 3 100 rows x 4 000 columns, ragged rows up to 300 entries;
    # second call: 700 x 900, so the scratch holds a longer stale transpose
    for call, (r, N, maxlen, seed) in enumerate([(3100, 4000, 300, 11), (700, 900, 60, 12)]):
        ptr, idx, val = random_csr(r, N, seed + b, p, maxlen)
        nnz = int(ptr[-1])
        A = c.matrix_from_csr(r, N, ptr, idx, val)
        dptr, didx, dval = c.to_device(ptr), c.to_device(idx), c.to_device(val)
        rng = np.random.default_rng(100 * call + b)
        for trans in (True, False):
            nin, nout = (r, N) if trans else (N, r)
            X = c.to_device(rng.integers(0, p, size=(nin, b), dtype=np.int64))
            say("noalloc call", call, "r", r, "N", N, "nnz", nnz, "p", p, "b", b, "trans", trans)
            want = c.spmm(p, A, X, trans=trans).to_host()
            out = c.device_array((nout, b))
            got = c.spmm_noalloc(p, r, N, nnz, dptr, didx, dval, X, out, trans=trans).to_host()
            assert np.array_equal(got, want), "allocation-free product differs (call %d, trans %s)" % (call, trans)
            X.free()
            out.free()
        A.free()
        for d in (dptr, didx, dval):
            d.free()


def test_noalloc_size_limit(env):
    f4, c = env
    r, N = 4, 4
    ptr, idx, val = np.array([0, 1, 2, 3, 4]), np.arange(4), np.ones(4, dtype=np.int64)
    dptr, didx, dval = c.to_device(ptr), c.to_device(idx), c.to_device(val)
    X, out = c.to_device(np.ones((r, 2), dtype=np.int64)), c.device_array((N, 2))
    # a transpose of 2^24 entries needs about 128 MiB of scratch: refused
    # from the sizes alone, before any array is read
    say("noalloc size limit")
    with pytest.raises(f4.F4Error) as e:
        c.spmm_noalloc(65521, r, N, 1 << 24, dptr, didx, dval, X, out, trans=True)
    assert e.value.code == f4.F4_E_RANGE
    # the same sizes without the transpose need no scratch and are fine
    Y = c.spmm_noalloc(65521, r, N, 4, dptr, didx, dval, c.to_device(np.ones((N, 2), dtype=np.int64)),
                       c.device_array((r, 2)))
    assert np.array_equal(Y.to_host(), np.ones((r, 2)))
