"""The 16-bit modular product used by the elimination kernels for p < 2^16:
x = a*b (exact in 32 bits), q = trunc(float(x) * float(1/p)), r = x - q*p,
then r <- min(r, r + p), r <- min(r, r - p) in wrapping 32-bit unsigned
arithmetic.  numpy's float32 multiply rounds to nearest even and its
float32 -> uint32 conversion truncates, like the device instructions, so
this emulation pins the claim that the result is a*b mod p for every product
of residues (the full range is swept off-line; here a dense sample and the
values next to every multiple of p near the top of the range)."""

import numpy as np
import pytest


def mul16(a, b, p):
    finv = np.float32(1.0) / np.float32(p)
    x = (a.astype(np.uint64) * b.astype(np.uint64)).astype(np.uint32)
    q = (x.astype(np.float32) * finv).astype(np.uint32)
    r = (x - q * np.uint32(p)).astype(np.uint32)
    r = np.minimum(r, r + np.uint32(p))
    return np.minimum(r, r - np.uint32(p))


@pytest.mark.parametrize("p", [65521, 65519, 32749, 257, 3])
def test_mul16_exact(p):
    rng = np.random.default_rng(p)
    a = rng.integers(0, p, 2_000_000, dtype=np.uint64)
    b = rng.integers(0, p, 2_000_000, dtype=np.uint64)
    want = (a * b) % np.uint64(p)
    assert np.array_equal(mul16(a, b, p).astype(np.uint64), want)
    # products next to multiples of p, up to (p-1)^2
    top = np.arange(max(1, p - 2000), p, dtype=np.uint64)
    a2 = np.repeat(top, 3)
    b2 = np.tile(np.array([p - 1, p - 2, 1], dtype=np.uint64), len(top))
    assert np.array_equal(mul16(a2, b2, p).astype(np.uint64), (a2 * b2) % np.uint64(p))


def ff64(piv, a, fk, b, p):
    """(piv*a - fk*b) mod p as the echelon block step computes it for p < 2^16:
    t is exact in double (|t| < 2^33), q = floor(t * fl(1/p)) rounds once, and
    t - q*p is exact; two corrections bring it into [0, p)."""
    dinv = np.float64(1.0) / np.float64(p)
    t = piv.astype(np.int64) * a.astype(np.int64) - fk.astype(np.int64) * b.astype(np.int64)
    q = np.floor(t.astype(np.float64) * dinv).astype(np.int64)
    r = t - q * p
    r = np.where(r < 0, r + p, r)
    return np.where(r >= p, r - p, r)


@pytest.mark.parametrize("p", [65521, 65519, 32749, 257, 3])
def test_fraction_free_update_exact(p):
    rng = np.random.default_rng(p + 1)
    k = 1_000_000
    piv, a, fk, b = (rng.integers(0, p, k, dtype=np.int64) for _ in range(4))
    want = (piv * a - fk * b) % p
    assert np.array_equal(ff64(piv, a, fk, b, p), want)
    # extremes: largest products of either sign, and exact multiples of p
    e = np.array([p - 1, p - 2, 1, 0], dtype=np.int64)
    P, A, F, B = (x.ravel() for x in np.meshgrid(e, e, e, e))
    assert np.array_equal(ff64(P, A, F, B, p), (P * A - F * B) % p)
