"""The modular forms of the kernels, emulated in numpy with the device's word
sizes, against Python's exact residues.

* One-word Barrett (any p < 2^31, x < 2^32): q = high word of x * floor(2^32/p),
  r = x - q*p wrapping, r <- min(r, r - p).  The elimination kernels' products
  for p < 2^16 (a*b and the fraction-free update piv*a - fk*b) use it.
* The 24-bit form of the modular inner-loop microbenchmark (p < 2^16):
  x = a*b, q = trunc(float(x) * float(1/p)), r = x - q*p, then
  r <- min(r, r + p), r <- min(r, r - p).  numpy's float32 multiply rounds to
  nearest even and its float32 -> uint32 conversion truncates, like the device
  instructions.

Each is checked on a dense random sample and on the values next to multiples
of p and at the top of the word."""

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


def red32(x, p):
    """One-word Barrett step: q = high word of x * floor(2^32 / p), r = x - q*p
    (wrapping 32-bit), then r <- min(r, r - p)."""
    mu = np.uint64((1 << 32) // p)
    x = x.astype(np.uint64)
    q = (x * mu) >> np.uint64(32)
    r = ((x - q * np.uint64(p)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return np.minimum(r, r - np.uint32(p))


def mul32(a, b, p):
    return red32((a.astype(np.uint64) * b.astype(np.uint64)) & np.uint64(0xFFFFFFFF), p)


def ff32(piv, a, fk, b, p):
    """(piv*a - fk*b) mod p as the echelon block step computes it for p < 2^16:
    (piv*a mod p) + (p - fk)*b stays below p^2 < 2^32, then one more step."""
    t = mul32(piv, a, p).astype(np.uint64) + (np.uint64(p) - fk.astype(np.uint64)) * b.astype(np.uint64)
    assert int(t.max(initial=0)) < 1 << 32
    return red32(t, p)


@pytest.mark.parametrize("p", [2147483647, 2147483629, 65521, 257, 3])
def test_one_word_barrett_exact(p):
    rng = np.random.default_rng(p + 2)
    x = rng.integers(0, 1 << 32, 2_000_000, dtype=np.uint64)
    # the top of the word and the values next to multiples of p
    top = np.arange((1 << 32) - 3000, 1 << 32, dtype=np.uint64)
    mult = (np.arange(1, 2000, dtype=np.uint64) * np.uint64(p))
    mult = mult[mult < (1 << 32) - 1]
    near = np.concatenate([mult - 1, mult, mult + 1])
    for v in (x, top, near):
        assert np.array_equal(red32(v, p).astype(np.uint64), v % np.uint64(p))


@pytest.mark.parametrize("p", [65521, 65519, 32749, 257, 3])
def test_mul32_exact(p):
    rng = np.random.default_rng(p + 3)
    a = rng.integers(0, p, 2_000_000, dtype=np.uint64)
    b = rng.integers(0, p, 2_000_000, dtype=np.uint64)
    assert np.array_equal(mul32(a, b, p).astype(np.uint64), (a * b) % np.uint64(p))


@pytest.mark.parametrize("p", [65521, 65519, 32749, 257, 3])
def test_fraction_free_update_exact(p):
    rng = np.random.default_rng(p + 1)
    k = 1_000_000
    piv, a, fk, b = (rng.integers(0, p, k, dtype=np.int64) for _ in range(4))
    want = (piv * a - fk * b) % p
    assert np.array_equal(ff32(piv, a, fk, b, p).astype(np.int64), want)
    # extremes: largest products of either sign, and exact multiples of p
    e = np.array([p - 1, p - 2, 1, 0], dtype=np.int64)
    P, A, F, B = (x.ravel() for x in np.meshgrid(e, e, e, e))
    assert np.array_equal(ff32(P, A, F, B, p).astype(np.int64), (P * A - F * B) % p)


# ------------------------------------------------ exact double-precision sums
# The echelon update forms sum_u w_u x_u mod p for 32 residue pairs with
# double-precision multiply-adds: p < 2^16 directly (sum < 2^37), otherwise w
# split into 16-bit halves (sums below 2^51 and 2^52) recombined as
# (S_hi mod p) 2^16 + S_lo, and x mod p as x - floor(x * (1/p)) p with one
# correction each way.  Every product and partial sum here is an integer below
# 2^53, so numpy's separate multiply and add give what the fused multiply-add
# gives on the device.

def dmod(x, p):
    pd = np.float64(p)
    pinv = np.float64(1.0) / pd
    q = np.floor(x * pinv)
    r = x - q * pd  # |r| < 2p: exact, as the device's fused form
    r = np.where(r < 0, r + pd, r)
    return np.where(r >= pd, r - pd, r)


def dot_mod(w, x, p, small):
    """w, x: (n, 32) residues; returns sum_u w x mod p per row, as the kernel forms it."""
    xd = x.astype(np.float64)
    if small:
        s = np.zeros(len(w))
        for u in range(w.shape[1]):
            s = s + w[:, u].astype(np.float64) * xd[:, u]
        return dmod(s, p)
    sh, sl = np.zeros(len(w)), np.zeros(len(w))
    for u in range(w.shape[1]):
        sh = sh + (w[:, u] >> 16).astype(np.float64) * xd[:, u]
        sl = sl + (w[:, u] & 0xffff).astype(np.float64) * xd[:, u]
    return dmod(dmod(sh, p) * 65536.0 + sl, p)


@pytest.mark.parametrize("p,small", [(3, True), (257, True), (65521, True), (65519, True), (3, False),
                                     (65521, False), (2147483647, False), (2147483629, False),
                                     (2147483497, False), (1000003, False)])
def test_double_split_dot_exact(p, small):
    rng = np.random.default_rng(p + small)
    n = 200_000
    w = rng.integers(0, p, (n, 32), dtype=np.uint64)
    x = rng.integers(0, p, (n, 32), dtype=np.uint64)
    # the largest sums: every factor p - 1, and rows of mixed extremes
    w[:1000] = p - 1
    x[:1000] = p - 1
    w[1000:2000, ::2] = p - 1
    x[1000:2000, 1::2] = p - 1
    want = np.array([sum(int(a) * int(b) for a, b in zip(wr, xr)) % p for wr, xr in zip(w[:3000], x[:3000])],
                    dtype=np.uint64)
    got = dot_mod(w, x, p, small).astype(np.uint64)
    assert np.array_equal(got[:3000], want)
    # the rest against exact object-integer sums, vectorised
    ws, xs = w[3000:].astype(object), x[3000:].astype(object)
    want2 = np.array((ws * xs).sum(axis=1) % p, dtype=np.uint64)
    assert np.array_equal(got[3000:], want2)


@pytest.mark.parametrize("p", [3, 65521, 2147483647, 2147483497])
def test_dmod_near_multiples(p):
    # integers next to multiples of p across the range the kernels reduce (< 2^53)
    k = np.unique(np.concatenate([np.arange(0, 4000), (np.float64(2) ** 53 // p) - np.arange(0, 4000)]))
    k = k[k >= 0]
    base = k * np.float64(p)
    for d in (-1, 0, 1, p - 1):
        x = base + d
        x = x[(x >= 0) & (x < 2.0 ** 53)]
        want = np.array([int(v) % p for v in x], dtype=np.float64)
        assert np.array_equal(dmod(x, p), want)


# --------------------------------------- folded products of the triangular solve
# For p = 2^31 - k with k < 2^8, the solve adds fold(t) = k h + l for each
# product t = h 2^31 + l < 2^62 to a 64-bit accumulator (fold(t) == t mod p,
# fold(t) < 2^39 + 2^31) and reduces the accumulator once at the end; with at
# most 2^24 additions the accumulator stays below 2^64.

def fold(t, k):
    return k * (t >> 31) + (t & 0x7fffffff)


@pytest.mark.parametrize("p", [2147483647, 2147483629, 2147483587, 2147483579, 2147483563, 2147483549,
                               2147483543, 2147483497])
def test_pseudo_mersenne_fold(p):
    k = (1 << 31) - p
    assert 1 <= k < 256
    rng = np.random.default_rng(k)
    a = rng.integers(0, p, 500_000, dtype=np.uint64)
    b = rng.integers(1, p, 500_000, dtype=np.uint64)
    a[:1000], b[:1000] = p - 1, p - 1  # the largest product
    t = a * b  # < 2^62: exact in uint64
    f = fold(t, np.uint64(k))
    assert int(f.max()) < (1 << 39) + (1 << 31)
    assert np.array_equal(f % np.uint64(p), t % np.uint64(p))
    # the accumulator bound: 2^24 additions of the largest fold on top of a residue
    worst = (p - 1) + (1 << 24) * (k * ((p - 1) * (p - 1) >> 31) + 0x7fffffff)
    assert worst < 1 << 64
    # a long accumulation reduced once equals the sum of the exact residues
    acc = np.uint64(p - 1)
    chunk = f[:200_000]
    acc = int(acc) + int(chunk.astype(object).sum())
    assert acc < 1 << 64
    assert acc % p == (p - 1 + int((t[:200_000] % np.uint64(p)).astype(object).sum())) % p
