"""Two-word monomial keys on the host (f4_pack_mw / f4_unpack_mw, no GPU):
exact round trips, the order key (lanes complemented, read as a 128-bit
number) agreeing with grevlex as O2 writes it (a sort key of its own) on
random pairs, distinct monomials never sharing a key (the key refines the
order), and the product being the word-wise sum.  The lane positions are
read off the packed unit vectors, not taken from the library's layout code."""

import random

import pytest

from oracle import buchberger as bb

pytestmark = []


@pytest.fixture(scope="module")
def f4():
    import paper_2601_06765_amd.f4 as mod
    return mod


def lane_mask(f4, n):
    w = f4._lib.f4_mw_lane_bits(n)
    mask = 0
    for v in range(n):
        e = [0] * n
        e[v] = 1
        hi, lo = f4.pack_mw(n, e)
        x = ((hi << 64) | lo) - (1 << 120)  # drop the degree byte (degree 1)
        assert x and x & (x - 1) == 0  # one bit: the lane's lowest
        mask |= ((1 << w) - 1) * x
    return w, mask


def key(words, mask):
    return ((words[0] << 64) | words[1]) ^ mask


def rand_mono(rng, n, w, dmax):
    e = [0] * n
    for _ in range(rng.randint(0, dmax)):
        v = rng.randrange(n)
        if e[v] + 1 < (1 << w):
            e[v] += 1
    return tuple(e)


@pytest.mark.parametrize("n", [1, 7, 15, 16, 17, 19, 20, 23, 24, 30])
def test_pack_order_and_product(f4, n):
    rng = random.Random(n)
    w, mask = lane_mask(f4, n)
    assert (w == 8) == (n <= 15) and w >= 4
    mons = list({rand_mono(rng, n, w, 9) for _ in range(400)})
    packed = {m: f4.pack_mw(n, m) for m in mons}
    for m, p in packed.items():
        assert f4.unpack_mw(n, p) == m
        assert p[0] >> 56 == sum(m)
    keys = {key(p, mask) for p in packed.values()}
    assert len(keys) == len(mons)
    for _ in range(3000):
        a, b = rng.choice(mons), rng.choice(mons)
        assert (key(packed[a], mask) > key(packed[b], mask)) == (bb.grevlex_key(a) > bb.grevlex_key(b))
        if all(x + y < (1 << w) for x, y in zip(a, b)) and sum(a) + sum(b) < 256:
            s = f4.pack_mw(n, tuple(x + y for x, y in zip(a, b)))
            assert s == ((packed[a][0] + packed[b][0]) & (2 ** 64 - 1), (packed[a][1] + packed[b][1]) & (2 ** 64 - 1))


def test_lane_widths_and_ranges(f4):
    assert [f4._lib.f4_mw_lane_bits(n) for n in (0, 1, 15, 16, 17, 18, 19, 20, 23, 24, 30, 31)] == \
        [0, 8, 8, 7, 7, 6, 6, 5, 5, 4, 4, 0]
    with pytest.raises(f4.F4Error):
        f4.pack_mw(24, [16] + [0] * 23)  # 4-bit lanes
    with pytest.raises(f4.F4Error):
        f4.pack_mw(31, [0] * 31)
