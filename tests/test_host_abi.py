"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side monomial encoding matches the term order.
No device call is made here."""

import itertools
import math
import os
import re

import pytest

from oracle import buchberger as bb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def f4():
    lib = os.path.join(ROOT, "paper_2601_06765_amd", "libf4.so")
    if not os.path.exists(lib):
        import paper_2601_06765_amd.build as b
        b.build()
    import paper_2601_06765_amd.f4 as mod
    return mod


def declared_functions():
    text = open(os.path.join(ROOT, "include", "f4.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|uint32_t|const char\*)\s+(f4_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(f4):
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(f4._lib, name), name


def test_pack_roundtrip_and_range(f4):
    for n in range(1, 15):
        w = f4.lane_bits(n)
        assert w == min(8, 56 // n)
        e = tuple((i * 3) % (1 << w) for i in range(n))
        if sum(e) <= 255:
            assert f4.unpack(n, f4.pack(n, e)) == e
    with pytest.raises(f4.F4Error) as ei:
        f4.pack(14, tuple([16] + [0] * 13))  # 4-bit lanes
    assert ei.value.code == f4.F4_E_RANGE
    assert f4.lane_bits(0) == 0 and f4.lane_bits(15) == 0


def monomials_upto(n, D):
    out = []
    for e in itertools.product(range(D + 1), repeat=n):
        if sum(e) <= D:
            out.append(e)
    return out


@pytest.mark.parametrize("n,D", [(1, 4), (2, 5), (3, 4), (4, 4), (5, 3), (6, 3)])
def test_dense_rank_is_grevlex_position(f4, n, D):
    mons = sorted(monomials_upto(n, D), key=bb.grevlex_key, reverse=True)
    assert len(mons) == math.comb(n + D, D)
    for pos, e in enumerate(mons):
        w = f4.pack(n, e)
        assert f4.grevlex_rank(n, D, w) == pos
        assert f4.grevlex_unrank(n, D, pos) == w


def test_dense_rank_large_n_samples(f4):
    # n = 14 at D = 5: check order preservation on a few hundred pairs
    import random
    rng = random.Random(5)
    n, D = 14, 5
    mons = []
    for _ in range(300):
        e = [0] * n
        for _ in range(rng.randint(0, D)):
            e[rng.randrange(n)] += 1
        mons.append(tuple(e))
    for a, b in zip(mons, mons[1:]):
        ra, rb = (f4.grevlex_rank(n, D, f4.pack(n, x)) for x in (a, b))
        ka, kb = bb.grevlex_key(a), bb.grevlex_key(b)
        assert (ra < rb) == (ka > kb) and (ra == rb) == (a == b)
        assert f4.unpack(n, f4.grevlex_unrank(n, D, ra)) == a


@pytest.mark.parametrize("n", [1, 3, 6, 10, 14])
def test_vectorised_packing_matches_the_library(f4, n):
    """The binding's bulk packer gives the library's words (f4_pack), and the
    same range errors."""
    import numpy as np
    rng = np.random.default_rng(100 + n)
    w = f4.lane_bits(n)
    exps = rng.integers(0, min(1 << w, 256 // n + 1), size=(200, n))
    exps = exps[exps.sum(axis=1) <= 255]
    got = f4.pack_many(n, exps)
    assert [int(x) for x in got] == [f4.pack(n, tuple(int(v) for v in e)) for e in exps]
    with pytest.raises(f4.F4Error) as e:
        f4.pack_many(n, [[1 << w] + [0] * (n - 1)])
    assert e.value.code == f4.F4_E_RANGE
    polys = [[(tuple(int(v) for v in exps[i]), i + 1) for i in range(k, k + 5)] for k in (0, 5, 10)]
    mon, coeff, off = f4.polys_to_arrays(n, polys, sort=True)
    assert off.tolist() == [0, 5, 10, 15]
    for a, f in enumerate(polys):
        want = sorted(((f4.pack(n, e), c) for e, c in f), key=lambda t: t[0] ^ ((1 << (n * w)) - 1),
                      reverse=True)
        got_a = list(zip(mon[5 * a:5 * a + 5].tolist(), coeff[5 * a:5 * a + 5].tolist()))
        assert got_a == [(int(m), int(c)) for m, c in want]
