"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side monomial encoding matches the term order.
No device call is made here."""

import itertools
import math
import os
import re

import numpy as np
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
    mon, coeff, off = f4.polys_to_arrays(n, polys)
    assert off.tolist() == [0, 5, 10, 15]
    assert [int(x) for x in mon] == [f4.pack(n, e) for f in polys for e, _ in f]


@pytest.mark.parametrize("n,p", [(3, 7), (6, 65521), (14, 2147483647)])
def test_normalize_polys(f4, n, p):
    """f4_normalize_polys against a plain normalisation with O2's grevlex key:
    terms sorted largest first, repeated monomials merged mod p, zero terms
    dropped, and with monic=True divided by the leading coefficient."""
    import random
    rnd = random.Random(n * 1000 + p % 997)
    mons = [tuple(rnd.randrange(0, 3) for _ in range(n)) for _ in range(12)]
    polys = [[(rnd.choice(mons), rnd.randrange(0, min(3 * p, 1 << 32))) for _ in range(rnd.randrange(1, 15))]
             for _ in range(6)]
    polys.append([(mons[0], 1), (mons[0], p - 1)])  # cancels to zero
    for monic in (False, True):
        got = f4.normalize(p, n, polys, monic=monic)
        want = []
        for f in polys:
            acc = {}
            for e, c in f:
                acc[e] = (acc.get(e, 0) + c) % p
            g = sorted(((e, c) for e, c in acc.items() if c), key=lambda t: bb.grevlex_key(t[0]), reverse=True)
            if not g:
                continue
            if monic:
                inv = pow(g[0][1], p - 2, p)
                g = [(e, c * inv % p) for e, c in g]
            want.append(g)
        assert got == want


def test_check_polys_rejects_malformed_input(f4):
    """The input contract of the matrix builders (F4_E_ARG with the failed
    rule): unsorted terms, repeated terms, a zero or too large coefficient, a
    non-monic element when monic input is required, a word whose lanes do not
    add up to its degree field, an empty polynomial."""
    n, p = 4, 65521
    good = f4.normalize(p, n, [[((1, 0, 0, 1), 5), ((0, 1, 0, 0), 3), ((0, 0, 0, 0), 2)],
                               [((0, 2, 0, 0), 1), ((1, 0, 0, 0), 7)]], monic=True)
    mon, coeff, off = f4.polys_to_arrays(n, good)
    assert f4.check_arrays(p, n, mon, coeff, off, monic=True) == (f4.F4_OK, 0)

    def bits(m, c, o, monic=False):
        rc, b = f4.check_arrays(p, n, m, c, o, monic=monic)
        assert rc == (f4.F4_E_ARG if b else f4.F4_OK)
        return b

    sw = mon.copy()
    sw[[0, 1]] = sw[[1, 0]]
    assert bits(sw, coeff, off) & 2  # unsorted
    rep = mon.copy()
    rep[1] = rep[0]
    assert bits(rep, coeff, off) & 2  # repeated
    for bad in (0, p, p + 5):
        cf = coeff.copy()
        cf[2] = bad
        assert bits(mon, cf, off) & 4  # coefficient not in [1, p)
    cf = coeff.copy()
    cf[0] = 2
    assert bits(mon, cf, off, monic=True) & 8 and bits(mon, cf, off) == 0  # non-monic
    w = f4.lane_bits(n)
    word = mon.copy()
    word[0] = int(word[0]) + (1 << w)  # an exponent more than the degree field says
    assert bits(word, coeff, off) & 1
    assert bits(mon, coeff, np.array([0, 3, 3, 5], dtype=np.uint64)) & 16  # empty polynomial