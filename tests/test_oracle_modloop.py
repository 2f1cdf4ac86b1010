"""Pins of O4, the modular inner loop (x <- b + x*a mod p, iterated), against
its closed form: after t updates
    x_t = a^t x_0 + b (a^t - 1) / (a - 1)   (a != 1),   x_t = x_0 + t b   (a = 1),
evaluated with modular powers and an inverse, not by iterating.  A swapped
operand, a dropped addend or an off-by-one in the count changes x_t."""

import numpy as np
import pytest

import synth
from oracle import modloop


def closed(p, x0, a, b, t):
    if a % p == 1:
        return (x0 + t * b) % p
    at = pow(a, t, p)
    return (at * x0 + b * (at - 1) * pow(a - 1, -1, p)) % p


@pytest.mark.parametrize("p", [3, 7, 257, 65521, synth.P31])
@pytest.mark.parametrize("iters", [0, 1, 2, 37])
def test_chains_closed_form(p, iters):
    n = 300
    x0, a, b = (synth.residues(p, n, 10 * k + iters) for k in (1, 2, 3))
    # the special multipliers 0, 1 and p - 1 on the first chains
    a[:3] = [0, 1, p - 1]
    got = modloop.chains(p, x0, a, b, iters)
    want = [closed(p, int(x0[i]), int(a[i]), int(b[i]), iters) for i in range(n)]
    assert [int(v) for v in got] == want


def test_chains_brute_force_tiny():
    # every (x0, a, b) over F_5, three updates, by repeated Python arithmetic
    p = 5
    pts = [(x, a, b) for x in range(p) for a in range(p) for b in range(p)]
    x0, a, b = (np.array(v) for v in zip(*pts))
    got = modloop.chains(p, x0, a, b, 3)
    for (x, aa, bb), g in zip(pts, got):
        for _ in range(3):
            x = (bb + x * aa) % p
        assert g == x
