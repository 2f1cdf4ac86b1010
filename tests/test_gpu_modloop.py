"""The modular inner-loop microbenchmark's kernels against O4: every form
gives, chain by chain, exactly the residues of the iterated definition, for
chain counts that leave a ragged last workgroup and for the largest and
smallest primes each form accepts.  Bad arguments give F4_E_ARG before any
launch.  Every test prints its case before the device call."""

import sys

import numpy as np
import pytest

import synth
from oracle import modloop as o4

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_06765_amd.f4 as mod
    c = mod.Context(0)
    yield c
    c.close()


CASES = [("mul24", 65521), ("mul24", 3), ("mul24", 257), ("barrett32", 65521), ("barrett32", 3),
         ("barrett64", 65521), ("barrett64", synth.P31), ("barrett64", 3),
         ("montgomery", 65521), ("montgomery", synth.P31), ("montgomery", 3)]


@pytest.mark.parametrize("form,p", CASES)
@pytest.mark.parametrize("nchains", [1, 1029, 4096 + 777])
def test_modloop_matches_definition(ctx, form, p, nchains):
    iters = 75
    x0, a, b = (synth.residues(p, nchains, 1000 * k + nchains) for k in (1, 2, 3))
    a[: min(3, nchains)] = [0, 1, p - 1][: min(3, nchains)]
    say("modloop", form, "p", p, "chains", nchains, "iters", iters)
    got, st = ctx.modloop(p, form, x0, a, b, iters)
    want = o4.chains(p, x0, a, b, iters)
    assert np.array_equal(got.astype(np.int64), want)
    assert st["kernel_ms"] > 0 and st["updates_per_s"] > 0 and st["private_bytes"] == 0


def test_modloop_rejects_bad_arguments(ctx):
    import paper_2601_06765_amd.f4 as mod
    say("modloop argument checks")
    v = np.ones(8, dtype=np.uint32)
    bad = [(65537, "mul24", v), (65537, "barrett32", v), (65521 * 3, "barrett64", v), (4, "montgomery", v),
           (7, "barrett64", np.full(8, 7, dtype=np.uint32))]
    for p, form, arr in bad:
        with pytest.raises(mod.F4Error) as e:
            ctx.modloop(p, form, arr, v, v, 10)
        assert e.value.code == mod.F4_E_ARG
    with pytest.raises(mod.F4Error) as e:
        ctx.modloop(7, "barrett64", v, v, v, 0)
    assert e.value.code == mod.F4_E_ARG
    with pytest.raises(mod.F4Error) as e:
        ctx.modloop(7, "barrett64", v[:0], v[:0], v[:0], 5)
    assert e.value.code == mod.F4_E_ARG
