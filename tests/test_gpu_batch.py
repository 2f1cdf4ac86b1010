"""Batched F4 (many systems per launch sequence): every system's result in the
batch equals its result alone and the oracle's, exactly."""

import sys

import pytest

import oracle
import synth
from oracle import buchberger as bb

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def f4():
    import paper_2601_06765_amd.f4 as mod
    return mod


@pytest.fixture(scope="module")
def ctx(f4):
    c = f4.Context(0)
    yield c
    c.close()


def canon(basis):
    out = []
    for f in basis:
        d = {tuple(e): c for e, c in f}
        out.append(tuple((e, d[e]) for e in sorted(d, key=bb.grevlex_key, reverse=True)))
    return tuple(out)


def shapes_of(steps):
    return [(s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"], s["rho"]) for s in steps]


def oracle_shapes(run):
    return [(s["d"], s["r"], s["N"], s["M"], s["npiv"], s["rank"], s["rho"]) for s in run.steps()]


def mixed_systems():
    """Uneven sizes, mixed primes, trivial and non-trivial bases."""
    out = []
    for n, p, polys in synth.batch_systems(6):
        out.append((p, n, polys))
    polys, _ = synth.planted_system(5, 6, 65521, 31)
    out.append((65521, 5, polys))
    out.append((2147483647, 4, synth.random_system(4, 4, 2147483647, 32)))
    out.append((31, 3, synth.random_system(3, 3, 31, 33, density=0.6)))
    n, polys = synth.crt_system()
    for p in synth.CRT_PRIMES[:3]:
        out.append((p, n, synth.reduce_coeffs(polys, p)))
    out.append((65521, 3, [[((1, 0, 0), 1)], [((0, 0, 0), 7)]]))  # unit ideal from the input
    out.append((65521, 2, [[((2, 0), 3), ((0, 1), 1)]]))          # single polynomial, no pairs
    return out


def test_batch_equals_alone_and_oracle(f4, ctx):
    systems = mixed_systems()
    say("batch of", len(systems))
    batch = ctx.groebner_batch(systems)
    assert len(batch) == len(systems)
    for (p, n, polys), (B, steps) in zip(systems, batch):
        say("alone n=%d p=%d" % (n, p))
        B1, steps1 = ctx.groebner(p, n, polys)
        assert canon(B) == canon(B1)
        assert shapes_of(steps) == shapes_of(steps1)
        run = oracle.OracleRun(n, p, polys)
        assert canon(B) == canon(run.basis())
        assert shapes_of(steps) == oracle_shapes(run)


def test_batch_of_one_and_repeat(f4, ctx):
    n, p, polys = synth.system("dense_n6")
    say("batch of 1 x2")
    a = ctx.groebner_batch([(p, n, polys)])
    b = ctx.groebner_batch([(p, n, polys)])
    assert canon(a[0][0]) == canon(b[0][0])
    assert shapes_of(a[0][1]) == shapes_of(b[0][1])
    assert canon(a[0][0]) == canon(oracle.OracleRun(n, p, polys).basis())


def test_batch_workload_sample_radix_dictionary(f4):
    c = f4.Context(0, dict_path="radix")
    try:
        systems = [(p, n, polys) for n, p, polys in synth.batch_systems(5)]
        say("batch radix of", len(systems))
        batch = c.groebner_batch(systems)
        for (p, n, polys), (B, steps) in zip(systems, batch):
            run = oracle.OracleRun(n, p, polys)
            assert canon(B) == canon(run.basis())
            assert shapes_of(steps) == oracle_shapes(run)
    finally:
        c.close()


def test_batch_workload_sample_and_all_crt_primes(f4, ctx):
    """One batch holding two systems of each n = 6..9 of the batch workload
    (seeds 4*2^32 + j) and the workload's n = 9 system under all 8 CRT primes:
    every basis and every step's shapes equal the oracle's."""
    sample, seen = [], {}
    for j, (n, p, polys) in enumerate(synth.batch_systems(256)):
        if seen.get(n, 0) < 2:
            seen[n] = seen.get(n, 0) + 1
            sample.append((j, p, n, polys))
    assert sorted(seen) == [6, 7, 8, 9]
    n9, polys9 = synth.crt_system()
    systems = [(p, n, polys) for _, p, n, polys in sample]
    systems += [(q, n9, synth.reduce_coeffs(polys9, q)) for q in synth.CRT_PRIMES]
    say("batch: workload sample", [j for j, _, _, _ in sample], "+ 8 CRT primes")
    batch = ctx.groebner_batch(systems)
    for (p, n, polys), (B, steps) in zip(systems, batch):
        say("oracle n=%d p=%d" % (n, p))
        run = oracle.OracleRun(n, p, polys)
        assert canon(B) == canon(run.basis())
        assert shapes_of(steps) == oracle_shapes(run)
