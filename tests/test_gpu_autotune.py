"""Schedules never change results: forced tile and radix schedules, and the
autotuner's measured picks, give bases and step shapes identical to the CPU
oracle's; the tuning table round-trips through its text form.

Every test prints its case before the device call.  Comparisons are exact.
"""

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


def canon(basis):
    out = []
    for f in basis:
        d = {tuple(e): c for e, c in f}
        out.append(tuple((e, d[e]) for e in sorted(d, key=bb.grevlex_key, reverse=True)))
    return tuple(out)


def shapes(steps):
    return [(s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"], s["rho"]) for s in steps]


def oracle_shapes(run):
    return [(s["d"], s["r"], s["N"], s["M"], s["npiv"], s["rank"], s["rho"]) for s in run.steps()]


@pytest.fixture(scope="module")
def dense_n10():
    n, p, polys = synth.system("dense_n10")
    run = oracle.OracleRun(n, p, polys)
    return n, p, polys, canon(run.basis()), oracle_shapes(run)


@pytest.mark.parametrize("rows", [1, 2, 3, 4])
def test_forced_trsm_rows(f4, dense_n10, rows):
    n, p, polys, want_b, want_s = dense_n10
    say("dense_n10 trsm_rows", rows)
    c = f4.Context(0, trsm_rows=rows)
    B, steps = c.groebner(p, n, polys)
    c.close()
    assert canon(B) == want_b and shapes(steps) == want_s


@pytest.mark.parametrize("bits", [1, 5, 6, 7])
def test_forced_radix_digits(f4, dense_n10, bits):
    # the radix dictionary sorts every generated key (hundreds of thousands,
    # multi-workgroup passes); row and emit sorts are single-workgroup
    n, p, polys, want_b, want_s = dense_n10
    say("dense_n10 radix dictionary, radix_bits", bits)
    c = f4.Context(0, dict_path="radix", radix_bits=bits)
    B, steps = c.groebner(p, n, polys)
    c.close()
    assert canon(B) == want_b and shapes(steps) == want_s


def test_autotuned_runs_and_table_round_trip(f4, dense_n10):
    n, p, polys, want_b, want_s = dense_n10
    say("dense_n10 autotune, radix dictionary")
    c = f4.Context(0, autotune=True, dict_path="radix")
    B, steps = c.groebner(p, n, polys)
    assert canon(B) == want_b and shapes(steps) == want_s
    text = c.tune_table()
    kinds = {ln.split()[0] for ln in text.splitlines()}
    assert kinds == {"trsm", "sort"}, text
    # a second run reuses the table (no new buckets) and gives the same result
    B2, steps2 = c.groebner(p, n, polys)
    assert canon(B2) == want_b and shapes(steps2) == want_s
    assert c.tune_table() == text
    c.close()
    say("dense_n10 imported table")
    d = f4.Context(0, autotune=True, dict_path="radix")
    d.load_tune_table(text)
    assert d.tune_table() == text
    B3, steps3 = d.groebner(p, n, polys)
    assert canon(B3) == want_b and shapes(steps3) == want_s
    assert d.tune_table() == text
    d.close()


def test_autotuned_sparse_large_prime(f4):
    # p = 2^31 - 1: the 64-bit accumulator class of the triangular solve
    n, p = 8, synth.P31
    polys = synth.sparse_quadratics(8, 9, 77, synth.P31 - 1, 12)
    run = oracle.OracleRun(n, p, polys)
    say("sparse n=8 p31 autotune")
    c = f4.Context(0, autotune=True)
    B, steps = c.groebner(p, n, polys)
    assert canon(B) == canon(run.basis()) and shapes(steps) == oracle_shapes(run)
    assert any(ln.startswith("trsm 0 ") for ln in c.tune_table().splitlines())
    c.close()


def test_tune_table_rejects_malformed_text(f4):
    say("tune table parsing")
    c = f4.Context(0)
    assert c.tune_table() == ""
    good = "trsm 1 10 11 2\nsort 1 13 21 7 8\n"
    c.load_tune_table(good)
    assert c.tune_table() == good
    for bad in ["trsm 1 10 11", "trsm 1 10 11 9", "sort 1 13 21 9 8", "sort 1 13 21 7 0", "tile 1 2 3 4",
                "trsm 1 10 11 2 extra"]:
        with pytest.raises(f4.F4Error) as e:
            c.load_tune_table(good + bad + "\n")
        assert e.value.code == f4.F4_E_ARG
        assert c.tune_table() == good
    c.close()
    with pytest.raises(f4.F4Error):
        f4.Context(0, trsm_rows=5)
    with pytest.raises(f4.F4Error):
        f4.Context(0, radix_bits=9)
