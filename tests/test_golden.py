"""The stored step shapes (tests/golden/steps_dense_n*.txt, written by
tests/golden/make_golden.py from O1 alone): the oracle still produces them,
and they satisfy what the mathematics fixes for any F4 step: |T| <= N(n, d) =
C(n+d, d) (equation "monomial-count"), rank(A) = |pivot columns| + rank of
the reduced trailing block, rank(A) <= min(r, N), and each step's matrix has
at least as many nonzeros as rows (no zero rows)."""

import os
from math import comb

import pytest

import oracle
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(cfg):
    rows = []
    for line in open(os.path.join(HERE, "steps_%s.txt" % cfg)):
        if line.startswith("#") or not line.strip():
            continue
        rows.append(tuple(int(x) for x in line.split()))
    return rows


@pytest.mark.parametrize("cfg", ["dense_n6", "dense_n10"])
def test_golden_shapes_invariants_and_oracle(cfg):
    n, p, polys = synth.system(cfg)
    stored = load(cfg)
    assert stored
    for d, r, N, M, npiv, rank, rho in stored:
        assert N <= comb(n + d, d)
        assert rank == npiv + rho and rank <= min(r, N)
        assert M >= r and npiv <= r
    run = oracle.OracleRun(n, p, polys)
    live = [(s["d"], s["r"], s["N"], s["M"], s["npiv"], s["rank"], s["rho"]) for s in run.steps()]
    assert live == stored
