"""Host pair-set logic: the fast Gebauer-Moeller insertion against the generic
one along leading-monomial sequences produced by the oracle (section "Pair
management and the normal strategy").  The replay program is host code only;
the selections it makes at step boundaries must match the oracle's counts."""

import os
import shutil
import subprocess

import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("gm") / "gm_replay")
    src = os.path.join(ROOT, "tests", "host", "gm_replay.hip")
    subprocess.run([HIPCC, "-O2", "-std=c++17", src, "-o", out], check=True, capture_output=True)
    return out


def insertion_sequence(n, p, polys):
    """Leading monomials in insertion order with the step boundaries."""
    run = oracle.OracleRun(n, p, polys, record=-2)
    lines = ["%d" % n]
    prev = 0
    last = None
    for k in range(len(run.steps())):
        rec = run.step_record(k)
        G = rec["G"]
        for f in G[prev:]:
            lines.append("I " + " ".join(map(str, f[0][0])))
        prev = len(G)
        lines.append("S %d %d" % (rec["d"], len(rec["sel"])))
        last = rec
    T, rp, rc = last["T"], last["rref_ptr"], last["rref_col"]
    for a in range(len(rp) - 1):
        lines.append("I " + " ".join(map(str, T[rc[rp[a]]])))
    return "\n".join(lines) + "\n"


CASES = {
    "dense_n6": lambda: synth.system("dense_n6"),
    "dense_n7": lambda: (7, synth.P16, synth.dense_quadratics(7, 8, 11, synth.P16 - 1)),
    "dense_n8_p31": lambda: (8, synth.P31, synth.dense_quadratics(8, 9, 12, synth.P31 - 1)),
    "sparse_n9": lambda: (9, synth.P16, synth.sparse_quadratics(9, 10, 13, synth.P16 - 1, 12)),
    "underdetermined_n6": lambda: (6, synth.P16, synth.dense_quadratics(6, 4, 14, synth.P16 - 1)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fast_insertion_matches_generic(replay, tmp_path, case):
    n, p, polys = CASES[case]()
    seq = tmp_path / "seq.txt"
    seq.write_text(insertion_sequence(n, p, polys))
    r = subprocess.run([replay, str(seq)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
