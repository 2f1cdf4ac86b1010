"""Writes the stored step shapes of the dense n=6 and n=10 systems from the CPU oracle O1
(and nothing else): one line per F4 step,
    d r N M npiv rank rho
the step degree, rows, dictionary size |T|, nonzeros, pivot columns, rank of
A and rank of the reduced trailing block (Definition "Symbolic preprocessing
operator", Algorithm "FBSP", section "PSGE"), under the readings R1-R3 of
the reducer, row-order and pivot-row rules.  Run from the repository root:
    python3 tests/golden/make_golden.py
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def shapes(cfg):
    n, p, polys = synth.system(cfg)
    run = oracle.OracleRun(n, p, polys)
    return [(s["d"], s["r"], s["N"], s["M"], s["npiv"], s["rank"], s["rho"]) for s in run.steps()]


def main():
    for cfg in ("dense_n6", "dense_n10"):
        path = os.path.join(HERE, "steps_%s.txt" % cfg)
        with open(path, "w") as f:
            f.write("# F4 step shapes of the %s system from the CPU oracle O1 (tests/golden/make_golden.py)\n" % cfg)
            f.write("# d r N M npiv rank rho\n")
            for row in shapes(cfg):
                f.write(" ".join(str(x) for x in row) + "\n")


if __name__ == "__main__":
    main()
