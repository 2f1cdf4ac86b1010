"""The GPU path's per-step shapes equal the stored oracle shapes of workloads
1 and 2 (tests/golden), exactly."""

import sys

import pytest

import synth
from test_golden import load

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", ["dense_n6", "dense_n10"])
def test_gpu_step_shapes_equal_golden(cfg):
    import paper_2601_06765_amd.f4 as f4
    n, p, polys = synth.system(cfg)
    print("[case] golden shapes, workload", cfg, flush=True)
    sys.stdout.flush()
    c = f4.Context(0)
    _, steps = c.groebner(p, n, polys)
    c.close()
    got = [(s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"], s["rho"]) for s in steps]
    assert got == load(cfg)
