"""Pins of O8 (oracle/schedule.py), the block schedule of Pi and its
SELL-C-sigma storage: a hand-worked example
(tests/golden/block_schedule_small.txt), and on random and Macaulay matrices
the properties the readings fix, checked by brute force: the order is a
permutation; each panel holds exactly the rows whose leading column lies in
it (empty rows last); inside a panel, window q holds the rows of positions
q sigma .. q sigma + sigma - 1 in row order, longest first, ties by index;
slices are runs of C inside one panel with width their longest row; and the
SELL storage read back row by row is the CSR matrix (so a product with it is
the product with the matrix: checked against O5)."""

import os
import random

import numpy as np
import pytest

import synth
from oracle import krylov as o5
from oracle import schedule as o8

HERE = os.path.dirname(os.path.abspath(__file__))


def load_golden():
    rows, want = {}, {}
    for line in open(os.path.join(HERE, "golden", "block_schedule_small.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tag, *rest = line.split()
        v = [int(x) for x in rest]
        if tag == "row":
            rows[v[0]] = v[1:]
        else:
            want[tag] = v
    rp, ci, vv = [0], [], []
    for i in range(len(rows)):
        ci += rows[i]
        vv += [10 * i + k + 1 for k in range(len(rows[i]))]
        rp.append(len(ci))
    return rp, ci, vv, want


def test_golden_hand_example():
    rp, ci, vv, want = load_golden()
    s = o8.block_schedule(rp, ci, 10, 4, 2, 2)
    for key in ("perm", "panel_ptr", "slice_start", "slice_panel", "slice_width", "slice_off"):
        assert s[key] == want[key], key
    cols, vals = o8.sell_storage(rp, ci, vv, s, 2)
    assert cols == want["sell_col"] and vals == want["sell_val"]


def random_csr(r, N, seed, empty=0.05):
    rng = random.Random(seed)
    rp, ci, vv = [0], [], []
    for _ in range(r):
        k = 0 if rng.random() < empty else rng.randint(1, min(N, 12))
        cols = sorted(rng.sample(range(N), k))
        ci += cols
        vv += [rng.randint(1, 100) for _ in cols]
        rp.append(len(ci))
    return rp, ci, vv


def check_properties(rp, ci, vv, N, W, C, sigma):
    r = len(rp) - 1
    s = o8.block_schedule(rp, ci, N, W, C, sigma)
    perm, pp = s["perm"], s["panel_ptr"]
    assert sorted(perm) == list(range(r))
    length = [rp[i + 1] - rp[i] for i in range(r)]
    npan = s["npanels"]
    assert npan == max(1, -(-N // W)) and len(pp) == npan + 2
    for l in range(npan + 1):
        members = sorted(perm[pp[l]:pp[l + 1]])
        want = [i for i in range(r) if (ci[rp[i]] // W if length[i] else npan) == l]
        assert members == want
        for q in range(0, len(want), sigma):
            win = want[q:q + sigma]
            got = perm[pp[l] + q:pp[l] + q + len(win)]
            assert sorted(got) == win
            assert all((-length[a], a) < (-length[b], b) for a, b in zip(got, got[1:]))
    ends = list(s["slice_start"][1:]) + [r]
    for q, s0 in enumerate(s["slice_start"]):
        l = s["slice_panel"][q]
        assert pp[l] <= s0 < pp[l + 1] and (s0 - pp[l]) % C == 0
        s1 = min(s0 + C, pp[l + 1])
        assert ends[q] >= s1  # the next slice starts where this one ends (or in the next panel)
        assert s["slice_width"][q] == max(length[i] for i in perm[s0:s1])
        assert s["slice_off"][q + 1] - s["slice_off"][q] == C * s["slice_width"][q]
    cols, vals = o8.sell_storage(rp, ci, vv, s, C)
    # read back: every row's entries, in order, then padding only
    for q, s0 in enumerate(s["slice_start"]):
        l = s["slice_panel"][q]
        for j, i in enumerate(perm[s0:min(s0 + C, pp[l + 1])]):
            got = [(cols[s["slice_off"][q] + k * C + j], vals[s["slice_off"][q] + k * C + j])
                   for k in range(s["slice_width"][q])]
            assert got[:length[i]] == list(zip(ci[rp[i]:rp[i + 1]], vv[rp[i]:rp[i + 1]]))
            assert all(v == 0 for _, v in got[length[i]:])
    return s, cols, vals


@pytest.mark.parametrize("r,N,W,C,sigma,seed", [(50, 40, 8, 4, 4, 1), (200, 300, 64, 64, 128, 2),
                                                (120, 30, 7, 3, 5, 3), (64, 16, 100, 8, 1, 4)])
def test_random_properties(r, N, W, C, sigma, seed):
    check_properties(*random_csr(r, N, seed), N, W, C, sigma)


def test_macaulay_product_through_sell():
    n, p, polys = synth.system("dense_n6")
    import oracle
    rec = oracle.OracleRun(n, p, polys, record=-2).step_record(2)
    rp, ci, vv = [list(map(int, rec[k])) for k in ("row_ptr", "col_ind", "val")]
    N = len(rec["T"])
    s, cols, vals = check_properties(rp, ci, vv, N, 16, 8, 32)
    X = np.random.default_rng(5).integers(0, p, size=(N, 3))
    want = o5.spmm(rp, ci, vv, N, X, p)
    got = np.zeros_like(want)
    for q, s0 in enumerate(s["slice_start"]):
        l = s["slice_panel"][q]
        for j, i in enumerate(s["perm"][s0:min(s0 + 8, s["panel_ptr"][l + 1])]):
            acc = np.zeros(3, dtype=object)
            for k in range(s["slice_width"][q]):
                at = s["slice_off"][q] + k * 8 + j
                acc = acc + vals[at] * X[cols[at]].astype(object)
            got[i] = [int(a) % p for a in acc]
    assert np.array_equal(got, want)
