"""Benchmark of the F4 reduction step over F_p on one MI355X, through the C-ABI.

Headline ("step" of this benchmark): the first degree-5 F4 step of 15 sparse
random quadratics in n=14 variables over F_(2^31-1) (20 monomials each,
grevlex, seed 3): symbolic preprocessing of its Macaulay matrix
(r = 7 169 rows, N = 9 482 columns, 3.28 million nonzeros) and its
elimination mod p.  value = nnz(A) / (t_DictBuild + t_RowAssemble +
t_NumericCore), the stage times of that step from HIP events on the
library's stream, median over the timed runs (each run repeats the steps of
lower degree untimed, to reach the step with its real basis).  The oracle
(textbook F4, one host thread) on the same step is the CPU baseline.

Secondary legs: full F4 runs of the n=10, m=12 dense system (nnz/s over all
steps), the batched and served forms against the plain one-system-at-a-time
path (systems/s), the block operator application of the Krylov branch, and
the modular inner-loop microbenchmark.

Prints one JSON line (rank 0, N=1).  `--gpus N` with N > 1 exits: this
build measures one GPU.
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SELL_W, SELL_SIGMA = 4096, 64  # block schedule of the operator: panel width, window of the length sort
# derived modular-product bound: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz integer
# issue, at least two instructions (a multiply and an add) per modular product
MODMUL_PEAK = 256 * 4 * 16 * 2.4e9 / 2
VALU_ISSUE = 256 * 4 * 16 * 2.4e9  # vector lane-instructions per second
STEP_DEG = 5  # the timed step of the headline workload
BATCH_RUNS = 5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed runs of the headline step (median reported)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-batch-systems", type=int, default=64,
                    help="batch systems the oracle solves for the batch baseline (0: skip)")
    ap.add_argument("--cpu-workers", type=int, default=16, help="host processes of the batch baseline")
    ap.add_argument("--dict", choices=["rank", "radix"], default=None)
    ap.add_argument("--full-runs", type=int, default=20, help="timed full F4 runs of the n=10 system (0: skip)")
    ap.add_argument("--batch-systems", type=int, default=256, help="systems in the batched leg (0: skip)")
    ap.add_argument("--crt", type=int, default=1, help="run the 8-prime CRT leg (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window of the serving leg (0: skip)")
    ap.add_argument("--serve-light-rate", type=float, default=60.0,
                    help="arrival rate of a second serving run below the service's throughput (0: skip)")
    ap.add_argument("--modloop-chains", type=int, default=1 << 21,
                    help="chains of the modular inner-loop microbenchmark (0: skip)")
    ap.add_argument("--modloop-iters", type=int, default=4096)
    ap.add_argument("--spmm-shift-deg", type=int, default=8,
                    help="shift degree of the Macaulay operator of the SpMM leg (0: skip)")
    ap.add_argument("--wiedemann-shift-deg", type=int, default=3,
                    help="shift degree of the Macaulay matrix of the block Wiedemann leg (-1: skip)")
    ap.add_argument("--sig-shift-deg", type=int, default=8,
                    help="shift degree of the rows of the signature-filter leg (0: skip)")
    ap.add_argument("--mw-vars", type=int, default=20,
                    help="variables of the two-word-key Macaulay leg (0: skip)")
    ap.add_argument("--mw-shift-deg", type=int, default=5, help="shift degree of that leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed schedules instead of the autotuner's measured picks (tuned during warm-up)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (reference kernel for HBM byte counters)")
    ap.add_argument("--step-only", action="store_true", help="only the headline step (for profiling runs)")
    return ap.parse_args()


def calibrate_copy(mib):
    """A plain device-to-device copy of known size: under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE per dispatch give the counters' scale."""
    import torch
    n = mib << 20
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 5}))


KERNEL_FILES = {"k_ech_block": "reduce.hip", "k_trsm": "reduce.hip"}
KERNEL_HEADS = {
    "k_ech_block": "__global__ __launch_bounds__(1024) void k_ech_block(",
    "k_trsm": "__global__ __launch_bounds__(TR_THREADS) void k_trsm(",
}


def kernel_fingerprint(kernel):
    """SHA-1 of the kernel's source text (its function plus csrc/common.hpp):
    counters taken on another version do not apply."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2601_06765_amd", "csrc")
    src = open(os.path.join(csrc, KERNEL_FILES[kernel])).read()
    a = src.index(KERNEL_HEADS[kernel])
    b = src.index("\n}\n", a)
    common = open(os.path.join(csrc, "common.hpp")).read()
    return hashlib.sha1((src[a:b] + common).encode()).hexdigest()


def recorded_traffic(kernel, summary):
    """HBM bytes per launch of `kernel` from a committed counter summary under
    profiles/, or None when it has none for the kernel or the kernel's source
    has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    value, sha = None, None
    try:
        for line in open(path):
            f = line.split()
            if len(f) == 3 and f[1] == kernel and f[0] == "traffic_bytes_per_launch":
                value = float(f[2])
            if len(f) == 3 and f[1] == kernel and f[0] == "kernel_source_sha1":
                sha = f[2]
    except OSError:
        return None
    if value is None or sha != kernel_fingerprint(kernel):
        return None
    return value


def step_bytes(s):
    """Algorithmic HBM bytes of one F4 step (unit: one nonzero of A).  Build:
    the CSR written once (u32 column + u32 value per nonzero), 16 B of row
    pointer and row metadata per row, the 8-byte dictionary; elimination: the
    CSR read once, the reduced trailing block D' written once (L x c words)
    and its echelon rows (rho x c words)."""
    c = s["N"] - s["npivot"]
    build = 8 * s["nnz"] + 16 * s["r"] + 8 * s["N"]
    reduce = 8 * s["nnz"] + 4 * s["r"] + 4 * s["lower"] * c + 4 * s["rho"] * c
    trsm = 8 * s["nnz"] + 4 * s["r"] + 4 * s["lower"] * c
    return build, reduce, trsm


def trsm_instr_per_product(p):
    """Fewest vector instructions per modular product of the triangular
    solve's arithmetic class: p < 2^16, the one-word Barrett product (multiply,
    high multiply, multiply, subtract, min: 5); p = 2^31 - k with k < 2^8, the
    fold k h + l of the 64-bit product (low and high multiply, shift, mask,
    multiply-add: 5); any other p, the two-word Barrett product (12)."""
    if p < 65536:
        return 5
    if p > (1 << 31) - 256:
        return 5
    return 12


def roofline_of(kstats, step, e3_peak, p):
    """Roofline of the dominant elimination kernel of the timed step (largest
    summed launch time, HIP events around each launch on the library's stream).
    Both candidates are bound by vector-integer arithmetic (their algorithmic
    bytes are far below what HBM moves in their time).  Triangular solve:
    achieved = its modular products / its launch time, against the integer
    issue rate divided by the fewest instructions per product of its
    arithmetic class (its HBM view, algorithmic bytes over time, is reported
    beside it).  Echelon block step: the same products against the rate the
    inner-loop microbenchmark measures for its arithmetic form."""
    cand = {
        "k_trsm": (sum(s["t_k_trsm_ms"] for s in kstats), sum(s["trsm_ops"] for s in kstats),
                   sum(s["n_k_trsm"] for s in kstats)),
        "k_ech_block": (sum(s["t_k_block_ms"] for s in kstats), sum(s["block_ops"] for s in kstats),
                        sum(s["n_k_block"] for s in kstats)),
    }
    name = max(cand, key=lambda k: cand[k][0])
    ms, ops, launches = cand[name]
    runs = len(kstats)
    per = ms / max(1, launches)
    traffic = recorded_traffic(name, "hbm_counters_n14_step.md")
    other = {k: {"ms_per_run": round(v[0] / runs, 4), "launches_per_run": v[2] / runs,
                 "modmul_per_run": v[1] / runs,
                 "Tmodmul_per_s": round(v[1] / (v[0] / 1e3) / 1e12, 4) if v[0] else None}
             for k, v in cand.items()}
    if name == "k_trsm":
        # bound by vector-integer issue (the counters show the vector ALUs busy
        # most of the kernel): achieved = its modular products / its launch time,
        # against the issue rate of the fewest instructions its arithmetic class
        # needs per product
        _, _, tb = step_bytes(step)
        byts = tb / max(1, launches / runs)
        achieved = ops / (ms / 1e3) / 1e12 if ms > 0 else 0.0
        ipp = trsm_instr_per_product(p)
        peak = VALU_ISSUE / ipp / 1e12
        return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(peak, 4), "unit": "Tmodmul/s",
                "frac": round(achieved / peak, 5), "traffic": traffic, "kernel": name,
                "peak_source": "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz integer issue / %d instructions per "
                               "product (the arithmetic class of the solve for this p)" % ipp,
                "ops_per_launch": ops / max(1, launches), "ms_per_launch": round(per, 5),
                "hbm_view": {"alg_bytes_per_launch": byts, "achieved_GBs": round(byts / (per / 1e3) / 1e9, 2),
                             "frac_of_8TBs": round(byts / (per / 1e3) / 1e9 / HBM_PEAK_GBS, 6)},
                "kernels": other}
    achieved = ops / (ms / 1e3) / 1e12 if ms > 0 else 0.0
    return {"bound": "alu", "achieved": round(achieved, 5), "peak": e3_peak, "unit": "Tmodmul/s",
            "frac": round(achieved / e3_peak, 6) if e3_peak else None, "traffic": traffic, "kernel": name,
            "peak_source": "modular inner-loop microbenchmark, measured in this run",
            "ms_per_launch": round(per, 5), "ops_per_launch": ops / max(1, launches), "kernels": other}


def headline_leg(f4, torch, steps, warmup, autotune, dict_path):
    """The timed step: F4 on the n=14 sparse system up to and including its
    first degree-5 step; stage times of that step from HIP events (median over
    `steps` runs), then the same runs with HIP events around every launch of the
    elimination kernels (roofline), and the autotuner's table."""
    import synth
    n, p, polys = synth.system("sparse_n14")
    ctx = f4.Context(0, timing=True, stop_deg=STEP_DEG, autotune=autotune, dict_path=dict_path)
    prep = ctx.prepare(p, n, polys)
    for _ in range(warmup):
        ctx.groebner_prepared(prep)
    torch.cuda.synchronize()
    runs, walls = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        _, st = ctx.groebner_prepared(prep)
        walls.append(time.perf_counter() - t1)
        runs.append(st[-1])
    torch.cuda.synchronize()
    timed_s = time.perf_counter() - t0
    table = ctx.tune_table()
    ctx.close()
    kctx = f4.Context(0, kernel_timing=True, stop_deg=STEP_DEG, autotune=autotune, dict_path=dict_path)
    kctx.load_tune_table(table)
    prep = kctx.prepare(p, n, polys)
    kctx.groebner_prepared(prep)
    kstats = [kctx.groebner_prepared(prep)[1][-1] for _ in range(steps)]
    kctx.close()
    s = runs[0]
    assert s["deg"] == STEP_DEG, "the run did not reach a degree-%d step" % STEP_DEG
    tot = [r["t_dict_ms"] + r["t_assemble_ms"] + r["t_numeric_ms"] for r in runs]
    med = statistics.median(tot)
    mid = lambda key: statistics.median(r[key] for r in runs)
    build, reduce, _ = step_bytes(s)
    return {
        "n": n, "p": p, "m": len(polys), "step": s, "ms": med, "timed_s": timed_s, "table": table,
        "kstats": kstats,
        "stages": {"t_dict_ms": round(mid("t_dict_ms"), 4), "t_assemble_ms": round(mid("t_assemble_ms"), 4),
                   "t_numeric_ms": round(mid("t_numeric_ms"), 4), "t_trsm_ms": round(mid("t_trsm_ms"), 4),
                   "t_echelon_ms": round(mid("t_echelon_ms"), 4),
                   "t_preprocess_ms": round(mid("t_dict_ms") + mid("t_assemble_ms"), 4),
                   "stage_sum_min_ms": round(min(tot), 4), "stage_sum_max_ms": round(max(tot), 4),
                   "host_wall_of_step_ms": round(mid("t_step_ms"), 4),
                   "run_to_step_wall_ms": round(1e3 * statistics.median(walls), 3)},
        "hbm_alg": {"build_bytes": build, "reduce_bytes": reduce,
                    "frac_of_8TBs": (build + reduce) / (med / 1e3) / (HBM_PEAK_GBS * 1e9),
                    "preprocess_frac": build / (((mid("t_dict_ms") + mid("t_assemble_ms")) / 1e3)
                                                * HBM_PEAK_GBS * 1e9)},
    }


def cpu_baseline_step(n, p, polys, nnz):
    """The oracle as it is (textbook F4, one host thread) run up to and
    including the same degree-5 step; value = nnz of that step / the oracle's
    own build + reduce time of the step."""
    import oracle
    t0 = time.perf_counter()
    run = oracle.OracleRun(n, p, polys, stop_deg=STEP_DEG)
    dt = time.perf_counter() - t0
    st = run.steps()[-1]
    assert st["d"] == STEP_DEG and st["M"] == nnz, "oracle step differs from the GPU step"
    tb, tr = run.times_ns()[-1]
    step_s = (tb + tr) * 1e-9
    return {"value": nnz / step_s, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": "one oracle run to the first degree-5 step of the n=14 sparse system (%.1f s in all); "
                      "that step's build %.2f s + elimination %.2f s, single thread" % (dt, tb * 1e-9, tr * 1e-9)}


def _oracle_basis(job):
    """One oracle Groebner basis (a worker of the batch baseline)."""
    import oracle
    n, p, polys = job
    oracle.OracleRun(n, p, polys).basis()
    return n


def cpu_baseline_batch(count, workers):
    """The oracle on the batch workload's first `count` systems (the same
    n ~ U{6..9} dense systems as the batched leg), one process per host core
    up to `workers`: systems per second of wall time."""
    import multiprocessing as mp
    import synth
    jobs = [(n, p, polys) for n, p, polys in synth.batch_systems(count)]
    cores = max(1, min(workers, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        sizes = pool.map(_oracle_basis, jobs, chunksize=1)
    dt = time.perf_counter() - t0
    return {"value": len(jobs) / dt, "unit": "systems/s", "cores": cores, "kind": "oracle",
            "sample": "the first %d systems of the batch workload (n = 6..9: %s), %.1f s of wall time" %
                      (len(jobs), "/".join(str(sizes.count(k)) for k in (6, 7, 8, 9)), dt)}


def full_f4_leg(f4, torch, runs, warmup, autotune, dict_path):
    """Full F4 runs of the n=10, m=12 dense quadratics over F_65521 (seed 2):
    nnz/s over all steps of a run, and the per-step stage times."""
    import synth
    n, p, polys = synth.system("dense_n10")
    ctx = f4.Context(0, dict_path=dict_path, autotune=autotune)
    prep = ctx.prepare(p, n, polys)
    for _ in range(warmup):
        ctx.groebner_prepared(prep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        basis, _ = ctx.groebner_prepared(prep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    table = ctx.tune_table()
    ctx.close()
    assert basis == [[((0,) * n, 1)]], "unexpected basis"
    ictx = f4.Context(0, timing=True, dict_path=dict_path, autotune=autotune)
    ictx.load_tune_table(table)
    prep = ictx.prepare(p, n, polys)
    ictx.groebner_prepared(prep)
    allsteps = [ictx.groebner_prepared(prep)[1] for _ in range(runs)]
    ictx.close()
    nnz_run = sum(s["nnz"] for s in allsteps[0])
    per_step = []
    for k in range(len(allsteps[0])):
        s0 = allsteps[0][k]
        mid = lambda key: statistics.median(run[k][key] for run in allsteps)
        gpu_ms = mid("t_dict_ms") + mid("t_assemble_ms") + mid("t_numeric_ms")
        build, reduce, _ = step_bytes(s0)
        per_step.append({"deg": s0["deg"], "r": s0["r"], "N": s0["N"], "nnz": s0["nnz"], "npivot": s0["npivot"],
                         "lower": s0["lower"], "rho": s0["rho"], "t_dict_ms": round(mid("t_dict_ms"), 4),
                         "t_assemble_ms": round(mid("t_assemble_ms"), 4),
                         "t_numeric_ms": round(mid("t_numeric_ms"), 4), "t_trsm_ms": round(mid("t_trsm_ms"), 4),
                         "t_echelon_ms": round(mid("t_echelon_ms"), 4),
                         "t_pairs_host_ms": round(mid("t_pairs_ms"), 4),
                         "nnz_per_s_gpu": s0["nnz"] / (gpu_ms / 1e3) if gpu_ms > 0 else None,
                         "hbm_frac_alg": (build + reduce) / (gpu_ms / 1e3) / (HBM_PEAK_GBS * 1e9)
                         if gpu_ms > 0 else None})
    return {"workload": "full F4, n=10, m=12 dense quadratics over F_65521, grevlex, normal strategy (seed 2)",
            "runs": runs, "f4_steps": len(allsteps[0]), "nnz_per_run": nnz_run, "ms_per_run": dt * 1e3 / runs,
            "nnz_per_s": nnz_run * runs / dt, "systems_per_s_plain": runs / dt, "per_f4_step": per_step}


def spmm_leg(f4, shift_deg, b, reps):
    """Block operator application of the Krylov solvers (Y = A X, Y = A^T X)
    on the Macaulay matrix of the sparse n=14 system's input: rows t*f_i for every monomial
    t of degree <= shift_deg and each of the 15 sparse quadratics over
    F_(2^31-1), built by the symbolic preprocessing; b random vectors.  Each
    product is timed with HIP events on the stream it runs on (the library's
    timed call: mean of `reps` after a warm-up that also builds the transpose)."""
    import numpy as np
    import synth
    n, p, polys = synth.system("sparse_n14")
    polys = f4.normalize(p, n, polys)
    t = f4.pack_many(n, synth.monomials_upto(n, shift_deg))
    ctx = f4.Context(0)
    tw, ks = np.repeat(t, len(polys)), np.tile(np.arange(len(polys), dtype=np.uint32), len(t))
    A = ctx.build_matrix_rows_packed(p, n, polys, tw, ks)  # warm-up build
    A.free()
    t0 = time.perf_counter()
    A = ctx.build_matrix_rows_packed(p, n, polys, tw, ks)
    ctx.download(A.view.row_ptr, 1, np.uint32)  # waits for the build's stream
    t_build = time.perf_counter() - t0
    r, N, nnz = A.view.r, A.view.N, A.view.nnz
    rng = np.random.default_rng(7)
    X = ctx.to_device(rng.integers(0, p, size=(N, b), dtype=np.int64))
    W = ctx.to_device(rng.integers(0, p, size=(r, b), dtype=np.int64))
    Y, YT = ctx.device_array((r, b)), ctx.device_array((N, b))
    res = {"workload": "Macaulay matrix of the n=14 sparse quadratics (15 x 20 terms, F_(2^31-1), seed 3), "
                       "shifts of degree <= %d; b = %d random vectors" % (shift_deg, b),
           "r": r, "N": N, "nnz": nnz, "b": b,
           # symbolic preprocessing of the same operator (f4_build_matrix_rows, wall clock including
           # its host-side row planning): algorithmic bytes 8 nnz + 16 r + 8 N (CSR out, row metadata, dictionary)
           "build_ms": round(t_build * 1e3, 3), "build_nnz_per_s": nnz / t_build,
           "build_alg_GBs": round((8 * nnz + 16 * r + 8 * N) / t_build / 1e9, 1)}
    for name, trans, src, dst, nout in (("ax", False, X, Y, r), ("atx", True, W, YT, N)):
        ctx.spmm(p, A, src, trans=trans, out=dst)  # warm-up (builds the transpose once)
        _, ms = ctx.spmm_timed(p, A, src, trans=trans, out=dst, reps=reps)
        nin = N if not trans else r
        byts = 4 * (nout + 1) + 8 * nnz + 4 * b * (nin + nout)  # pointers, entries, X once, Y once
        gbs = byts / (ms * 1e-3) / 1e9
        gather = 4 * b * nnz  # every stored entry gathers its b words of X (cache traffic beyond the first touch)
        res[name] = {"ms": round(ms, 4), "alg_bytes": byts, "achieved_GBs": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "gather_bytes": gather,
                     "with_gathers_GBs": round((byts - 4 * b * nin + gather) / (ms * 1e-3) / 1e9, 1),
                     "entries_x_vectors_per_s": nnz * b / (ms * 1e-3)}
    for d in (X, W, Y, YT):
        d.free()
    # other block widths, A X only: b = 1 (the scalar Wiedemann product) and 32
    res["ax_other_b"] = {}
    for bb in (1, 32):
        Xb = ctx.to_device(rng.integers(0, p, size=(N, bb), dtype=np.int64))
        Yb = ctx.device_array((r, bb))
        ctx.spmm(p, A, Xb, out=Yb)
        _, ms = ctx.spmm_timed(p, A, Xb, out=Yb, reps=reps)
        byts = 4 * (r + 1) + 8 * nnz + 4 * bb * (N + r)
        res["ax_other_b"][str(bb)] = {"ms": round(ms, 4), "achieved_GBs": round(byts / (ms * 1e-3) / 1e9, 1),
                                      "frac_hbm": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                      "entries_x_vectors_per_s": nnz * bb / (ms * 1e-3)}
        Xb.free()
        Yb.free()
    # the block schedule of the same operator (panels of SELL_W columns, slices of
    # 64 rows, windows of SELL_SIGMA rows) and A X through its padded slices
    t0 = time.perf_counter()
    v = ctx.schedule_build(A, SELL_W, 64, SELL_SIGMA)
    ctx.download(A.view.row_ptr, 1, np.uint32)  # waits for the schedule's stream
    t_sched = time.perf_counter() - t0
    res["sell"] = {"W": SELL_W, "C": 64, "sigma": SELL_SIGMA, "npanels": v["npanels"], "nslices": v["nslices"],
                   "padded": v["padded"], "pad_ratio": round(v["padded"] / max(1, nnz), 4),
                   "schedule_ms": round(t_sched * 1e3, 3)}
    for bb in (1, 8):
        Xb = ctx.to_device(rng.integers(0, p, size=(N, bb), dtype=np.int64))
        Yb = ctx.device_array((r, bb))
        ctx.spmm_sell(p, A, Xb, out=Yb)
        _, ms = ctx.spmm_sell_timed(p, A, Xb, out=Yb, reps=reps)
        _, ms_csr = ctx.spmm_timed(p, A, Xb, out=Yb, reps=reps)
        # slice table (start, panel, width: 3 words, offset: 2), perm, padded entries, X once, Y once
        byts = 20 * v["nslices"] + 4 * r + 8 * v["padded"] + 4 * bb * (N + r)
        res["sell"]["ax_b%d" % bb] = {"ms": round(ms, 4), "csr_ms": round(ms_csr, 4),
                                      "achieved_GBs": round(byts / (ms * 1e-3) / 1e9, 1),
                                      "frac_hbm": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                      "entries_x_vectors_per_s": nnz * bb / (ms * 1e-3)}
        Xb.free()
        Yb.free()
    A.free()
    ctx.close()
    return res




def wiedemann_leg(f4, shift_deg, b):
    """Block Wiedemann (left-kernel vectors = syzygies) on the Macaulay matrix of
    the sparse n=14 system's input at degree shift_deg + 2: rows t*f_i for every monomial t
    of degree <= shift_deg and each of the 15 sparse quadratics over
    F_(2^31-1), built by the symbolic preprocessing; the diagonal D and the
    blocks X, Y from splitmix64 (seed 6).  Reports the three phases' times
    and the vectors found (each checked on the device against A^T v = 0)."""
    import numpy as np
    import synth
    n, p, polys = synth.system("sparse_n14")
    polys = f4.normalize(p, n, polys)
    t = f4.pack_many(n, synth.monomials_upto(n, shift_deg))
    tw, ks = np.repeat(t, len(polys)), np.tile(np.arange(len(polys), dtype=np.uint32), len(t))
    ctx = f4.Context(0)
    A = ctx.build_matrix_rows_packed(p, n, polys, tw, ks)
    r, N, nnz = A.view.r, A.view.N, A.view.nnz
    d = ctx.to_device(synth.residues(p, N, 6 * 2**32 + 0) % (p - 1) + 1)
    X = ctx.to_device(synth.residues(p, r * b, 6 * 2**32 + 1).reshape(r, b))
    Y = ctx.to_device(synth.residues(p, r * b, 6 * 2**32 + 2).reshape(r, b))
    ctx.block_wiedemann(p, A, d, X, Y)  # warm-up (transpose, code objects)
    t0 = time.perf_counter()
    vecs, st = ctx.block_wiedemann(p, A, d, X, Y)
    wall = time.perf_counter() - t0
    for a in (d, X, Y, A):
        a.free()
    ctx.close()
    L = st["L"]
    # each sequence term applies A^T and A to b vectors: 2 nnz b products
    return {"workload": "degree-%d Macaulay matrix of the n=14 sparse quadratics (F_(2^31-1)): r = %d, N = %d, "
                        "%d nonzeros; b = %d" % (shift_deg + 2, r, N, nnz, b),
            "r": r, "N": N, "nnz": nnz, "b": b, "L": L, "generators": st["generators"], "vectors": len(vecs),
            "wall_ms": round(wall * 1e3, 2), "t_sequence_ms": round(st["t_sequence_ms"], 2),
            "t_mbasis_ms": round(st["t_mbasis_ms"], 2), "t_vectors_ms": round(st["t_vectors_ms"], 2),
            "sequence_entry_vector_products_per_s": 2.0 * nnz * b * L / (st["t_sequence_ms"] * 1e-3)}


def signature_leg(f4, shift_deg, build_shift_deg, reps):
    """Signature admissibility in bulk on the sparse n=14 system's input (the 15 sparse
    quadratics in n=14 over F_(2^31-1)): f_i carries the signature 1 e_i and
    index i lists the principal syzygies LM(f_j), j < i, so the filter is the
    F5 syzygy criterion.  (1) f4_sig_filter over the Macaulay rows t*f_i for
    every t of degree <= shift_deg: device time (HIP events around predicate,
    scan, compaction; with the bucketed schedule separately), rows/s and
    algorithmic bytes (read t and k, 12 B a row; write the flag, 1 B, and each
    kept row, 12 B).  (2) f4_build_matrix_sig on the rows of degree <=
    build_shift_deg + 2 against f4_build_matrix_rows of the same rows:
    rows, nonzeros and device time of both."""
    import numpy as np
    import synth
    n, p, polys = synth.system("sparse_n14")
    G = f4.normalize(p, n, polys, monic=True)
    m = len(G)
    lms = [tuple(g[0][0]) for g in G]
    syz = [[lms[j] for j in range(i)] for i in range(m)]
    sidx, smon = list(range(m)), [(0,) * n] * m
    ctx = f4.Context(0)
    sg = ctx._sigs(n, sidx, smon, syz)
    t = f4.pack_many(n, synth.monomials_upto(n, shift_deg))
    tw, ks = np.repeat(t, m), np.tile(np.arange(m, dtype=np.uint32), len(t))
    r = len(tw)
    res = {"workload": "F5 syzygy criterion on the Macaulay rows t*f_i of the n=14 sparse quadratics "
                       "(15 x 20 terms, F_(2^31-1), seed 3), deg t <= %d; signatures 1 e_i, principal "
                       "syzygies" % shift_deg, "rows": r}
    for name, sched in (("filter", False), ("filter_and_schedule", True)):
        ctx.sig_filter_packed(p, n, G, sg, tw, ks, schedule=sched)  # warm-up
        ms = []
        for _ in range(reps):
            flags, nk, _, st = ctx.sig_filter_packed(p, n, G, sg, tw, ks, schedule=sched)
            ms.append(st["t_device_ms"])
        med = statistics.median(ms)
        byts = 12 * r + r + 12 * nk
        res[name] = {"device_ms": round(med, 4), "rows_per_s": r / (med * 1e-3),
                     "alg_bytes": byts, "alg_GBs": round(byts / (med * 1e-3) / 1e9, 1),
                     "frac_hbm": round(byts / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "kept": nk, "syzygy": st["syzygy"], "rewritten": st["rewritten"]}
    # (2) the closure over admissible reducers on a smaller matrix
    t2 = synth.monomials_upto(n, build_shift_deg)
    rows = [(tuple(int(x) for x in e), k) for e in t2 for k in range(m)]
    A, st = ctx.build_matrix_sig(p, n, G, [1] * m, sidx, smon, syz, rows)
    A.free()
    A, st = ctx.build_matrix_sig(p, n, G, [1] * m, sidx, smon, syz, rows)
    sig_view = (A.view.r, A.view.N, A.view.nnz)
    A.free()
    B = ctx.build_matrix_rows(p, n, G, rows)
    B.free()
    t0 = time.perf_counter()
    B = ctx.build_matrix_rows(p, n, G, rows)
    ctx.download(B.view.row_ptr, 1, np.uint32)
    t_plain = time.perf_counter() - t0
    res["build"] = {"rows_in": len(rows), "deg": build_shift_deg + 2,
                    "sig": {"r": sig_view[0], "N": sig_view[1], "nnz": sig_view[2],
                            "rejected_syzygy": st["syzygy"], "device_ms": round(st["t_device_ms"], 4)},
                    "plain": {"r": B.view.r, "N": B.view.N, "nnz": B.view.nnz, "wall_ms": round(t_plain * 1e3, 3)}}
    B.free()
    ctx.close()
    return res


def multiword_leg(f4, n, shift_deg, reps):
    """Two-word monomial keys (f4_build_matrix_rows_mw): the Macaulay matrix of
    n+1 sparse quadratics in n > 14 variables (20 terms each, F_65521, seeded)
    with rows t*f_i for every t of degree <= shift_deg; wall time of the call
    after a warm-up (median of `reps`), nonzeros per second and algorithmic
    bytes (8 nnz for the CSR out, 24 r for the row records in and the row
    metadata out, 16 N for the dictionary), then A X on 8 vectors with the
    resulting handle (HIP events)."""
    import numpy as np
    import synth
    p = 65521
    G = f4.normalize_mw(p, n, synth.sparse_quadratics(n, n + 1, 11, p - 1, 20))
    m = len(G)
    t = f4.pack_many_mw(n, synth.monomials_upto(n, shift_deg))
    tw = np.repeat(t, m, axis=0)
    ks = np.tile(np.arange(m, dtype=np.uint32), len(t))
    ctx = f4.Context(0)
    A = ctx.build_matrix_rows_mw_packed(p, n, G, tw, ks)
    A.free()
    walls = []
    for _ in range(reps):
        t0 = time.perf_counter()
        A = ctx.build_matrix_rows_mw_packed(p, n, G, tw, ks)
        ctx.download(A.view.row_ptr, 1, np.uint32)
        walls.append(time.perf_counter() - t0)
        r, N, nnz = A.view.r, A.view.N, A.view.nnz
        A.free()
    w = statistics.median(walls)
    A = ctx.build_matrix_rows_mw_packed(p, n, G, tw, ks)
    rng = np.random.default_rng(3)
    X = ctx.to_device(rng.integers(0, p, size=(N, 8), dtype=np.int64))
    Y = ctx.device_array((r, 8))
    ctx.spmm(p, A, X, out=Y)
    _, ms = ctx.spmm_timed(p, A, X, out=Y, reps=10)
    X.free()
    Y.free()
    A.free()
    ctx.close()
    byts = 8 * nnz + 24 * r + 16 * N
    return {"workload": "Macaulay matrix of %d sparse quadratics (20 terms each, F_65521, seed 11) in n=%d "
                        "variables (two-word keys, %d-bit lanes), shifts of degree <= %d"
                        % (m, n, f4._lib.f4_mw_lane_bits(n), shift_deg),
            "r": r, "N": N, "nnz": nnz, "build_wall_ms": round(w * 1e3, 3), "build_nnz_per_s": nnz / w,
            "build_alg_GBs": round(byts / w / 1e9, 1), "ax_b8_ms": round(ms, 4)}


def modloop_leg(f4, nchains, iters):
    """Modular inner-loop microbenchmark (randomized residues, seed 5): the
    update rate of each arithmetic form, its registers and spill bytes per
    lane, and the rate as a fraction of the derived modular-product peak."""
    import synth
    res = {"workload": "%d chains x %d updates x <- b + x*a mod p, uniform residues (splitmix64 seed 5)"
                       % (nchains, iters), "forms": []}
    cases = [("mul24", synth.P16), ("barrett32", synth.P16), ("barrett64", synth.P16), ("barrett64", synth.P31),
             ("montgomery", synth.P16), ("montgomery", synth.P31)]
    ctx = f4.Context(0)
    for form, p in cases:
        x0, a, b = (synth.residues(p, nchains, 5 * 2**32 + k) for k in range(3))
        _, st = ctx.modloop(p, form, x0, a, b, iters)
        res["forms"].append({"form": form, "p": p, "updates_per_s": st["updates_per_s"],
                             "kernel_ms": round(st["kernel_ms"], 4), "regs": st["regs"],
                             "private_bytes": st["private_bytes"],
                             "frac_of_peak": round(st["updates_per_s"] / MODMUL_PEAK, 4)})
    ctx.close()
    return res


def same_bases(a, b):
    return [x[0] for x in a] == [y[0] for y in b]


def batch_leg(f4, torch, count, autotune):
    """The batch workload: `count` independent systems (n ~ U{6..9}, m = n+1 dense,
    F_65521): one f4_groebner_batch call vs the same systems one by one; every
    batched basis must equal its one-by-one basis (the bench fails otherwise)."""
    import synth
    ctx = f4.Context(0, autotune=autotune)
    systems = [(p, n, polys) for n, p, polys in synth.batch_systems(count)]
    prep = ctx.prepare_batch(systems)
    ctx.groebner_batch_prepared(prep)  # warm-up
    torch.cuda.synchronize()
    tbs = []
    for _ in range(BATCH_RUNS):
        t0 = time.perf_counter()
        res = ctx.groebner_batch_prepared(prep)
        torch.cuda.synchronize()
        tbs.append(time.perf_counter() - t0)
    tb = statistics.median(tbs)
    preps = [ctx.prepare(p, n, polys) for p, n, polys in systems]  # marshalled once, as for the batch
    t0 = time.perf_counter()
    plain = [ctx.groebner_prepared(q) for q in preps]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    ctx.close()
    bad = [j for j in range(count) if res[j][0] != plain[j][0]]
    if bad:
        raise SystemExit("batched bases differ from the one-by-one bases for systems %s" % bad[:10])
    nnz = sum(s["nnz"] for _, steps in res for s in steps)
    return {"workload": "%d dense systems, n ~ U{6..9}, m = n+1, F_65521 (seeds 4*2^32+j)" % count,
            "systems": count, "batched_s": tb, "batched_s_min": min(tbs),
            "stat": "batched: median of %d runs after a warm-up; plain: one pass" % BATCH_RUNS, "plain_s": tp,
            "systems_per_s_batched": count / tb, "systems_per_s_plain": count / tp,
            "speedup": tp / tb, "nnz_total": nnz, "nnz_per_s_batched": nnz / tb,
            "checked": "all %d batched bases equal their one-by-one bases" % count}


def crt_leg(f4, torch, autotune):
    """The CRT part of the batch workload: one n=9 dense system read modulo the 8 largest
    primes below 2^31, as one batch of 8 against 8 plain runs; bases compared."""
    import synth
    n, polys = synth.crt_system()
    systems = [(q, n, polys) for q in synth.CRT_PRIMES]
    ctx = f4.Context(0, autotune=autotune)
    prep = ctx.prepare_batch(systems)
    ctx.groebner_batch_prepared(prep)
    torch.cuda.synchronize()
    tbs = []
    for _ in range(BATCH_RUNS):
        t0 = time.perf_counter()
        res = ctx.groebner_batch_prepared(prep)
        torch.cuda.synchronize()
        tbs.append(time.perf_counter() - t0)
    tb = statistics.median(tbs)
    preps = [ctx.prepare(q, n, polys) for q, n, polys in systems]
    t0 = time.perf_counter()
    plain = [ctx.groebner_prepared(q) for q in preps]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    ctx.close()
    if not same_bases(res, plain):
        raise SystemExit("CRT batch bases differ from the plain runs")
    return {"workload": "one n=9, m=10 dense system under the 8 largest primes below 2^31",
            "systems": len(systems), "stat": "batched: median of %d runs after a warm-up" % BATCH_RUNS,
            "systems_per_s_batched": len(systems) / tb,
            "systems_per_s_plain": len(systems) / tp, "speedup": tp / tb,
            "nnz_total": sum(s["nnz"] for _, st in res for s in st)}


def serve_leg(f4, ctx, seconds, rate=500.0):
    """The serving workload: Poisson arrivals (500/s) of systems n ~ U{5..12}, p from
    {65521, 2^31-1}.  The continuous-batching server (admission by estimated
    device footprint) against a plain FIFO that runs f4_groebner per request,
    both on this GPU, on the same stream; latency = completion - arrival.
    At 500/s both saturate (the latencies grow with the window); a lower
    `rate`, below both throughputs, gives the latencies of the service
    itself."""
    import synth
    stream = synth.serve_stream(rate=rate, duration=seconds)
    preps = [f4.Server.prepare(p, n, polys) for _, n, p, polys in stream]
    arrivals = [t for t, _, _, _ in stream]

    def pct(xs, q):
        xs = sorted(xs)
        return xs[min(len(xs) - 1, int(q * len(xs)))]

    # served: admit arrivals whose time has come, step, poll
    srv = f4.Server(ctx, hbm_budget=64 << 30, max_slots=512)
    lat, tickets, nxt, done = [], {}, 0, 0
    t0 = time.perf_counter()
    while done < len(preps):
        now = time.perf_counter() - t0
        while nxt < len(preps) and arrivals[nxt] <= now:
            t = srv.submit_prepared(preps[nxt])
            if t is None:
                break
            tickets[t] = nxt
            nxt += 1
        if tickets:
            srv.step()
        elif nxt < len(preps):
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
        now = time.perf_counter() - t0
        for t in list(tickets):
            if srv.poll(t) is not None:
                lat.append(now - arrivals[tickets.pop(t)])
                done += 1
    served_s = time.perf_counter() - t0
    srv.close()
    # plain: one request at a time in arrival order (inputs marshalled
    # beforehand, as for the server)
    pprep = [ctx.prepare(p, n, polys) for _, n, p, polys in stream]
    plat = []
    t0 = time.perf_counter()
    for i in range(len(stream)):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        ctx.groebner_prepared(pprep[i])
        plat.append(time.perf_counter() - t0 - arrivals[i])
    plain_s = time.perf_counter() - t0
    return {"workload": "Poisson %g/s for %.1f s: %d requests, n ~ U{5..12}, p in {65521, 2^31-1}" %
                        (rate, seconds, len(stream)),
            "requests": len(stream),
            "served_systems_per_s": len(stream) / served_s,
            "served_p50_s": pct(lat, 0.50), "served_p99_s": pct(lat, 0.99),
            "plain_systems_per_s": len(stream) / plain_s,
            "plain_p50_s": pct(plat, 0.50), "plain_p99_s": pct(plat, 0.99)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (this build has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    import torch
    import paper_2601_06765_amd.f4 as f4

    torch.cuda.init()
    tune = not args.no_autotune
    h = headline_leg(f4, torch, args.steps, args.warmup, tune, args.dict)
    s = h["step"]
    out = {
        "metric": "Macaulay nnz/s built+reduced per F4 step; systems/sec batched vs plain",
        "value": s["nnz"] / (h["ms"] / 1e3),
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded sparse random quadratics, splitmix64 seed 3)",
        "config": {"workload": "first degree-5 F4 step of 15 sparse random quadratics (20 monomials each) "
                               "in n=14 variables over F_(2^31-1), grevlex",
                   "n": h["n"], "m": h["m"], "p": h["p"], "deg": s["deg"], "r": s["r"], "N": s["N"],
                   "nnz": s["nnz"], "npivot": s["npivot"], "lower": s["lower"], "rho": s["rho"],
                   "rank": s["rank"], "dict_path": args.dict or "auto"},
        "rows_per_s": s["r"] / (h["ms"] / 1e3),
        "stat": "median of %d runs of the step (stage times from HIP events)" % args.steps,
        "stages": h["stages"],
        "hbm_alg": h["hbm_alg"],
        "autotune": {"on": tune, "table": h["table"].splitlines()},
    }
    e3 = None
    if args.modloop_chains and not args.step_only:
        out["modloop"] = modloop_leg(f4, args.modloop_chains, args.modloop_iters)
        # the echelon's large-prime form (two-word Barrett) at the workload's prime
        f = [x for x in out["modloop"]["forms"] if x["form"] == "barrett64" and x["p"] == h["p"]]
        e3 = round(f[0]["updates_per_s"] / 1e12, 4) if f else None
    out["roofline"] = roofline_of(h["kstats"], s, e3, h["p"])
    if not args.step_only:
        if args.full_runs:
            out["full_f4_n10"] = full_f4_leg(f4, torch, args.full_runs, args.warmup, tune, args.dict)
        if args.spmm_shift_deg:
            out["spmm"] = spmm_leg(f4, args.spmm_shift_deg, 8, 20)
        if args.wiedemann_shift_deg >= 0:
            out["block_wiedemann"] = wiedemann_leg(f4, args.wiedemann_shift_deg, 8)
        if args.sig_shift_deg:
            out["signatures"] = signature_leg(f4, args.sig_shift_deg, 3, 5)
        if args.mw_vars:
            out["multiword"] = multiword_leg(f4, args.mw_vars, args.mw_shift_deg, 5)
        if args.batch_systems:
            out["batch"] = batch_leg(f4, torch, args.batch_systems, tune)
            out["systems_per_s_batched"] = out["batch"]["systems_per_s_batched"]
            out["systems_per_s_plain"] = out["batch"]["systems_per_s_plain"]
        if args.crt:
            out["crt"] = crt_leg(f4, torch, tune)
        if args.serve_seconds > 0:
            sctx = f4.Context(0, autotune=tune)
            out["serve"] = serve_leg(f4, sctx, args.serve_seconds)
            if args.serve_light_rate > 0:
                out["serve_below_capacity"] = serve_leg(f4, sctx, args.serve_seconds, args.serve_light_rate)
            sctx.close()
    if not args.no_cpu_baseline:
        import synth
        n, p, polys = synth.system("sparse_n14")
        out["cpu_baseline"] = cpu_baseline_step(n, p, polys, s["nnz"])
        if args.batch_systems and args.cpu_batch_systems:
            # the batch metric's host reference, in the same leg (a process pool)
            out["cpu_baseline"]["batch"] = cpu_baseline_batch(min(args.batch_systems, args.cpu_batch_systems),
                                                              args.cpu_workers)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
