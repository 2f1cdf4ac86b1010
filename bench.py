"""Benchmark: full F4 runs of the n=10, m=12 dense quadratic system over
F_65521 (grevlex, seed 2) through the C-ABI on one MI355X.

One "step" of this benchmark is one complete pass of the hot path over one
system: every F4 reduction step (symbolic preprocessing + elimination mod p)
until the reduced Groebner basis is known.  The headline value is Macaulay
nnz built+reduced per second: the sum over F4 steps of nnz(A) divided by the
wall time of the run.  Per-degree figures use the HIP-event stage times.

Prints one JSON line (rank 0, N=1).  `--gpus N` with N > 1 exits: this
build measures one GPU.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dict", choices=["rank", "radix"], default=None)
    ap.add_argument("--batch-systems", type=int, default=256, help="systems in the batched leg (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window of the serving leg (0: skip)")
    ap.add_argument("--sparse-repeats", type=int, default=3, help="timed runs of the n=14 sparse step (0: skip)")
    ap.add_argument("--modloop-chains", type=int, default=1 << 21,
                    help="chains of the modular inner-loop microbenchmark (0: skip)")
    ap.add_argument("--modloop-iters", type=int, default=4096)
    ap.add_argument("--spmm-shift-deg", type=int, default=8,
                    help="shift degree of the Macaulay operator of the SpMM leg (0: skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed schedules instead of the autotuner's measured picks (tuned during warm-up)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (reference kernel for HBM byte counters)")
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


# int32 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# a modular product needs at least a 24-bit multiply and an add (reductions
# amortised over lazy accumulation)
MODMUL_PEAK = VALU_OPS_PER_S / 2


KERNEL_HEADS = {
    "k_ech_block": "__global__ __launch_bounds__(1024) void k_ech_block(",
    "k_trsm": "__global__ __launch_bounds__(TR_THREADS) void k_trsm(",
}


def kernel_fingerprint(kernel):
    """SHA-1 of the kernel's source text (its function in csrc/reduce.hip plus
    csrc/common.hpp): counters taken on another version do not apply."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2601_06765_amd", "csrc")
    src = open(os.path.join(csrc, "reduce.hip")).read()
    a = src.index(KERNEL_HEADS[kernel])
    b = src.index("\n}\n", a)
    common = open(os.path.join(csrc, "common.hpp")).read()
    return hashlib.sha1((src[a:b] + common).encode()).hexdigest()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/hbm_counters_n10.md), or None when it has none for the kernel
    or the kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_counters_n10.md")
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


def roofline_of(allsteps):
    """Roofline of the kernel with the largest total time over the timed runs
    (HIP events around each launch): the triangular solve or the echelon block
    step, both bound by integer vector arithmetic.  achieved = modular products
    the kernel performed / its summed launch time."""
    cand = {
        "k_trsm": (sum(s["t_k_trsm_ms"] for run in allsteps for s in run),
                   sum(s["trsm_ops"] for run in allsteps for s in run),
                   sum(s["n_k_trsm"] for run in allsteps for s in run)),
        "k_ech_block": (sum(s["t_k_block_ms"] for run in allsteps for s in run),
                        sum(s["block_ops"] for run in allsteps for s in run),
                        sum(s["n_k_block"] for run in allsteps for s in run)),
    }
    name = max(cand, key=lambda k: cand[k][0])
    ms, ops, launches = cand[name]
    achieved = ops / (ms / 1000.0) / 1e12 if ms > 0 else 0.0
    peak = MODMUL_PEAK / 1e12
    traffic = recorded_traffic(name)
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(peak, 3), "unit": "Tmodmul/s",
            "frac": round(achieved / peak, 5), "traffic": traffic, "kernel": name,
            "launches_per_run": launches / len(allsteps), "ms_per_launch": ms / max(1, launches),
            "ops_per_launch": ops / max(1, launches),
            "other_kernel_ms_per_run": {k: round(v[0] / len(allsteps), 4) for k, v in cand.items()}}


def cpu_baseline(n, p, polys, seconds):
    """The oracle as it is (textbook F4, one thread) on whole runs of the same system."""
    import oracle
    t0 = time.perf_counter()
    runs, nnz = 0, 0
    while True:
        run = oracle.OracleRun(n, p, polys)
        nnz += sum(s["M"] for s in run.steps())
        runs += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": nnz / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": "%d full F4 run(s) of the same n=10 m=12 system, single thread, %.1f s" % (runs, dt)}


def sparse_step_leg(f4, repeats, autotune):
    """Workload 3: 15 sparse quadratics in n=14 over F_(2^31-1) (20 monomials
    each, seed 3); F4 on the GPU up to and including the first step of degree
    5, whose preprocessing (DictBuild + RowAssemble) and elimination
    (NumericCore) are reported separately."""
    import synth
    n, p, polys = synth.config_system(3)
    ctx = f4.Context(0, timing=True, stop_deg=5, autotune=autotune)
    ctx.groebner(p, n, polys)  # warm-up (and tuning)
    runs = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        _, steps = ctx.groebner(p, n, polys)
        runs.append((time.perf_counter() - t0, steps[-1]))
    ctx.close()
    s = runs[0][1]
    avg = lambda key: sum(r[1][key] for r in runs) / len(runs)
    sp = avg("t_dict_ms") + avg("t_assemble_ms")
    el = avg("t_numeric_ms")
    return {"workload": "n=14, m=15 sparse quadratics (20 monomials), F_(2^31-1), seed 3: first degree-5 step",
            "deg": s["deg"], "r": s["r"], "N": s["N"], "nnz": s["nnz"], "npivot": s["npivot"],
            "lower": s["lower"], "rho": s["rho"],
            "t_preprocess_ms": round(sp, 4), "t_elimination_ms": round(el, 4),
            "t_trsm_ms": round(avg("t_trsm_ms"), 4), "t_echelon_ms": round(avg("t_echelon_ms"), 4),
            "nnz_per_s_preprocess": s["nnz"] / (sp / 1000.0), "nnz_per_s_step": s["nnz"] / ((sp + el) / 1000.0),
            "rows_per_s_step": s["r"] / ((sp + el) / 1000.0),
            "run_to_step_ms": round(1000.0 * sum(r[0] for r in runs) / len(runs), 3)}


def spmm_leg(f4, shift_deg, b, reps):
    """Block operator application of the Krylov solvers (Y = A X, Y = A^T X)
    on the Macaulay matrix of workload 3's input: rows t*f_i for every monomial
    t of degree <= shift_deg and each of the 15 sparse quadratics over
    F_(2^31-1), built by the symbolic preprocessing; b random vectors.  Each
    product is timed with HIP events on the stream it runs on (the library's
    timed call: mean of `reps` after a warm-up that also builds the transpose)."""
    import numpy as np
    import synth
    n, p, polys = synth.config_system(3)
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
    A.free()
    ctx.close()
    return res


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


def batch_leg(ctx, count):
    """Workload 4: `count` independent systems (n ~ U{6..9}, m = n+1 dense,
    F_65521): one f4_groebner_batch call vs the same systems one by one."""
    import torch
    import synth
    systems = [(p, n, polys) for n, p, polys in synth.batch_systems(count)]
    prep = ctx.prepare_batch(systems)
    ctx.groebner_batch_prepared(prep)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.groebner_batch_prepared(prep)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    preps = [ctx.prepare(p, n, polys) for p, n, polys in systems]  # marshalled once, as for the batch
    t0 = time.perf_counter()
    for q in preps:
        ctx.groebner_prepared(q)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    nnz = sum(s["nnz"] for _, steps in res for s in steps)
    return {"workload": "%d dense systems, n ~ U{6..9}, m = n+1, F_65521 (seeds 4*2^32+j)" % count,
            "systems": count, "batched_s": tb, "plain_s": tp,
            "systems_per_s_batched": count / tb, "systems_per_s_plain": count / tp,
            "speedup": tp / tb, "nnz_total": nnz, "nnz_per_s_batched": nnz / tb}


def serve_leg(f4, ctx, seconds):
    """Workload 5: Poisson arrivals (500/s) of systems n ~ U{5..12}, p from
    {65521, 2^31-1}.  The continuous-batching server (admission by estimated
    device footprint) against a plain FIFO that runs f4_groebner per request,
    both on this GPU, on the same stream; latency = completion - arrival."""
    import synth
    stream = synth.serve_stream(rate=500.0, duration=seconds)
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
    return {"workload": "Poisson 500/s for %.1f s: %d requests, n ~ U{5..12}, p in {65521, 2^31-1}" %
                        (seconds, len(stream)),
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
    import synth
    import paper_2601_06765_amd.f4 as f4

    torch.cuda.init()
    n, p, polys = synth.config_system(2)
    # the headline: the timed runs without instrumentation
    tune = not args.no_autotune
    plain = f4.Context(0, dict_path=args.dict, autotune=tune)
    prep = plain.prepare(p, n, polys)  # host SoA arrays of the input, built once
    for _ in range(args.warmup):
        plain.groebner_prepared(prep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        basis, _ = plain.groebner_prepared(prep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    table = plain.tune_table()
    plain.close()
    assert basis == [[((0,) * n, 1)]], "unexpected basis"
    # the same runs again with HIP events around every stage and around each
    # launch of the two elimination kernels (stage times, roofline)
    ctx = f4.Context(0, timing=True, dict_path=args.dict, autotune=tune)
    ctx.load_tune_table(table)  # the headline runs' schedules
    prep = ctx.prepare(p, n, polys)
    for _ in range(args.warmup):
        ctx.groebner_prepared(prep)
    torch.cuda.synchronize()
    allsteps = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        basis, steps = ctx.groebner_prepared(prep)
        allsteps.append(steps)
    torch.cuda.synchronize()
    dt_instr = time.perf_counter() - t1

    nnz_run = sum(s["nnz"] for s in allsteps[0])
    rows_run = sum(s["r"] for s in allsteps[0])
    ms_run = dt * 1000.0 / args.steps
    value = nnz_run * args.steps / dt

    # per F4 step (averaged over runs): GPU stage times from HIP events
    per_step = []
    nsteps = len(allsteps[0])
    avg = lambda k, key: sum(run[k][key] for run in allsteps) / len(allsteps)
    for k in range(nsteps):
        s0 = allsteps[0][k]
        gpu_ms = avg(k, "t_dict_ms") + avg(k, "t_assemble_ms") + avg(k, "t_numeric_ms")
        c = s0["N"] - s0["npivot"]
        # algorithmic bytes of the step (unit: one nonzero of A): build writes
        # the CSR (8 B per nonzero, 16 per row, 8 per column), the elimination
        # reads it once and writes the trailing block and its echelon rows
        alg = (8 * s0["nnz"] + 16 * s0["r"] + 8 * s0["N"]) + (8 * s0["nnz"] + 4 * s0["r"]
                                                               + 4 * s0["lower"] * c + 4 * s0["rho"] * c)
        per_step.append({
            "deg": s0["deg"], "r": s0["r"], "N": s0["N"], "nnz": s0["nnz"], "npivot": s0["npivot"],
            "lower": s0["lower"], "rho": s0["rho"],
            "t_dict_ms": round(avg(k, "t_dict_ms"), 4),
            "t_assemble_ms": round(avg(k, "t_assemble_ms"), 4),
            "t_numeric_ms": round(avg(k, "t_numeric_ms"), 4),
            "t_trsm_ms": round(avg(k, "t_trsm_ms"), 4),
            "t_echelon_ms": round(avg(k, "t_echelon_ms"), 4),
            "wall_ms": round(avg(k, "t_step_ms"), 4),
            "t_pairs_host_ms": round(avg(k, "t_pairs_ms"), 4),
            "nnz_per_s_gpu": s0["nnz"] / (gpu_ms / 1000.0) if gpu_ms > 0 else None,
            "rows_per_s_gpu": s0["r"] / (gpu_ms / 1000.0) if gpu_ms > 0 else None,
            "hbm_frac_alg": alg / (gpu_ms / 1000.0) / (HBM_PEAK_GBS * 1e9) if gpu_ms > 0 else None,
        })

    out_roof = roofline_of(allsteps)
    out = {
        "metric": "Macaulay nnz/s built+reduced per F4 step; systems/sec batched vs plain",
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_run,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded dense random quadratics, splitmix64 seed 2)",
        "config": {"workload": "full F4, n=10, m=12 dense quadratics over F_65521, grevlex, normal strategy",
                   "n": n, "m": len(polys), "p": p, "f4_steps": nsteps, "nnz_per_run": nnz_run,
                   "rows_per_run": rows_run, "dict_path": args.dict or "auto"},
        "rows_per_s": rows_run * args.steps / dt,
        "ms_per_step_instrumented": dt_instr * 1000.0 / args.steps,
        "systems_per_s_plain": args.steps / dt,
        "per_f4_step": per_step,
        "roofline": out_roof,
        "autotune": {"on": tune, "table": table.splitlines()},
    }
    ctx.close()
    if args.sparse_repeats:
        out["sparse_step"] = sparse_step_leg(f4, args.sparse_repeats, tune)
    if args.spmm_shift_deg:
        out["spmm"] = spmm_leg(f4, args.spmm_shift_deg, 8, 20)
    if args.modloop_chains:
        out["modloop"] = modloop_leg(f4, args.modloop_chains, args.modloop_iters)
        # the kernels' own small-prime form (one-word Barrett) at the workload's prime
        e3 = [x for x in out["modloop"]["forms"] if x["form"] == "barrett32" and x["p"] == p]
        if e3:
            mp = e3[0]["updates_per_s"] / 1e12
            out_roof["measured_peak"] = {"value": round(mp, 3), "unit": "Tmodmul/s",
                                         "source": "modular inner-loop microbenchmark, one-word Barrett, p = %d" % p,
                                         "frac": round(out_roof["achieved"] / mp, 5)}
    if args.batch_systems:
        bctx = f4.Context(0, autotune=tune)
        out["batch"] = batch_leg(bctx, args.batch_systems)
        bctx.close()
        out["systems_per_s_batched"] = out["batch"]["systems_per_s_batched"]
    if args.serve_seconds > 0:
        sctx = f4.Context(0, autotune=tune)
        out["serve"] = serve_leg(f4, sctx, args.serve_seconds)
        sctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, p, polys, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
