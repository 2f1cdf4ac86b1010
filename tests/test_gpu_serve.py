"""Serving (continuous batching): requests admitted between engine steps
share the batched launches; each result equals the system's result alone and
the oracle's, exactly."""

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


def test_server_mix_invariance_and_admission(f4):
    ctx = f4.Context(0)
    try:
        stream = synth.serve_stream(duration=0.04)  # ~20 requests, n in 5..12, mixed primes
        reqs = [(p, n, polys) for _, n, p, polys in stream if n <= 8]
        polys, _ = synth.planted_system(5, 6, 65521, 41)
        reqs.insert(3, (65521, 5, polys))
        reqs.insert(5, (2147483647, 4, synth.random_system(4, 4, 2147483647, 42)))
        assert len(reqs) >= 6
        fp = max(f4.server_footprint(n, len(pl)) for p, n, pl in reqs)
        srv = f4.Server(ctx, hbm_budget=3 * fp, max_slots=3)
        say("serve", len(reqs), "requests, 3 slots")
        pending = list(range(len(reqs)))
        tickets, results, busy = {}, {}, 0
        steps = 0
        while len(results) < len(reqs):
            while pending:
                t = srv.submit(*reqs[pending[0]])
                if t is None:
                    busy += 1
                    break
                tickets[t] = pending.pop(0)
            srv.step()
            steps += 1
            for t in list(tickets):
                r = srv.poll(t)
                if r is not None:
                    results[tickets.pop(t)] = r
            assert steps < 10000
        assert busy > 0  # admission control engaged
        for i, (p, n, polys) in enumerate(reqs):
            say("alone", i, n, p)
            B, st = results[i]
            B1, st1 = ctx.groebner(p, n, polys)
            assert canon(B) == canon(B1)
            assert [(s["deg"], s["r"], s["N"], s["nnz"], s["rank"]) for s in st] == \
                   [(s["deg"], s["r"], s["N"], s["nnz"], s["rank"]) for s in st1]
            assert canon(B) == canon(oracle.OracleRun(n, p, polys).basis())
        srv.close()
    finally:
        ctx.close()


def test_server_busy_and_unknown_ticket(f4):
    ctx = f4.Context(0)
    try:
        n, p, polys = synth.system("dense_n6")
        srv = f4.Server(ctx, hbm_budget=f4.server_footprint(n, len(polys)), max_slots=8)
        t = srv.submit(p, n, polys)
        assert t is not None
        assert srv.submit(p, n, polys) is None  # over the footprint budget
        with pytest.raises(f4.F4Error) as ei:
            srv.poll(t + 100)
        assert ei.value.code == f4.F4_E_STATE
        while srv.poll(t) is None:
            srv.step()
        assert srv.load() == (0, 0, 0)
        srv.close()
    finally:
        ctx.close()


def test_server_mix_with_large_requests(f4):
    """Requests of the serving workload with n = 9..12 under both primes (the
    ones that dominate its GPU time), served four at a time next to small
    ones: each result equals the system's run alone; the n = 9 requests of
    both primes and an n = 10 request also equal the oracle's basis."""
    ctx = f4.Context(0)
    try:
        stream = synth.serve_stream(duration=0.2)
        picked, seen = [], {}
        for j, (_, n, p, polys) in enumerate(stream):
            key = (n, p)
            if n >= 9 and seen.get(key, 0) < 1:
                seen[key] = 1
                picked.append((j, p, n, polys))
            elif n <= 6 and seen.get(key, 0) < 2:
                seen[key] = seen.get(key, 0) + 1
                picked.append((j, p, n, polys))
        assert {(n, p) for _, p, n, _ in picked if n >= 9} == {(n, p) for n in (9, 10, 11, 12)
                                                                  for p in (synth.P16, synth.P31)}
        srv = f4.Server(ctx, hbm_budget=64 << 30, max_slots=4)
        say("serve", len(picked), "requests (n = 5..12, both primes), 4 slots")
        pending = list(range(len(picked)))
        tickets, results, steps = {}, {}, 0
        while len(results) < len(picked):
            while pending:
                _, p, n, polys = picked[pending[0]]
                t = srv.submit(p, n, polys)
                if t is None:
                    break
                tickets[t] = pending.pop(0)
            srv.step()
            steps += 1
            for t in list(tickets):
                r = srv.poll(t)
                if r is not None:
                    results[tickets.pop(t)] = r
            assert steps < 100000
        srv.close()
        for i, (j, p, n, polys) in enumerate(picked):
            say("alone request", j, "n=%d p=%d" % (n, p))
            B, st = results[i]
            B1, st1 = ctx.groebner(p, n, polys)
            assert canon(B) == canon(B1)
            assert [(s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"]) for s in st] == \
                   [(s["deg"], s["r"], s["N"], s["nnz"], s["npivot"], s["rank"]) for s in st1]
        for i, (j, p, n, polys) in enumerate(picked):
            if n == 9 or (n == 10 and p == synth.P16):
                say("oracle request", j, "n=%d p=%d" % (n, p))
                assert canon(results[i][0]) == canon(oracle.OracleRun(n, p, polys).basis())
    finally:
        ctx.close()
