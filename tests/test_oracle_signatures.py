"""Pins of O7 (oracle/signatures.py): the signature filter and the closure
over admissible reducers, checked against facts that do not come from O7's
own code paths:

* a hand-worked example (tests/golden/signature_filter_n2.txt);
* every row rejected by the syzygy test with principal syzygy lists carries
  the signature of an explicit syzygy: the module element
  (u / LM(f_j)) (f_j e_i - f_i e_j) is built, its image under
  e_l -> f_l is zero (polynomial arithmetic), and its position-over-term
  leading term is the row's signature; admissible rows have no such j;
* with no constraint the closure is O1's symbolic preprocessing: the whole
  matrix of every recorded step equals O1's (a different implementation);
* Theorem "Signature-sound compilation" and the closure's fixed point, by
  brute force: every row of the result is admissible, every dictionary
  monomial without a row has no admissible reducer, each reducer is the
  admissible one of largest index, and the dictionary is exactly the union
  of the row supports;
* the schedule is a stable sort of the kept rows by its bucket key.
"""

import os
import random

import pytest

import oracle
import synth
from oracle import buchberger as bb
from oracle import signatures as o7

HERE = os.path.dirname(os.path.abspath(__file__))


def load_golden():
    basis, sidx, smon, syz, rows, flags, order = [], [], [], {}, [], [], None
    for line in open(os.path.join(HERE, "golden", "signature_filter_n2.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tag, rest = line.split(None, 1)
        if tag == "basis":
            parts = [p.split() for p in rest.split(";")]
            v = [int(x) for x in parts[0]][1:]
            basis.append([((v[q], v[q + 1]), v[q + 2]) for q in range(0, len(v), 3)])
            sidx.append(int(parts[1][0]))
            smon.append(tuple(int(x) for x in parts[2]))
        elif tag == "syz":
            v = [int(x) for x in rest.split()]
            syz.setdefault(v[0], []).append((v[1], v[2]))
        elif tag == "row":
            v = [int(x) for x in rest.split()]
            rows.append(((v[0], v[1]), v[2]))
            flags.append(v[3])
        elif tag == "order":
            order = [int(x) for x in rest.split()]
    syz_list = [syz.get(i, []) for i in range(max(sidx) + 1)]
    return basis, sidx, smon, syz_list, rows, flags, order


def test_golden_hand_example():
    G, sidx, smon, syz, rows, want_flags, want_order = load_golden()
    flags, kept, order = o7.filter_rows(rows, G, sidx, smon, syz)
    assert flags == want_flags
    assert kept == [rows[q] for q in range(len(rows)) if want_flags[q] == 0]
    assert order == want_order


def poly_mul_mono(f, t, c, p):
    return {o7.mono_mul(e, t): v * c % p for e, v in f.items()}


def poly_add(a, b, p):
    out = dict(a)
    for e, v in b.items():
        out[e] = (out.get(e, 0) + v) % p
        if out[e] == 0:
            del out[e]
    return out


def as_dict(f):
    return {tuple(e): c for e, c in f}


@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2), (5, 3)])
def test_syzygy_rejections_are_principal_syzygies(n, seed):
    p = 65521
    F = synth.random_system(n, n, p, seed, density=0.6, max_deg=2)
    F = [sorted(f, key=lambda t: bb.grevlex_key(t[0]), reverse=True) for f in F]
    m = len(F)
    lms = [o7.lead(f) for f in F]
    sidx = list(range(m))
    smon = [(0,) * n] * m
    syz = [[lms[j] for j in range(i)] for i in range(m)]
    shifts = synth.monomials_upto(n, 2)
    rows = [(tuple(t), k) for k in range(m) for t in shifts]
    flags, kept, _ = o7.filter_rows(rows, F, sidx, smon, syz)
    nsyz = 0
    for (t, i), fl in zip(rows, flags):
        js = [j for j in range(i) if bb.divides(lms[j], t)]
        if fl != o7.ADM_SYZYGY:
            assert not js
            continue
        nsyz += 1
        assert js
        j = js[0]
        u = o7.mono_div(t, lms[j])
        # sigma = u (f_j e_i - f_i e_j): component i is u f_j, component j is -u f_i
        comp = {i: poly_mul_mono(as_dict(F[j]), u, 1, p), j: poly_mul_mono(as_dict(F[i]), u, p - 1, p)}
        image = {}
        for l, c in comp.items():
            for e, v in c.items():
                image = poly_add(image, poly_mul_mono(as_dict(F[l]), e, v, p), p)
        assert image == {}
        # leading module term under position over term: the largest index,
        # then the largest monomial of that component
        top = max(comp)
        assert top == i and max(comp[top], key=bb.grevlex_key) == tuple(t)
    assert nsyz > 0


def step_records(cfg):
    n, p, polys = synth.system(cfg)
    run = oracle.OracleRun(n, p, polys, record=-2)
    return n, [run.step_record(k) for k in range(len(run.steps()))]


def halves(rec, n):
    lms = [o7.lead(g) for g in rec["G"]]
    rows = []
    for i, j in rec["sel"]:
        L = tuple(max(a, b) for a, b in zip(lms[i], lms[j]))
        rows.append((o7.mono_div(L, lms[i]), i))
        rows.append((o7.mono_div(L, lms[j]), j))
    return rows


@pytest.mark.parametrize("cfg", ["dense_n6", "dense_n10"])
def test_unconstrained_closure_is_o1(cfg):
    n, recs = step_records(cfg)
    for rec in recs:
        G = [list(g) for g in rec["G"]]
        got = o7.fbsp(G, rec["active"], halves(rec, n))
        assert got["T"] == rec["T"]
        assert got["rows_t"] == rec["rows_t"] and list(got["rows_k"]) == list(rec["rows_k"])
        assert list(got["row_ptr"]) == list(rec["row_ptr"])
        assert list(got["col_ind"]) == list(rec["col_ind"]) and list(got["val"]) == list(rec["val"])
        # all-admissible signatures (distinct indices, no syzygies): the same matrix
        m = len(G)
        sig = (list(range(m)), [(0,) * n] * m, [[] for _ in range(m)])
        assert o7.fbsp(G, rec["active"], halves(rec, n), sig) == got


def synthetic_signatures(G, n, m_index, seed):
    """Signature index and monomial per element (input-like elements first)."""
    return synth.signatures([o7.lead(g) for g in G], m_index, seed)


@pytest.mark.parametrize("cfg,m_index,seed", [("dense_n6", 7, 5), ("dense_n6", 3, 6)])
def test_signature_aware_closure_fixed_point(cfg, m_index, seed):
    n, recs = step_records(cfg)
    tested = 0
    for rec in recs:
        G = [list(g) for g in rec["G"]]
        lms = [o7.lead(g) for g in G]
        sidx, smon = synthetic_signatures(G, n, min(m_index, len(G)), seed)
        syz = [[lms[j] for j in range(i)] for i in range(max(sidx) + 1)]
        sig = (sidx, smon, syz)
        init = halves(rec, n)
        got = o7.fbsp(G, rec["active"], init, sig)
        rows = list(zip(got["rows_t"], got["rows_k"]))
        # soundness: every row is admissible (brute force over the definition)
        for t, k in rows:
            u = o7.mono_mul(t, smon[k])
            i = sidx[k]
            assert not any(bb.divides(mm, u) for mm in syz[i])
            assert not any(sidx[k2] == i and bb.divides(smon[k2], u) for k2 in range(k + 1, len(G)))
        T = got["T"]
        support = set()
        for t, k in rows:
            support |= {o7.mono_mul(t, e) for e, _ in G[k]}
        assert set(T) == support and len(T) == len(support)
        leads = {}
        for t, k in rows:
            leads.setdefault(o7.mono_mul(t, lms[k]), set()).add(k)
        assert len(set(rows)) == len(rows)
        admissible_init = {(tuple(t), k) for t, k in init
                           if o7.admissible(tuple(t), k, sidx, smon, syz) == o7.ADM_OK}
        for mono in T:
            cands = [g for g in range(len(G) - 1, -1, -1)
                     if rec["active"][g] and bb.divides(lms[g], mono)
                     and o7.admissible(o7.mono_div(mono, lms[g]), g, sidx, smon, syz) == o7.ADM_OK]
            init_here = {k for t, k in admissible_init if o7.mono_mul(t, lms[k]) == mono}
            # a monomial led by admissible initial rows keeps exactly those;
            # any other gets the admissible reducer of largest index, or none
            if init_here:
                assert leads[mono] == init_here
            elif cands:
                assert leads.get(mono) == {cands[0]}
            else:
                assert mono not in leads
        tested += 1
    assert tested > 0


def test_schedule_is_stable_bucket_sort():
    rng = random.Random(9)
    n, recs = step_records("dense_n6")
    rec = recs[-1]
    G = [list(g) for g in rec["G"]]
    sidx, smon = synthetic_signatures(G, n, 4, 10)
    lms = [o7.lead(g) for g in G]
    syz = [[lms[j] for j in range(i)] for i in range(4)]
    rows = [(o7.mono_div(tuple(t), (0,) * n), rng.randrange(len(G))) for t in synth.monomials_upto(n, 2)]
    flags, kept, order = o7.filter_rows(rows, G, sidx, smon, syz)
    assert sorted(order) == list(range(len(kept)))
    keys = [(sum(o7.mono_mul(kept[x][0], lms[kept[x][1]])), len(G[kept[x][1]]), sidx[kept[x][1]], x)
            for x in order]
    assert keys == sorted(keys)
