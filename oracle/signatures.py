"""O7: signature admissibility as a bulk row filter, and symbolic
preprocessing relative to the admissible reducers (test infrastructure only,
like the rest of this package).

The paper states what the signature regime must guarantee and how a GPU
should run it, but leaves the signature order and the rewrite rule to the
chosen framework (section "Signature regime: correctness under admissibility
predicates", Theorem "Signature-sound compilation"; section "Discussion:
Integrating Signatures, Admissibility, and GPU Scheduling").  The readings
taken here:

* Signatures.  Basis element k carries a signature s_k e_{i_k} (a monomial
  s_k and an index i_k, given as input).  The shifted reducer t * g_k has the
  signature (t s_k) e_{i_k}.  Order: position over term (index first, then
  grevlex on the monomial).
* Syzygy criterion (F5).  For each index i a list of monomials u with u e_i
  the signature of a known syzygy (for instance LM(f_j) for j < i, the
  principal syzygies f_j e_i - f_i e_j).  A row whose signature u e_i has
  some listed monomial dividing u is rejected: its signature is that of a
  multiple of a syzygy.
* Rewrite criterion.  A row t * g_k is rejected when a newer basis element
  k' > k with the same index has s_{k'} dividing t s_k: the newest element
  whose signature divides a signature is the one allowed to produce it.
* The syzygy test is applied first; the flag records the first failing test
  (0 admissible, 1 syzygy, 2 rewritten).
* Bulk filtering: the flags of all rows, the admissible rows compacted in
  input order, and a schedule of them bucketed by (row degree, length of
  g_k, signature index), stable within a bucket.
* Signature-aware closure: the dictionary closure of symbolic preprocessing
  is run over the admissible reducers only (the fixed point "propose rows,
  filter, close, recheck"): the initial rows are filtered, and a monomial m
  of the dictionary gets as reducer the active element g of largest index
  with LM(g) | m whose row (m / LM(g), g) is admissible; m gets no row when
  no such g exists.  With every row admissible this is the ordinary closure
  (the reducer rule of the F4 step).

Monomials are exponent tuples; a polynomial is a list of (exponent tuple,
coefficient).  Everything here is plain Python sets, loops and sorts.
"""

from .buchberger import divides, grevlex_key

ADM_OK, ADM_SYZYGY, ADM_REWRITTEN = 0, 1, 2


def mono_mul(a, b):
    return tuple(x + y for x, y in zip(a, b))


def mono_div(a, b):
    """a / b for b | a."""
    return tuple(x - y for x, y in zip(a, b))


def lead(f):
    return max((e for e, _ in f), key=grevlex_key)


def signature(t, k, sig_index, sig_mon):
    """Signature of the row t * g_k as (index, monomial)."""
    return sig_index[k], mono_mul(t, sig_mon[k])


def pot_key(sig):
    """Position-over-term order key of a signature (index, monomial)."""
    return sig[0], grevlex_key(sig[1])


def admissible(t, k, sig_index, sig_mon, syz):
    """Flag of the row t * g_k: ADM_OK, ADM_SYZYGY or ADM_REWRITTEN."""
    i, u = signature(t, k, sig_index, sig_mon)
    for m in syz[i]:
        if divides(m, u):
            return ADM_SYZYGY
    for k2 in range(k + 1, len(sig_index)):
        if sig_index[k2] == i and divides(sig_mon[k2], u):
            return ADM_REWRITTEN
    return ADM_OK


def filter_rows(rows, G, sig_index, sig_mon, syz):
    """Flags of the rows (t, k), the admissible rows in input order, and the
    schedule: positions in that list sorted by (degree of t * LM(g_k),
    length of g_k, signature index), stable."""
    flags = [admissible(t, k, sig_index, sig_mon, syz) for t, k in rows]
    kept = [rows[q] for q in range(len(rows)) if flags[q] == ADM_OK]

    def key(x):
        t, k = kept[x]
        return sum(mono_mul(t, lead(G[k]))), len(G[k]), sig_index[k]

    order = sorted(range(len(kept)), key=key)  # Python's sort is stable
    return flags, kept, order


def fbsp(G, active, rows, sig=None):
    """Symbolic preprocessing of the explicit rows (t, k) with the dictionary
    closure; sig = (sig_index, sig_mon, syz) restricts both the rows and the
    reducers to admissible ones.  Returns the matrix in the library's
    conventions: dictionary T in descending grevlex, rows ordered by leading
    monomial descending then basis index, column indices ascending per row."""
    lms = [lead(g) for g in G]
    ok = (lambda t, k: True) if sig is None else (lambda t, k: admissible(t, k, *sig) == ADM_OK)
    R = set()
    for t, k in rows:
        if ok(tuple(t), k):
            R.add((tuple(t), k))
    present, done = set(), set()
    for t, k in R:
        done.add(mono_mul(t, lms[k]))
        for e, _ in G[k]:
            present.add(mono_mul(t, e))
    while True:
        frontier = present - done
        if not frontier:
            break
        for m in frontier:
            done.add(m)
            for g in range(len(G) - 1, -1, -1):
                if not active[g] or not divides(lms[g], m):
                    continue
                t = mono_div(m, lms[g])
                if ok(t, g):
                    R.add((t, g))
                    for e, _ in G[g]:
                        present.add(mono_mul(t, e))
                    break
    T = sorted(present, key=grevlex_key, reverse=True)
    col = {m: c for c, m in enumerate(T)}
    order = sorted(R, key=lambda r: (col[mono_mul(r[0], lms[r[1]])], r[1]))
    row_ptr, col_ind, val = [0], [], []
    for t, k in order:
        ent = sorted((col[mono_mul(t, e)], c) for e, c in G[k])
        col_ind += [c for c, _ in ent]
        val += [v for _, v in ent]
        row_ptr.append(len(col_ind))
    return {"T": T, "rows_t": [t for t, _ in order], "rows_k": [k for _, k in order],
            "row_ptr": row_ptr, "col_ind": col_ind, "val": val}
