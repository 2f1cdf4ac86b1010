"""Oracle O2: Buchberger's algorithm in pure Python (test infrastructure only).

A polynomial is a dict {exponent tuple: coefficient in [1, p)}.  Every
S-polynomial (Definition "S-polynomial") of every pair is reduced by
multivariate division; nonzero remainders join the basis until all pairs
reduce to zero (Buchberger's criterion, stated right after that definition).
No pair criteria are used.  The result is then made minimal, inter-reduced,
monic and sorted, i.e. the unique reduced Groebner basis.  Meant for tiny
systems only (a handful of variables and polynomials).

The term order is grevlex with x_1 > ... > x_n, written here through a sort
key: total degree first, then the reversed exponent vector compared with the
opposite sign.  This is a different formulation from the one in the C++
oracle, so the two check each other.
"""


def grevlex_key(e):
    """Sort key: larger key = larger monomial under grevlex (x_1 > ... > x_n)."""
    return (sum(e), tuple(-a for a in reversed(e)))


def lead(f):
    return max(f, key=grevlex_key)


def clean(f, p):
    return {e: c % p for e, c in f.items() if c % p}


def from_terms(terms, p):
    f = {}
    for e, c in terms:
        f[tuple(e)] = (f.get(tuple(e), 0) + c) % p
    return clean(f, p)


def divides(a, b):
    return all(x <= y for x, y in zip(a, b))


def monomial_quotient(b, a):
    return tuple(y - x for x, y in zip(a, b))


def add_scaled(f, g, c, shift, p):
    """f + c * x^shift * g."""
    out = dict(f)
    for e, v in g.items():
        m = tuple(x + y for x, y in zip(e, shift))
        out[m] = (out.get(m, 0) + c * v) % p
        if out[m] == 0:
            del out[m]
    return out


def normal_form(f, G, p):
    """Remainder of f on division by the list G (all nonzero)."""
    f = dict(f)
    rem = {}
    while f:
        m = lead(f)
        c = f[m]
        for g in G:
            lg = lead(g)
            if divides(lg, m):
                inv = pow(g[lg], p - 2, p)
                f = add_scaled(f, g, (-c * inv) % p, monomial_quotient(m, lg), p)
                break
        else:
            rem[m] = c
            del f[m]
    return rem


def spoly(f, g, p):
    lf, lg = lead(f), lead(g)
    L = tuple(max(x, y) for x, y in zip(lf, lg))
    a = add_scaled({}, f, pow(f[lf], p - 2, p), monomial_quotient(L, lf), p)
    return add_scaled(a, g, (-pow(g[lg], p - 2, p)) % p, monomial_quotient(L, lg), p)


def monic(f, p):
    inv = pow(f[lead(f)], p - 2, p)
    return {e: c * inv % p for e, c in f.items()}


def reduced_basis(G, p):
    """Minimal, inter-reduced, monic basis sorted by leading monomial (largest first)."""
    G = [monic(g, p) for g in G if g]
    minimal = []
    for i, g in enumerate(G):
        lg = lead(g)
        dominated = False
        for j, h in enumerate(G):
            if j == i:
                continue
            lh = lead(h)
            if divides(lh, lg) and (lh != lg or j < i):
                dominated = True
                break
        if not dominated:
            minimal.append(g)
    out = []
    for i, g in enumerate(minimal):
        others = [h for j, h in enumerate(minimal) if j != i]
        lg = lead(g)
        tail = {e: c for e, c in g.items() if e != lg}
        r = normal_form(tail, others, p)
        r[lg] = 1
        out.append(r)
    out.sort(key=lambda f: grevlex_key(lead(f)), reverse=True)
    return out


def groebner(n, p, polys):
    """Reduced Groebner basis of the ideal spanned by `polys` (lists of (exps, coeff))."""
    G = [from_terms(f, p) for f in polys]
    G = [g for g in G if g]
    pairs = [(i, j) for j in range(len(G)) for i in range(j)]
    while pairs:
        i, j = pairs.pop()
        r = normal_form(spoly(G[i], G[j], p), G, p)
        if r:
            G.append(r)
            k = len(G) - 1
            pairs.extend((a, k) for a in range(k))
    return reduced_basis(G, p)


def as_sorted_terms(f):
    """Polynomial as a list of (exps, coeff), largest monomial first."""
    return [(e, f[e]) for e in sorted(f, key=grevlex_key, reverse=True)]
