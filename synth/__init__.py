"""Seeded synthetic polynomial systems shared by the oracle tests and the GPU path.

This module only draws random numbers and lays out terms; it performs none of
the method's arithmetic (no term order, no monomial products, no reduction).
A polynomial is returned as a list of ``(exps, coeff)`` pairs, ``exps`` a tuple
of n non-negative ints and ``coeff`` an int, in the generator's own draw order
(not in any term order).  Consumers sort and normalise terms themselves.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), one stream per seed.  Uniform
integers are drawn by rejection so that every value is equally likely.

Workloads follow the paper's third benchmark family, dense random quadratic
systems over F_p (benchmark protocol section, "Algebraic benchmark families").
"""

MASK64 = (1 << 64) - 1

# The eight largest primes below 2^31 (found by trial division; checked in tests).
CRT_PRIMES = (2147483647, 2147483629, 2147483587, 2147483579,
              2147483563, 2147483549, 2147483543, 2147483497)
P16 = 65521
P31 = 2147483647


class SplitMix64:
    """splitmix64: state += golden gamma, then a two-round xorshift-multiply mix."""

    def __init__(self, seed):
        self.state = seed & MASK64

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, k):
        """Uniform integer in [0, k) by rejection on the top multiple of k."""
        if k <= 0:
            raise ValueError("k must be positive")
        limit = ((1 << 64) // k) * k
        while True:
            u = self.next()
            if u < limit:
                return u % k

    def uniform01(self):
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def residues(p, count, seed):
    """``count`` uniform residues in [0, p): exactly the values that successive
    ``SplitMix64(seed).below(p)`` calls return, drawn in bulk with numpy (the
    i-th raw output is the mix of seed + i * gamma; outputs at or above the
    top multiple of p are skipped, as ``below`` skips them)."""
    import numpy as np
    if p <= 0:
        raise ValueError("p must be positive")
    limit = np.uint64(((1 << 64) // p) * p - 1)  # largest accepted raw value
    gamma = np.uint64(0x9E3779B97F4A7C15)
    parts, have, start = [], 0, 0
    while have < count:
        m = count - have + 16
        i = np.arange(start + 1, start + m + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + i * gamma
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        z = z[z <= limit] % np.uint64(p)
        parts.append(z[:count - have])
        have += len(parts[-1])
        start += m
    return np.concatenate(parts).astype(np.uint32) if parts else np.zeros(0, dtype=np.uint32)


def monomials_upto(n, d):
    """Every exponent vector of degree <= d in n variables, as rows of an int
    array (degree 0 first; inside a degree, the order of
    itertools.combinations_with_replacement over the variable indices)."""
    import itertools
    import numpy as np
    rows = []
    for k in range(d + 1):
        for c in itertools.combinations_with_replacement(range(n), k):
            e = [0] * n
            for i in c:
                e[i] += 1
            rows.append(e)
    return np.array(rows, dtype=np.int64).reshape(-1, n)


def quadratic_support(n):
    """All monomials of degree <= 2 in n variables, as exponent tuples.

    Generator order (a fixed convention of this module, used only to decide
    which coefficient is drawn when): degree 2 first, x_i*x_j for j = 1..n and
    i = 1..j; then x_1..x_n; then 1.
    """
    out = []
    for j in range(n):
        for i in range(j + 1):
            e = [0] * n
            e[i] += 1
            e[j] += 1
            out.append(tuple(e))
    for i in range(n):
        e = [0] * n
        e[i] = 1
        out.append(tuple(e))
    out.append(tuple([0] * n))
    return out


def dense_quadratics(n, m, seed, cmax):
    """m dense quadratics: every monomial of degree <= 2, coefficients U[1, cmax].

    Coefficients are drawn polynomial by polynomial, monomial by monomial in
    :func:`quadratic_support` order.
    """
    rng = SplitMix64(seed)
    sup = quadratic_support(n)
    return [[(e, 1 + rng.below(cmax)) for e in sup] for _ in range(m)]


def sparse_quadratics(n, m, seed, cmax, k):
    """m quadratics with k distinct monomials of degree <= 2 each.

    Per polynomial: a partial Fisher-Yates shuffle of :func:`quadratic_support`
    picks k monomials (k uniform index draws), then k coefficients U[1, cmax]
    are drawn in pick order.
    """
    rng = SplitMix64(seed)
    sup = quadratic_support(n)
    if k > len(sup):
        raise ValueError("k exceeds the number of monomials of degree <= 2")
    polys = []
    for _ in range(m):
        idx = list(range(len(sup)))
        for s in range(k):
            t = s + rng.below(len(sup) - s)
            idx[s], idx[t] = idx[t], idx[s]
        picks = idx[:k]
        polys.append([(sup[q], 1 + rng.below(cmax)) for q in picks])
    return polys


def reduce_coeffs(polys, p):
    """Read integer coefficients mod p (the CRT convention: one integer system, many primes)."""
    return [[(e, c % p) for (e, c) in f] for f in polys]


# ---------------------------------------------------------------------------
# The workloads: dense random quadratic systems and one sparse variant.
# ---------------------------------------------------------------------------

def system(name):
    """(n, p, polys) of a named single system: "dense_n6" (n=6, m=7, all 28
    monomials of degree <= 2, F_65521, seed 1), "dense_n10" (n=10, m=12,
    F_65521, seed 2), "sparse_n14" (n=14, m=15, 20 monomials each, F_(2^31-1),
    seed 3)."""
    if name == "dense_n6":
        return 6, P16, dense_quadratics(6, 7, 1, P16 - 1)
    if name == "dense_n10":
        return 10, P16, dense_quadratics(10, 12, 2, P16 - 1)
    if name == "sparse_n14":
        return 14, P31, sparse_quadratics(14, 15, 3, P31 - 1, 20)
    raise ValueError("single systems: dense_n6, dense_n10, sparse_n14")


def batch_systems(count=256):
    """The batch workload: `count` systems, n ~ U{6..9}, m = n+1 dense, F_65521.

    System j uses the stream seeded 4*2^32 + j: the first draw picks n, the
    following draws the coefficients.
    """
    out = []
    for j in range(count):
        rng_seed = (4 << 32) + j
        rng = SplitMix64(rng_seed)
        n = 6 + rng.below(4)
        sup = quadratic_support(n)
        polys = [[(e, 1 + rng.below(P16 - 1)) for e in sup] for _ in range(n + 1)]
        out.append((n, P16, polys))
    return out


def crt_system():
    """The CRT leg of the batch workload: one n=9, m=10 dense system (seed 4*2^32+256) with
    integer coefficients in [1, 65520]; read it mod each of CRT_PRIMES."""
    return 9, dense_quadratics(9, 10, (4 << 32) + 256, P16 - 1)


def serve_stream(rate=500.0, duration=60.0, limit=None):
    """The serving workload: Poisson arrivals (exponential gaps from seed 5*2^32 + 2^31).

    Request j: seed 5*2^32 + j; first draw n ~ U{5..12}, second draw
    p ~ U{65521, 2^31-1}, then dense coefficients U[1, p-1].
    Returns a list of (arrival_seconds, n, p, polys).
    """
    import math
    gaps = SplitMix64((5 << 32) + (1 << 31))
    t = 0.0
    out = []
    j = 0
    while True:
        t += -math.log(1.0 - gaps.uniform01()) / rate
        if t >= duration or (limit is not None and j >= limit):
            break
        rng = SplitMix64((5 << 32) + j)
        n = 5 + rng.below(8)
        p = (P16, P31)[rng.below(2)]
        sup = quadratic_support(n)
        polys = [[(e, 1 + rng.below(p - 1)) for e in sup] for _ in range(n + 1)]
        out.append((t, n, p, polys))
        j += 1
    return out


def random_system(n, m, p, seed, density=1.0, max_deg=2):
    """Small random system for tests: each monomial of degree <= max_deg kept
    with probability `density` (Bernoulli from the stream), coefficients U[1, p-1]."""
    rng = SplitMix64(seed)
    sup = []
    # all exponent tuples of degree <= max_deg, generated by a plain odometer
    e = [0] * n
    while True:
        if sum(e) <= max_deg:
            sup.append(tuple(e))
        i = 0
        while i < n:
            e[i] += 1
            if sum(e) <= max_deg:
                break
            e[i] = 0
            i += 1
        if i == n:
            break
    polys = []
    for _ in range(m):
        f = []
        for mono in sup:
            if density >= 1.0 or rng.uniform01() < density:
                f.append((mono, 1 + rng.below(p - 1)))
        polys.append(f)
    return polys


def planted_system(n, m, p, seed):
    """m dense quadratics vanishing at a planted point s in F_p^n.

    f_i = q_i - q_i(s) with q_i a dense random quadratic.  The constant term is
    set so that f_i(s) = 0 (evaluation by plain integer arithmetic).
    Returns (polys, s).
    """
    rng = SplitMix64(seed)
    s = [rng.below(p) for _ in range(n)]
    sup = quadratic_support(n)
    polys = []
    for _ in range(m):
        f = [(e, 1 + rng.below(p - 1)) for e in sup if sum(e) > 0]
        val = 0
        for e, c in f:
            v = c
            for i, a in enumerate(e):
                v = v * pow(s[i], a, p) % p
            val = (val + v) % p
        f.append((tuple([0] * n), (p - val) % p))
        polys.append(f)
    return polys, s


def signatures(leads, m_index, seed, max_deg=2):
    """Synthetic signatures for a basis whose elements have the exponent
    vectors ``leads`` (one per element, e.g. its leading exponents): the
    first ``m_index`` elements get index k and the exponent vector 0 (input
    polynomials); every later element a uniform index below ``m_index`` and an
    exponent vector obtained from its lead by removing uniformly chosen unit
    exponents until at most ``max_deg`` remain (a divisor of the lead).
    Returns (index list, exponent-vector list)."""
    rng = SplitMix64((9 << 32) + seed)
    idx, mon = [], []
    for k, e in enumerate(leads):
        n = len(e)
        if k < m_index:
            idx.append(k)
            mon.append((0,) * n)
            continue
        idx.append(rng.below(m_index))
        v = list(e)
        while sum(v) > max_deg:
            nz = [q for q in range(n) if v[q]]
            v[nz[rng.below(len(nz))]] -= 1
        mon.append(tuple(v))
    return idx, mon
