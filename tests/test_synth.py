"""The seeded input generator: published PRNG vectors, prime list, workload shapes."""

import synth


def test_splitmix64_reference_vectors():
    # Reference outputs of splitmix64 (Steele-Lea-Flood; Vigna's public C code)
    r = synth.SplitMix64(0)
    assert [r.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    r = synth.SplitMix64(1234567)
    assert [r.next() for _ in range(3)] == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def _is_prime(q):
    if q < 2:
        return False
    d = 2
    while d * d <= q:
        if q % d == 0:
            return False
        d += 1
    return True


def test_crt_primes_are_the_eight_largest_below_2_31():
    ps = []
    q = (1 << 31) - 1
    while len(ps) < 8:
        if _is_prime(q):
            ps.append(q)
        q -= 1
    assert tuple(ps) == synth.CRT_PRIMES
    assert _is_prime(synth.P16) and _is_prime(synth.P31)


def test_below_is_uniform_and_in_range():
    r = synth.SplitMix64(99)
    k = 7
    counts = [0] * k
    for _ in range(70000):
        v = r.below(k)
        assert 0 <= v < k
        counts[v] += 1
    chi2 = sum((c - 10000) ** 2 / 10000 for c in counts)
    assert chi2 < 30  # 6 degrees of freedom; 30 is far in the tail


def test_workload_shapes():
    n, p, polys = synth.system("dense_n6")
    assert (n, p, len(polys)) == (6, 65521, 7)
    assert all(len(f) == 28 for f in polys)
    assert all(1 <= c <= 65520 for f in polys for _, c in f)
    n, p, polys = synth.system("dense_n10")
    assert (n, p, len(polys)) == (10, 65521, 12) and all(len(f) == 66 for f in polys)
    n, p, polys = synth.system("sparse_n14")
    assert (n, p, len(polys)) == (14, 2147483647, 15)
    for f in polys:
        mons = [e for e, _ in f]
        assert len(mons) == 20 and len(set(mons)) == 20
        assert all(sum(e) <= 2 for e in mons)
        assert all(1 <= c <= p - 1 for _, c in f)
    # determinism
    assert synth.system("dense_n10") == synth.system("dense_n10")


def test_batch_and_stream_shapes():
    sys_ = synth.batch_systems(16)
    for n, p, polys in sys_:
        assert 6 <= n <= 9 and p == 65521 and len(polys) == n + 1
        assert all(len(f) == (n + 1) * (n + 2) // 2 for f in polys)
    n, polys = synth.crt_system()
    assert n == 9 and len(polys) == 10
    st = synth.serve_stream(duration=0.2)
    assert len(st) > 20  # ~100 expected at 500/s
    last = 0.0
    for t, n, p, polys in st:
        assert t > last and 5 <= n <= 12 and p in (65521, 2147483647)
        last = t


def test_planted_point_is_a_root():
    p = 31
    polys, s = synth.planted_system(4, 5, p, 7)
    for f in polys:
        v = 0
        for e, c in f:
            t = c
            for i, a in enumerate(e):
                t = t * pow(s[i], a, p) % p
            v = (v + t) % p
        assert v == 0


def test_bulk_residues_equal_the_sequential_stream():
    for p, seed in [(3, 0), (65521, 12345), (synth.P31, 2**64 - 1), (2**31 + 11, 7)]:
        got = synth.residues(p, 2000, seed)
        g = synth.SplitMix64(seed)
        assert [int(v) for v in got] == [g.below(p) for _ in range(2000)]
    assert len(synth.residues(65521, 0, 1)) == 0
