"""Pins for the walk function (Sec. 2, Sec. 3): coset invariance of the hash, the
planted-claw identity, representation independence, decoding, the
distinguished-point rate and the trail merge property."""

import math

import numpy as np
import pytest

import seeded_inputs
from oracle import bfs, walk, zmat


def target(n, k, seed):
    tw = seeded_inputs.target_words(n, k, seed)
    return tw, zmat.target_from_words(n, tw.paulis, tw.clifford)


def test_phi_is_a_ring_homomorphism():
    # phi(sqrt2)^2 = 2 and phi(sqrt2) phi(1/sqrt2) = 1 in Z/p
    assert (walk.RHO * walk.RHO) % walk.P61 == 2
    assert (walk.RHO * walk.RHO_INV) % walk.P61 == 1
    # multiplicativity on Z[sqrt2]: (a + b s)(c + d s) = (ac + 2bd) + (ad + bc) s
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, b, c, d = (int(v) for v in rng.integers(-1000, 1000, 4))
        lhs = walk.phi(a, b, 0) * walk.phi(c, d, 0) % walk.P61
        assert lhs == walk.phi(a * c + 2 * b * d, a * d + b * c, 0)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_hash_independent_of_representation(n):
    _, u = target(n, 5, 11)
    keys = walk.make_keys(n, 5, 1, 77)
    assert walk.matrix_hash(u, keys) == walk.matrix_hash(u.raise_to(u.e + 3), keys)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_hash_invariant_under_left_cliffords(n):
    _, u = target(n, 6, 4)
    keys = walk.make_keys(n, 6, 0, 5)
    h0 = walk.matrix_hash(u, keys)
    for s in range(3):
        d = zmat.clifford_from_word(n, seeded_inputs.random_clifford_word(n, 200 + s))
        assert walk.matrix_hash(d @ u, keys) == h0
    # a rotation on the left leaves the coset and changes the hash
    assert walk.matrix_hash(zmat.rot_hat(3, n) @ u, keys) != h0


def test_hash_invariant_under_row_permutation_and_signs():
    n = 2
    _, u = target(n, 4, 8)
    keys = walk.make_keys(n, 4, 0, 1)
    rng = np.random.default_rng(3)
    perm = rng.permutation(16)
    sign = rng.choice([-1, 1], 16)
    m = zmat.ZMat(u.A[perm] * sign[:, None], u.B[perm] * sign[:, None], u.e)
    assert walk.matrix_hash(m, keys) == walk.matrix_hash(u, keys)
    # swapping two entries inside one row is not a coset move
    a = u.A.copy()
    b = u.B.copy()
    a[5, [3, 7]] = a[5, [7, 3]]
    b[5, [3, 7]] = b[5, [7, 3]]
    assert walk.matrix_hash(zmat.ZMat(a, b, u.e), keys) != walk.matrix_hash(u, keys)


@pytest.mark.parametrize("n,k,seed", [(1, 3, 1), (1, 4, 2), (2, 2, 3), (2, 3, 4), (2, 4, 5), (2, 5, 6),
                                      (2, 6, 7), (3, 3, 8), (3, 5, 9), (3, 6, 10)])
def test_planted_claw_identity(n, k, seed):
    tw, u = target(n, k, seed)
    xv, xw, c = walk.planted_points(n, k, tw.paulis)
    spec = walk.make_spec(u, n, k, c, 1234, delta=4)
    fv, hv = walk.f_with_hash(spec, walk.pack(xv, 0))
    fw, hw = walk.f_with_hash(spec, walk.pack(xw, 1))
    assert hv == hw and fv == fw
    # and the two half-matrices are in one left-Clifford coset
    V = walk.half_matrix(spec, xv, 0)
    W = walk.half_matrix(spec, xw, 1)
    assert (W @ V.T()).is_signed_perm()


def test_planted_claw_identity_n4():
    n, k = 4, 7
    tw, u = target(n, k, 1)
    xv, xw, c = walk.planted_points(n, k, tw.paulis)
    spec = walk.make_spec(u, n, k, c, 3000, delta=12)
    assert walk.f_with_hash(spec, walk.pack(xv, 0)) == walk.f_with_hash(spec, walk.pack(xw, 1))


def test_planted_claw_breaks_with_wrong_chunk():
    n, k = 2, 5
    tw, u = target(n, k, 6)
    xv, xw, c = walk.planted_points(n, k, tw.paulis)
    wrong = c % 15 + 1
    spec = walk.make_spec(u, n, k, wrong, 1234, delta=4)
    _, hv = walk.f_with_hash(spec, walk.pack(xv, 0))
    _, hw = walk.f_with_hash(spec, walk.pack(xw, 1))
    assert hv != hw


@pytest.mark.parametrize("n,h", [(1, 4), (2, 3), (3, 2), (4, 3)])
def test_decode_is_bijection(n, h):
    xi = 4 ** n - 1
    rng = np.random.default_rng(n)
    for x in [0, xi ** h - 1] + [int(v) for v in rng.integers(0, xi ** h, 50)]:
        ps = walk.decode(x, n, h)
        assert all(1 <= p <= xi for p in ps)
        assert walk.encode(ps, n) == x


def test_nh_element_closed_forms():
    """The element map is NH on two 32-bit words: ((lo + a) mod 2^32) ((hi + b) mod 2^32)."""
    two32 = 1 << 32
    assert walk.nh_element(0, 0) == 0
    assert walk.nh_element((5 << 32) | 7, 0) == 35
    # key words wrap modulo 2^32 before the product
    assert walk.nh_element((5 << 32) | 7, (3 << 32) | (two32 - 1)) == 6 * 8
    assert walk.nh_element((two32 - 2) << 32, 1 << 32) == 0
    # largest product: both words two32 - 1, still below 2^64
    assert walk.nh_element((two32 - 1) | ((two32 - 2) << 32), 1 << 32) == (two32 - 1) ** 2
    # the order of the rows does not matter: the hash is a sum of element maps
    salt = 0x0123456789ABCDEF
    vals = [3, 1 << 40, (1 << 60) - 5, 77]
    assert sum(walk.nh_element(v, salt) for v in vals) == sum(walk.nh_element(v, salt) for v in reversed(vals))


def test_distinct_cosets_have_distinct_hashes_n2():
    # every coset of T-count <= 3 at n = 2 (brute force) gets its own 64-bit hash
    counts, seen, levels = bfs.cosets_by_tcount(2, 3)
    keys = walk.make_keys(2, 6, 0, 99)
    hashes = {walk.matrix_hash(m, keys) for lvl in levels for m in lvl}
    assert len(hashes) == sum(counts)


def test_distinguished_rate_binomial():
    n, k = 3, 6
    _, u = target(n, k, 2)
    for delta in (2, 4, 6):
        spec = walk.make_spec(u, n, k, 0, 17, delta=delta)
        trials = 40000
        hits = sum(walk.distinguished(spec, walk.pack(x, b)) for x in range(trials // 2) for b in (0, 1))
        mean = trials / (1 << delta)
        sd = math.sqrt(trials * (1 / (1 << delta)) * (1 - 1 / (1 << delta)))
        assert abs(hits - mean) < 5 * sd


def test_start_points_in_range_and_deterministic():
    n, k = 2, 4
    _, u = target(n, k, 2)
    spec = walk.make_spec(u, n, k, 0, 5, delta=4)
    pts = [walk.start_point(spec, w, j) for w in range(20) for j in range(5)]
    assert pts == [walk.start_point(spec, w, j) for w in range(20) for j in range(5)]
    assert all(walk.unpack(p)[0] < spec.n_half for p in pts)
    sides = [walk.unpack(p)[1] for p in pts]
    assert 20 < sum(sides) < 80


def test_trails_merge_and_end_at_same_dp():
    n, k = 2, 4
    _, u = target(n, k, 3)
    spec = walk.make_spec(u, n, k, 0, 8, delta=3)
    # a trail can fall into a cycle without distinguished points (then it hits the cap and is
    # abandoned); take the first start whose trail ends
    for w in range(16):
        s0 = walk.start_point(spec, w, 0)
        dp0, d0 = walk.trail(spec, s0)
        if dp0 is not None:
            break
    assert dp0 is not None and d0 >= 1 and walk.distinguished(spec, dp0)
    # a trail started from the second point of trail 0 ends at the same place, one step sooner
    if d0 >= 2:
        s1 = walk.f(spec, s0)
        dp1, d1 = walk.trail(spec, s1)
        assert dp1 == dp0 and d1 == d0 - 1
    # trail points are all non-distinguished before the end
    pt = s0
    for _ in range(d0 - 1):
        pt = walk.f(spec, pt)
        assert not walk.distinguished(spec, pt)


def test_f_output_roughly_uniform():
    n, k = 2, 4
    _, u = target(n, k, 9)
    spec = walk.make_spec(u, n, k, 0, 21, delta=4)
    outs = [walk.f(spec, walk.pack(x, b)) for x in range(spec.n_half) for b in (0, 1)]
    sides = sum(walk.unpack(o)[1] for o in outs)
    assert abs(sides - len(outs) / 2) < 5 * math.sqrt(len(outs) / 4)
    xs = [walk.unpack(o)[0] for o in outs]
    assert abs(np.mean(xs) - spec.n_half / 2) < 0.1 * spec.n_half


def test_input_generator_and_oracle_mixers_agree():
    # two independent implementations of SplitMix64's published definition
    for s in (0, 1, 0xDEADBEEF, (1 << 64) - 1):
        for i in range(5):
            assert seeded_inputs.splitmix64(s, i) == walk.sm64(s, i)


def test_splitmix64_published_sequence():
    """The mixer is SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): from state 0 its reference
    generator's first three outputs are these published values."""
    assert [walk.sm64(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_collisions_of_f_match_a_random_mapping():
    """Appendix: in a space of N points a random mapping shows about N/2 colliding pairs (the `bad'
    collisions met before the golden one).  f is a random mapping on cosets: points whose half
    matrices lie in one left-Clifford coset collide by construction (grouped here by the exact
    canonical form), and G distinct cosets collide as a random mapping of G points into N would,
    G (G - 1) / (2 N) pairs in expectation (N (N - 1) / (2 N), about N/2, when every coset is
    distinct)."""
    from collections import Counter
    n, k = 2, 6
    _, u = target(n, k, 12)
    spec = walk.make_spec(u, n, k, 0, 77, delta=4)
    cosets = {}
    for x in range(spec.n_half):
        for b in (0, 1):
            cosets.setdefault(zmat.canonical_form(walk.half_matrix(spec, x, b)), []).append(walk.pack(x, b))
    big = max(cosets.values(), key=len)
    assert len({walk.f(spec, p) for p in big}) == 1        # one coset, one image
    reps = [v[0] for v in cosets.values()]
    g, N = len(reps), 2 * spec.n_half
    images = Counter(walk.f(spec, p) for p in reps)
    pairs = sum(c * (c - 1) // 2 for c in images.values())
    mean = g * (g - 1) / (2 * N)
    assert abs(pairs - mean) < 5 * math.sqrt(mean), (pairs, mean, g, N)


@pytest.mark.parametrize("delta", [1, 3])
def test_mean_trail_length_is_one_over_theta(delta):
    """Appendix: a trail runs 1/theta steps on average before it reaches a distinguished point (the
    number of steps is geometric with parameter theta when f behaves as a random mapping).  Each
    trail runs under its own function version (a re-salted f), so the trails are independent; under
    one version they merge and share their distinguished points.  At theta = 1/2 a step counted
    wrongly by one is 17 standard deviations out."""
    n, k = 2, 8
    _, u = target(n, k, 5)
    lens = []
    for v in range(600):
        spec = walk.make_spec(u, n, k, 0, 91, delta=delta, version=v)
        dp, d = walk.trail(spec, walk.start_point(spec, 0, 0))
        if dp is not None:
            lens.append(d)
    theta = 1.0 / (1 << delta)
    assert len(lens) >= 570   # a few trails fall into short cycles without distinguished points
    sd = math.sqrt(1 - theta) / theta / math.sqrt(len(lens))
    assert abs(sum(lens) / len(lens) - 1 / theta) < 5 * sd, (sum(lens) / len(lens), len(lens))
