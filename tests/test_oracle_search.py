"""Pins for backtracking, claw checks and the search driver (Sec. 3, Fig. 2; Sec. 4.1)
against planted solutions, constructed merge cases and brute-force T-counts."""

import pytest

import seeded_inputs
from oracle import bfs, search, walk, zmat


def target(n, k, seed):
    tw = seeded_inputs.target_words(n, k, seed)
    return tw, zmat.target_from_words(n, tw.paulis, tw.clifford)


def test_claw_check_planted_and_reconstruct():
    for n, k, seed in [(2, 4, 1), (2, 5, 2), (3, 6, 3), (3, 3, 4)]:
        tw, u = target(n, k, seed)
        xv, xw, c = walk.planted_points(n, k, tw.paulis)
        spec = walk.make_spec(u, n, k, c, 1, delta=4)
        dec = search.claw_check(spec, walk.pack(xv, 0), walk.pack(xw, 1))
        assert dec is not None and dec.t == k
        assert search.reconstruct(n, dec).equals(u)
        # argument order does not matter
        assert search.claw_check(spec, walk.pack(xw, 1), walk.pack(xv, 0)) is not None


def test_claw_check_rejects_non_claws():
    n, k = 2, 4
    tw, u = target(n, k, 1)
    xv, xw, c = walk.planted_points(n, k, tw.paulis)
    spec = walk.make_spec(u, n, k, c, 1, delta=4)
    assert search.claw_check(spec, walk.pack((xv + 1) % spec.n_half, 0), walk.pack(xw, 1)) is None
    assert search.claw_check(spec, walk.pack(xv, 0), walk.pack(xv, 0)) is None


def _trail_points(spec, start, d):
    pts = [start]
    for _ in range(d):
        pts.append(walk.f(spec, pts[-1]))
    return pts


def test_backtrack_robin_hood():
    n, k = 2, 4
    _, u = target(n, k, 3)
    spec = walk.make_spec(u, n, k, 0, 8, delta=3)
    for j in range(30):
        s0 = walk.start_point(spec, 0, j)
        dp, d = walk.trail(spec, s0)
        if dp is not None and d >= 3:
            pts = _trail_points(spec, s0, d)
            kind, pair, _ = search.backtrack(spec, (s0, d), (pts[2], d - 2))
            assert kind == "robin_hood" and pair is None
            return
    pytest.fail("no trail of length >= 3")


def test_backtrack_finds_true_merge_point():
    # build two trails from random starts that end at the same DP, then check the
    # reported predecessors are distinct with equal images
    n, k = 2, 4
    _, u = target(n, k, 5)
    spec = walk.make_spec(u, n, k, 0, 12, delta=3)
    ends = {}
    found = None
    for j in range(400):
        s = walk.start_point(spec, 1, j)
        dp, d = walk.trail(spec, s)
        if dp is None:
            continue
        if dp in ends and ends[dp][0] != s:
            found = ((s, d), ends[dp])
            kind, pair, _ = search.backtrack(spec, *found)
            if kind == "robin_hood":
                continue
            a, b = pair
            assert a != b and walk.f(spec, a) == walk.f(spec, b)
            sa, sb = walk.unpack(a)[1], walk.unpack(b)[1]
            if kind == "same_side":
                assert sa == sb
            else:
                assert sa != sb
            return
        ends.setdefault(dp, (s, d))
    pytest.fail("no merged pair of trails found")


def test_search_plain_matches_bfs_n2():
    counts, seen, _ = bfs.cosets_by_tcount(2, 3)
    for seed, k in [(1, 2), (2, 3), (3, 3)]:
        tw, u = target(2, k, seed)
        res = search.search(u, 2, k_max=4, seed=42, delta_of_k=lambda kk: 3, walks=16)
        assert res.found
        t_min = bfs.min_tcount(u, seen)
        assert t_min is not None and res.decomposition.t == t_min
        assert search.reconstruct(2, res.decomposition).equals(u)


def test_search_walks_at_n2_k4():
    # the cfg1 shape: n = 2, k = 4 searched by walks (not enumeration), 64 walks, theta = 2^-4
    tw, u = target(2, 4, 1)
    res = search.search(u, 2, k_max=4, seed=1001, delta_of_k=lambda kk: 4, walks=64,
                        enum_max=32, depth_order=[4])
    assert res.found and res.decomposition.t == 4
    assert search.reconstruct(2, res.decomposition).equals(u)
    assert res.stats.dps > 0


def test_search_n1_finds_minimum():
    counts, seen, _ = bfs.cosets_by_tcount(1, 6)
    for seed in range(4):
        tw, u = target(1, 5, seed)
        res = search.search(u, 1, k_max=6, seed=3, delta_of_k=lambda kk: 2, walks=8)
        assert res.found
        assert res.decomposition.t == bfs.min_tcount(u, seen)
        assert search.reconstruct(1, res.decomposition).equals(u)


def test_clifford_target_is_depth_zero():
    d = zmat.clifford_from_word(2, seeded_inputs.random_clifford_word(2, 1))
    res = search.search(d, 2, k_max=2, seed=1, delta_of_k=lambda kk: 2)
    assert res.found and res.decomposition.t == 0
    assert search.reconstruct(2, res.decomposition).equals(d)
