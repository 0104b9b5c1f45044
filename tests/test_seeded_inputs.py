"""The seeded input recipe (no method arithmetic): Paulis uniform over the 4^n - 1 non-identity
codes, walk points uniform over [0, N_half) with either side, deterministic in the seed."""

import pytest

import seeded_inputs


def _chi2(counts, expected):
    return sum((c - expected) ** 2 / expected for c in counts)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_target_paulis_uniform_over_non_identity_codes(n):
    xi = 4 ** n - 1
    counts = [0] * (xi + 1)
    draws = 0
    for seed in range(400):
        tw = seeded_inputs.target_words(n, 7, seed)
        for p in tw.paulis + tw.clifford:
            counts[p] += 1
            draws += 1
    assert counts[0] == 0                      # never the identity
    # chi-square over xi cells: mean xi - 1, sd sqrt(2 (xi - 1)); allow 6 sd
    stat = _chi2(counts[1:], draws / xi)
    assert abs(stat - (xi - 1)) < 6 * (2 * (xi - 1)) ** 0.5, stat


def test_target_words_deterministic_and_seed_dependent():
    a = seeded_inputs.target_words(3, 6, 11)
    assert a == seeded_inputs.target_words(3, 6, 11)
    assert a.paulis != seeded_inputs.target_words(3, 6, 12).paulis
    assert len(a.paulis) == 6 and len(a.clifford) == 48


def test_random_points_cover_both_sides_uniformly():
    n_half = 255 ** 3
    pts = seeded_inputs.random_points(n_half, 20000, 5)
    xs = [p & 0xFFFFFFFF for p in pts]
    sides = [(p >> 32) & 1 for p in pts]
    assert all(0 <= x < n_half for x in xs) and set(sides) == {0, 1}
    assert abs(sum(sides) - 10000) < 6 * 70.8                  # binomial sd sqrt(20000 / 4)
    bins = [0] * 16
    for x in xs:
        bins[x * 16 // n_half] += 1
    assert abs(_chi2(bins, 1250) - 15) < 6 * (30 ** 0.5)


def test_array_generator_equals_scalar_one():
    """The vectorised generator draws exactly what the scalar SplitMix64 form draws, including
    bounds near 2^32 (the 64 x 32-bit multiply-high taken from two halves) and seeds near 2^64."""
    import numpy as np
    seeds = [0, 1, 7, (1 << 64) - 1, (1 << 63) + 12345, 0x6B]
    for bound in (1, 3, 63, 255, 1000003, (1 << 32) - 1):
        got = seeded_inputs.uniform_below_np(np.array(seeds, dtype=np.uint64), np.arange(len(seeds)), bound)
        want = [seeded_inputs.uniform_below(s, i, bound) for i, s in enumerate(seeds)]
        assert got.tolist() == want
    words, offsets, ks = seeded_inputs.mlp_target_arrays(123, 423)
    ref = seeded_inputs.mlp_targets(123, 423)
    assert ks.tolist() == [t.k for t in ref]
    for i, t in enumerate(ref):
        assert words[offsets[i]:offsets[i + 1]].tolist() == t.paulis + t.clifford
    assert offsets[0] == 0 and offsets[-1] == len(words)
