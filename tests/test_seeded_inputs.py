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
