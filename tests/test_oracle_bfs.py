"""Brute-force coset counts by T-count (the brute force of Sec. 3) against closed forms.

Level 1 has xi = 4^n - 1 cosets (one per non-identity Pauli).  Level 2: R(p)R(p)
is Clifford; R(p)R(q) = R(q)R(p) for commuting p != q; anticommuting ordered pairs
give distinct cosets.  Each non-identity Pauli commutes with 4^n/2 - 2 other
non-identity Paulis, so level 2 has xi (4^n/2 - 2)/2 + xi 4^n/2 cosets.
"""

import pytest

import seeded_inputs
from oracle import bfs, zmat


@pytest.mark.parametrize("n", [1, 2])
def test_level_counts_closed_form(n):
    counts, _, _ = bfs.cosets_by_tcount(n, 2)
    r = 4 ** n
    xi = r - 1
    assert counts[0] == 1
    assert counts[1] == xi
    assert counts[2] == xi * (r // 2 - 2) // 2 + xi * (r // 2)


def test_single_qubit_levels_double():
    # one qubit: the Matsumoto-Amano normal form (2008) has 3 choices for the first
    # T-syllable and 2 for each later one, so there are 3 * 2^(t-1) cosets of T-count t
    counts, _, _ = bfs.cosets_by_tcount(1, 6)
    assert counts[1:] == [3 * 2 ** (t - 1) for t in range(1, 7)]


def test_planted_targets_have_tcount_at_most_k():
    _, seen, _ = bfs.cosets_by_tcount(2, 3)
    for seed in range(6):
        for k in (1, 2, 3):
            tw = seeded_inputs.target_words(2, k, seed)
            u = zmat.target_from_words(2, tw.paulis, tw.clifford)
            t = bfs.min_tcount(u, seen)
            assert t is not None and t <= k


@pytest.mark.slow
def test_level4_n2():
    counts, seen, levels = bfs.cosets_by_tcount(2, 4)
    assert counts[:3] == [1, 15, 165]
    # every level-4 coset is a genuinely new class: none equals a lower level
    assert len(seen) == sum(counts)
