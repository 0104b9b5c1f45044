"""Pins for oracle.pauli against explicit textbook Pauli matrices (Sec. 4.1)."""

import itertools

import numpy as np
import pytest

from oracle import pauli


@pytest.mark.parametrize("n", [1, 2])
def test_product_phase_against_explicit_matrices(n):
    r = 4 ** n
    for a, b in itertools.product(range(r), repeat=2):
        lhs = pauli.matrix(a, n) @ pauli.matrix(b, n)
        c = pauli.product_phase(a, b, n)
        rhs = (1j ** c) * pauli.matrix(a ^ b, n)
        assert np.array_equal(lhs, rhs), (a, b, c)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_commutation_against_explicit_matrices(n):
    r = 4 ** n
    rng = np.random.default_rng(n)
    pairs = list(itertools.product(range(r), repeat=2)) if n < 3 else [tuple(rng.integers(0, r, 2)) for _ in range(200)]
    for a, b in pairs:
        pa, pb = pauli.matrix(int(a), n), pauli.matrix(int(b), n)
        anti = pauli.anticommutes(int(a), int(b), n)
        assert np.array_equal(pa @ pb, (-1 if anti else 1) * (pb @ pa))


def test_single_qubit_layout():
    # x bits low, z bits high: code 1 = X, 2 = Z, 3 = Y (x = z = 1)
    assert np.array_equal(pauli.matrix(1, 1), pauli.X2)
    assert np.array_equal(pauli.matrix(2, 1), pauli.Z2)
    assert np.array_equal(pauli.matrix(3, 1), pauli.Y2)
    # qubit 0 is the leftmost Kronecker factor
    assert np.array_equal(pauli.matrix(1, 2), np.kron(pauli.X2, pauli.I2))


def test_each_pauli_anticommutes_with_half():
    # a non-identity Pauli anticommutes with exactly half of all 4^n Paulis
    for n in (1, 2, 3):
        r = 4 ** n
        for p in range(1, r):
            assert sum(pauli.anticommutes(p, q, n) for q in range(r)) == r // 2


def test_rotation_sign_antisymmetric_in_pair():
    # s(p, p^q) = -s(p, q): the 2x2 block of R_hat(p) on {q, p^q} is orthogonal
    for n in (1, 2):
        r = 4 ** n
        for p in range(1, r):
            for q in range(r):
                if pauli.anticommutes(p, q, n):
                    assert pauli.rotation_sign(p, p ^ q, n) == -pauli.rotation_sign(p, q, n)
