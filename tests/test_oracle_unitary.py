"""Pins of the oracle's unitary -> channel rep route (Sec. 4.1 trace formula) and of the named
3-qubit gates of Sec. 5.2 (benchmarking known circuits), against closed forms and textbook identities."""

import numpy as np
import pytest

import seeded_inputs
from oracle import pauli, unitary, zmat
from oracle.cyclotomic import CycMat, rotation


def _coeffs_of_cycmat(m: CycMat):
    v = np.zeros(m.shape + (4,), dtype=np.int64)
    for a in range(4):
        v[:, :, a] = np.array(m.c[a], dtype=np.int64)
    return v


def _diag_signs(n, signs):
    d = 2 ** n
    v = np.zeros((d, d, 4), dtype=np.int64)
    for i, s in enumerate(signs):
        v[i, i, 0] = s
    return v


def _kron_coeffs(*mats):
    """Kronecker product of small real integer matrices, as Z[omega] coefficients (c0 only)."""
    m = np.array([[1]], dtype=np.int64)
    for x in mats:
        m = np.kron(m, np.array(x, dtype=np.int64))
    v = np.zeros(m.shape + (4,), dtype=np.int64)
    v[:, :, 0] = m
    return v


def _perm_coeffs_from_bits(f):
    return seeded_inputs.permutation_unitary(seeded_inputs._perm3(f))


def test_hadamard_closed_form():
    # H = (X + Z)/sqrt2: H X H = Z, H Z H = X, H Y H = -Y.  Codes at n = 1: X = 1, Z = 2, Y = 3.
    m = unitary.channel_of_unitary(1, _kron_coeffs([[1, 1], [1, -1]]), 1)
    want = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, -1]])
    assert m.e == 0 and np.array_equal(m.A.astype(int), want) and not m.B.any()


@pytest.mark.parametrize("n", [1, 2])
def test_pauli_unitary_is_signed_identity(n):
    # P_q P_i P_q = +P_i if they commute, -P_i otherwise
    for q in range(4 ** n):
        pm = pauli.matrix(q, n)
        v = np.zeros(pm.shape + (4,), dtype=np.int64)
        v[:, :, 0] = np.rint(pm.real).astype(np.int64)
        v[:, :, 2] = np.rint(pm.imag).astype(np.int64)  # i = omega^2
        m = unitary.channel_of_unitary(n, v, 0)
        want = np.diag([-1 if pauli.anticommutes(q, i, n) else 1 for i in range(4 ** n)])
        assert m.e == 0 and np.array_equal(m.A.astype(int), want) and not m.B.any()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_word_unitary_matches_column_rule(seed):
    # a Clifford+T word as an explicit matrix product of R(P) (denominator 2^d, i.e. sqrt2^(2d))
    # against the sparse column rule
    n = 2
    tw = seeded_inputs.target_words(n, 3, seed, clifford_len=4)
    u = CycMat.identity(n)
    for c in tw.clifford:
        u = u @ rotation(c, n) @ rotation(c, n)
    for p in reversed(tw.paulis):
        u = u @ rotation(p, n)
    got = unitary.channel_of_unitary(n, _coeffs_of_cycmat(u), 2 * u.d)
    want = zmat.target_from_words(n, tw.paulis, tw.clifford)
    assert got.equals(want)


def test_non_unitary_rejected():
    v = _kron_coeffs([[1, 1], [0, 1]])
    with pytest.raises(ValueError):
        unitary.channel_of_unitary(1, v, 0)


# Z-type Pauli codes at n = 3: z in bits 3..5, qubit j on z bit j.
Z0, Z1, Z2 = 8, 16, 32


def _ccz_hat():
    return unitary.channel_of_unitary(3, _diag_signs(3, [1] * 7 + [-1]), 0)


def test_ccz_phase_polynomial():
    # (-1)^(x0 x1 x2) = omega^(x0 + x1 + x2 - x0^x1 - x0^x2 - x1^x2 + x0^x1^x2), and R(Z_S) multiplies
    # |x> by omega^(parity of x on S): CCZ is the product of R(Z_S) for |S| odd and R(Z_S)^-1 for
    # |S| = 2; the channel rep of R^-1 is the transpose.
    m = zmat.product_of_rotations([Z0, Z1, Z2, Z0 | Z1 | Z2], 3)
    m = zmat.product_of_rotations([Z0 | Z1, Z0 | Z2, Z1 | Z2], 3, start=m, transpose=True)
    assert _ccz_hat().equals(m)


def _hat_of_perm(f):
    return unitary.channel_of_unitary(3, _perm_coeffs_from_bits(f), 0)


def test_toffoli_is_hadamard_conjugated_ccz():
    h2 = unitary.channel_of_unitary(3, _kron_coeffs(np.eye(2), np.eye(2), [[1, 1], [1, -1]]), 1)
    tof = unitary.channel_of_unitary(3, seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES["toffoli"]), 0)
    assert tof.equals(h2 @ _ccz_hat() @ h2)
    assert (tof @ tof).equals(zmat.ZMat.identity(3))


def test_fredkin_and_peres_from_toffoli():
    tof = unitary.channel_of_unitary(3, seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES["toffoli"]), 0)
    fred = unitary.channel_of_unitary(3, seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES["fredkin"]), 0)
    peres = unitary.channel_of_unitary(3, seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES["peres"]), 0)
    cnot_21 = _hat_of_perm(lambda a, b, c: (a, b ^ c, c))   # CNOT control q2, target q1
    cnot_01 = _hat_of_perm(lambda a, b, c: (a, a ^ b, c))   # CNOT control q0, target q1
    assert fred.equals(cnot_21 @ tof @ cnot_21)
    assert peres.equals(cnot_01 @ tof)
    # the three are distinct and none is Clifford (a Clifford channel rep is a signed permutation)
    assert not tof.equals(fred) and not tof.equals(peres) and not fred.equals(peres)
    for m in (tof, fred, peres):
        assert not m.is_signed_perm() and m.is_orthogonal()


def test_named_gates_are_permutations():
    for name, perm in seeded_inputs.NAMED_GATES.items():
        assert sorted(perm) == list(range(8)), name
    assert seeded_inputs.NAMED_GATES["toffoli"] == [0, 1, 2, 3, 4, 5, 7, 6]
    assert seeded_inputs.NAMED_GATES["fredkin"] == [0, 1, 2, 3, 4, 6, 5, 7]
    assert seeded_inputs.NAMED_GATES["peres"] == [0, 1, 2, 3, 6, 7, 5, 4]
