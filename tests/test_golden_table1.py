"""Pins against values the paper prints: the optimal T-count 7 of the 3-qubit circuits of Table 1
(Sec. 5.2), read from tests/golden/table1_optimal_tcount.txt.  Here, on the CPU, the upper bound:
a product of exactly that many single rotations R(P) or R(P)^-1, with Clifford factors around it,
reproduces each gate's channel rep exactly (the phase polynomial of CCZ, then Hadamard and CNOT
conjugations).  The lower bound and the searches' T-count are checked on the GPU against the same
file (tests/test_gpu_named.py)."""

import numpy as np

import seeded_inputs
from golden_fixtures import table1
from oracle import unitary, zmat


def _channel_of_real(mats, e):
    m = np.array([[1]], dtype=np.int64)
    for x in mats:
        m = np.kron(m, np.array(x, dtype=np.int64))
    v = np.zeros(m.shape + (4,), dtype=np.int64)
    v[:, :, 0] = m
    return unitary.channel_of_unitary(3, v, e)


def _channel_of_perm(f):
    return unitary.channel_of_unitary(3, seeded_inputs.permutation_unitary(seeded_inputs._perm3(f)), 0)


def _named(name):
    return unitary.channel_of_unitary(3, seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES[name]), 0)


def test_table1_lists_the_named_gates():
    rows = table1()
    assert set(rows) == {"toffoli", "fredkin", "peres"}
    assert all(q == 3 for q, _ in rows.values())


def test_table1_tcount_is_reached_by_explicit_rotations():
    rows = table1()
    z0, z1, z2 = 8, 16, 32   # Z on qubits 0, 1, 2 (code = x | z << n)
    # CCZ = (-1)^(x0 x1 x2): R(Z_S) multiplies |x> by omega^(parity of x on S), and
    # 4 x0 x1 x2 = x0 + x1 + x2 - (x0^x1) - (x0^x2) - (x1^x2) + (x0^x1^x2), so CCZ is the product of
    # R(Z_S) for |S| = 1, 3 and R(Z_S)^-1 (channel rep: the transpose) for |S| = 2
    plus = [z0, z1, z2, z0 | z1 | z2]
    minus = [z0 | z1, z0 | z2, z1 | z2]
    ccz = zmat.product_of_rotations(plus, 3)
    ccz = zmat.product_of_rotations(minus, 3, start=ccz, transpose=True)
    n_rot = len(plus) + len(minus)
    h2 = _channel_of_real([np.eye(2), np.eye(2), [[1, 1], [1, -1]]], 1)
    tof = h2 @ ccz @ h2
    cnot_21 = _channel_of_perm(lambda a, b, c: (a, b ^ c, c))
    cnot_01 = _channel_of_perm(lambda a, b, c: (a, a ^ b, c))
    built = {"toffoli": tof, "fredkin": cnot_21 @ tof @ cnot_21, "peres": cnot_01 @ tof}
    for name, (_, t) in rows.items():
        assert n_rot == t, name
        assert built[name].equals(_named(name)), name
    # the Clifford factors carry no T: each is a signed permutation
    for cl in (h2, cnot_21, cnot_01):
        assert cl.is_signed_perm()
