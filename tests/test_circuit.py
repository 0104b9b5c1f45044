"""Decompositions as gate lists (tcw_circuit, host code of the library) checked against the
oracle's exact gate matrices (Sec. 5.3).  No GPU needed: the synthesis runs on the host."""

import ctypes

import numpy as np
import pytest

import seeded_inputs
from oracle import circuit as ocircuit
from oracle import pauli, zmat
from oracle.cyclotomic import CycMat, rotation


def lib_or_skip():
    from paper_1606_07413_amd import tcw
    try:
        return tcw, tcw.load()
    except ImportError as e:  # the library is built by __graft_entry__.build()
        pytest.skip(str(e))


def make_result(tcw, n, paulis, clifford_word):
    """A verified-decomposition record for U = D R(P_k) ... R(P_1), D = prod R(C_j)^2, with D's action
    on Paulis taken from the oracle."""
    res = tcw.Result()
    res.status = 1
    res.n = n
    res.t = len(paulis)
    for i, p in enumerate(reversed(paulis)):   # P_t first
        res.paulis[i] = p
    perm, sign = zmat.clifford_from_word(n, clifford_word).signed_perm_of()
    for q in range(4 ** n):
        res.clifford_perm[q] = perm[q]
        res.clifford_sign[q] = sign[q]
    return res


# ---- pins of the oracle's gate matrices against definitions -----------------------------------

def _conj_code(gates, n, code):
    """U P_code U^dag for the circuit, as (sign, code), from explicit matrices."""
    u = ocircuit.circuit_unitary(n, gates).to_complex()
    p = pauli.matrix(code, n)
    img = u @ p @ u.conj().T
    for q in range(4 ** n):
        for s in (1, -1):
            if np.allclose(img, s * pauli.matrix(q, n)):
                return s, q
    raise AssertionError("not a Pauli")


def test_gate_matrices_textbook():
    # n = 1 codes: X = 1, Z = 2, Y = 3
    assert _conj_code([("h", (0,))], 1, 1) == (1, 2) and _conj_code([("h", (0,))], 1, 3) == (-1, 3)
    assert _conj_code([("s", (0,))], 1, 1) == (1, 3) and _conj_code([("s", (0,))], 1, 3) == (-1, 1)
    assert _conj_code([("sdg", (0,))], 1, 1) == (-1, 3)
    # CNOT(0 -> 1) at n = 2: X_0 -> X_0 X_1, Z_1 -> Z_0 Z_1 (x bits 0..1, z bits 2..3)
    assert _conj_code([("cx", (0, 1))], 2, 0b0001) == (1, 0b0011)
    assert _conj_code([("cx", (0, 1))], 2, 0b1000) == (1, 0b1100)
    # T is R(Z); T^2 = S; S^2 = Z; T T^dag = I (channel reps)
    assert ocircuit.circuit_channel(1, [("t", (0,))]).equals(zmat.rot_hat(2, 1))
    assert ocircuit.circuit_channel(1, [("t", (0,))] * 2).equals(ocircuit.circuit_channel(1, [("s", (0,))]))
    assert ocircuit.circuit_channel(1, [("s", (0,))] * 2).equals(ocircuit.circuit_channel(1, [("z", (0,))]))
    assert ocircuit.circuit_channel(1, [("t", (0,)), ("tdg", (0,))]).equals(zmat.ZMat.identity(1))


# ---- the library's synthesis -------------------------------------------------------------------

def _check(tcw, n, k, seed, clen):
    tw = seeded_inputs.target_words(n, k, seed, clifford_len=clen)
    res = make_result(tcw, n, tw.paulis, tw.clifford)
    gates = tcw.circuit_of(res)
    assert sum(1 for g, _ in gates if g in ("t", "tdg")) == k
    assert all(0 <= q < n for _, qs in gates for q in qs)
    want = zmat.target_from_words(n, tw.paulis, tw.clifford)
    assert ocircuit.circuit_channel(n, gates).equals(want), (n, k, seed)
    return gates


@pytest.mark.parametrize("n,k,seed,clen", [(1, 3, 1, 4), (1, 6, 2, 8), (2, 4, 3, 8), (2, 5, 4, 32), (3, 3, 5, 16),
                                           (3, 7, 6, 48)])
def test_circuit_reproduces_target(n, k, seed, clen):
    tcw, _ = lib_or_skip()
    _check(tcw, n, k, seed, clen)


@pytest.mark.parametrize("n,seed", [(1, 11), (2, 12), (3, 13), (3, 14)])
def test_circuit_of_clifford_only(n, seed):
    tcw, _ = lib_or_skip()
    gates = _check(tcw, n, 0, seed, 16 * n)
    assert not any(g in ("t", "tdg") for g, _ in gates)


def test_circuit_n4_up_to_phase():
    """n = 4 (the trace formula is slow there): the circuit's unitary equals the word's unitary up to a
    global phase omega^j."""
    tcw, _ = lib_or_skip()
    n = 4
    tw = seeded_inputs.target_words(n, 3, 21, clifford_len=12)
    gates = tcw.circuit_of(make_result(tcw, n, tw.paulis, tw.clifford))
    uc = ocircuit.circuit_unitary(n, gates)
    uw = CycMat.identity(n)
    for c in tw.clifford:
        uw = uw @ rotation(c, n) @ rotation(c, n)
    for p in reversed(tw.paulis):
        uw = uw @ rotation(p, n)
    assert any(uc.equals(uw.scale([int(a == j) for a in range(4)] if j < 4 else [-int(a == j - 4) for a in range(4)], 0))
               for j in range(8))


def test_circuit_errors():
    tcw, lib = lib_or_skip()
    res = tcw.Result()
    count = ctypes.c_int32(0)
    assert lib.tcw_circuit(ctypes.byref(res), None, 0, ctypes.byref(count)) == tcw.TCW_EINVAL  # status 0
    tw = seeded_inputs.target_words(2, 3, 5)
    res = make_result(tcw, 2, tw.paulis, tw.clifford)
    assert lib.tcw_circuit(ctypes.byref(res), None, 0, ctypes.byref(count)) == 0 and count.value > 3
    buf = (tcw.Gate * 2)()
    assert lib.tcw_circuit(ctypes.byref(res), buf, 2, ctypes.byref(count)) == tcw.TCW_EOVERFLOW
    res.clifford_perm[1] = 0   # the image of X_0 cannot be the identity
    assert lib.tcw_circuit(ctypes.byref(res), None, 0, ctypes.byref(count)) == tcw.TCW_EINVAL


def _gates(tcw, lib, res):
    count = ctypes.c_int32(0)
    rc = lib.tcw_circuit(ctypes.byref(res), None, 0, ctypes.byref(count))
    if rc:
        return rc
    buf = (tcw.Gate * max(1, count.value))()
    assert lib.tcw_circuit(ctypes.byref(res), buf, count.value, ctypes.byref(count)) == 0
    return [(g.kind, g.q0, g.q1) for g in buf[:count.value]]


@pytest.mark.parametrize("n,seed", [(1, 2), (2, 3), (3, 4), (4, 5)])
def test_circuit_validates_generator_images(n, seed):
    """Only the images of the generators X_j, Z_j (codes 1 << j) are read: an invalid one (code out of
    range or the identity, sign outside +-1) is refused; changing any other entry changes nothing."""
    tcw, lib = lib_or_skip()
    tw = seeded_inputs.target_words(n, 3, seed, clifford_len=6 * n)
    base = _gates(tcw, lib, make_result(tcw, n, tw.paulis, tw.clifford))
    assert isinstance(base, list)
    r = 4 ** n
    gens = [1 << j for j in range(2 * n)]
    for g in gens:
        for bad in (0, -7, r, r + 100):
            res = make_result(tcw, n, tw.paulis, tw.clifford)
            res.clifford_perm[g] = bad
            assert _gates(tcw, lib, res) == tcw.TCW_EINVAL
        for bad in (0, 2, -3):
            res = make_result(tcw, n, tw.paulis, tw.clifford)
            res.clifford_sign[g] = bad
            assert _gates(tcw, lib, res) == tcw.TCW_EINVAL
    others = [q for q in range(r) if q not in gens][:20]
    for q in others:
        res = make_result(tcw, n, tw.paulis, tw.clifford)
        res.clifford_perm[q] = r + 5
        res.clifford_sign[q] = 0
        assert _gates(tcw, lib, res) == base
    # Pauli codes outside 1 .. 4^n - 1 are refused
    for bad in (0, r, 65535):
        res = make_result(tcw, n, tw.paulis, tw.clifford)
        res.paulis[0] = bad
        assert _gates(tcw, lib, res) == tcw.TCW_EINVAL
