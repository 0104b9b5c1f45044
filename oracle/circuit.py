"""Exact unitaries of gate lists over {H, S, S^dag, CNOT, T, T^dag, X, Y, Z} (Sec. 5.3: the output of
synthesis as a circuit).

Test infrastructure only: imported by the tests, never by the library.

Each gate is its textbook matrix over Z[omega] / 2^d (omega = e^{i pi/4}): H = (X + Z)/sqrt2 with
1/sqrt2 = (omega - omega^3)/2, S = diag(1, i), T = diag(1, omega), CNOT the basis permutation
|c, t> -> |c, t xor c>; a gate on qubit q of n is the Kronecker product with identities, qubit 0
the leftmost factor.  The circuit's unitary is the product in application order (first gate
rightmost); its channel rep comes from the trace formula (cyclotomic.channel_rep_trace).
"""

from __future__ import annotations

import numpy as np

from .cyclotomic import CycMat, channel_rep_trace
from .zmat import ZMat


def _one_qubit(name: str) -> CycMat:
    z = np.zeros((2, 2), dtype=object)
    if name == "h":
        return CycMat([np.array([[1, 1], [1, -1]], dtype=object), z, z.copy(), z.copy()], 0).scale([0, 1, 0, -1], 1)
    if name in ("s", "sdg", "t", "tdg"):
        c = [np.array([[1, 0], [0, 0]], dtype=object), z.copy(), z.copy(), z.copy()]
        if name == "s":
            c[2][1, 1] = 1            # i = omega^2
        elif name == "sdg":
            c[2][1, 1] = -1           # -i
        elif name == "t":
            c[1][1, 1] = 1            # omega
        else:
            c[3][1, 1] = -1           # omega^7 = -omega^3
        return CycMat(c, 0)
    code = {"x": 1, "z": 2, "y": 3}[name]  # n = 1 codes: X = x bit, Z = z bit
    return CycMat.from_pauli(code, 1)


def _embed(g: CycMat, q: int, n: int) -> CycMat:
    eye = np.eye(2, dtype=int).astype(object)
    zero = np.zeros((2, 2), dtype=object)
    out = [np.array([[1]], dtype=object), np.zeros((1, 1), dtype=object), np.zeros((1, 1), dtype=object),
           np.zeros((1, 1), dtype=object)]
    d = 0
    for j in range(n):
        if j == q:
            f, fd = g.c, g.d
        else:
            f, fd = [eye, zero, zero, zero], 0
        new = [np.zeros((out[0].shape[0] * 2, out[0].shape[1] * 2), dtype=object) for _ in range(4)]
        for a in range(4):
            for b in range(4):
                prod = np.kron(out[a], f[b])
                k = a + b
                if k >= 4:
                    new[k - 4] = new[k - 4] - prod
                else:
                    new[k] = new[k] + prod
        out, d = new, d + fd
    return CycMat(out, d)


def _cnot(c: int, t: int, n: int) -> CycMat:
    dim = 2 ** n
    m = np.zeros((dim, dim), dtype=object)
    for b in range(dim):
        cb = (b >> (n - 1 - c)) & 1
        m[b ^ (cb << (n - 1 - t)), b] = 1
    z = np.zeros((dim, dim), dtype=object)
    return CycMat([m, z, z.copy(), z.copy()], 0)


def gate_unitary(name: str, qubits, n: int) -> CycMat:
    if name == "cx":
        return _cnot(qubits[0], qubits[1], n)
    return _embed(_one_qubit(name), qubits[0], n)


def circuit_unitary(n: int, gates) -> CycMat:
    """U = G_m ... G_1 for gates [(name, qubits), ...] in application order."""
    u = CycMat.identity(n)
    for name, qubits in gates:
        u = gate_unitary(name, qubits, n) @ u
        # keep the denominator small: divide by 2 while every coefficient is even
        while u.d > 0 and all(not (x % 2).any() for x in u.c):
            u = CycMat([x // 2 for x in u.c], u.d - 1)
    return u


def circuit_channel(n: int, gates) -> ZMat:
    A, B, e = channel_rep_trace(circuit_unitary(n, gates), n)
    return ZMat(A, B, e).reduce()
