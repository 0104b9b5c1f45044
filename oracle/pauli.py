"""n-qubit Paulis in binary symplectic form (Sec. 4.1: each R(P) is named by a Pauli,
written as a binary string through the symplectic representation).

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

Code layout (this project's reading; the paper fixes only that the encoding is
binary symplectic): a code q in [0, 4^n) has x = q mod 2^n (low n bits) and
z = q >> n.  Qubit j carries bit j of x and of z; qubit 0 is the leftmost factor
of the Kronecker product.  sigma(0,0)=I, sigma(1,0)=X, sigma(1,1)=Y, sigma(0,1)=Z.
"""

from __future__ import annotations

import numpy as np

I2 = np.array([[1, 0], [0, 1]], dtype=complex)
X2 = np.array([[0, 1], [1, 0]], dtype=complex)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z2 = np.array([[1, 0], [0, -1]], dtype=complex)
_SIGMA = {(0, 0): I2, (1, 0): X2, (1, 1): Y2, (0, 1): Z2}


def split(q: int, n: int):
    return q & ((1 << n) - 1), q >> n


def popcount(v: int) -> int:
    return bin(v).count("1")


def anticommutes(a: int, b: int, n: int) -> bool:
    """Symplectic inner product <a, b> = x_a.z_b + z_a.x_b (mod 2)."""
    xa, za = split(a, n)
    xb, zb = split(b, n)
    return (popcount(xa & zb) + popcount(za & xb)) % 2 == 1


def product_phase(a: int, b: int, n: int) -> int:
    """c in Z/4 with P_a P_b = i^c P_{a xor b}.

    Derivation: per qubit sigma(x,z) = i^{xz} X^x Z^z, and Z^z X^x = (-1)^{xz} X^x Z^z,
    so P_a P_b = i^{x_a.z_a + x_b.z_b - (x_a^x_b).(z_a^z_b) + 2 z_a.x_b} P_{a^b}.
    """
    xa, za = split(a, n)
    xb, zb = split(b, n)
    c = popcount(xa & za) + popcount(xb & zb) - popcount((xa ^ xb) & (za ^ zb)) + 2 * popcount(za & xb)
    return c % 4


def matrix(q: int, n: int) -> np.ndarray:
    """Explicit 2^n x 2^n matrix of P_q (textbook Kronecker product; entries 0, +-1, +-i exactly)."""
    x, z = split(q, n)
    m = np.array([[1]], dtype=complex)
    for j in range(n):
        m = np.kron(m, _SIGMA[((x >> j) & 1, (z >> j) & 1)])
    return m


def rotation_sign(p: int, q: int, n: int) -> int:
    """Sign s(p, q) of the off-diagonal entry in column q of the channel rep of R(P_p).

    For <p,q> = 1, R(P) P_q R(P)^dag = (P_q - i P_p P_q)/sqrt2 = (P_q + s P_{p^q})/sqrt2,
    with -i * i^c = +1 for c = 1 and -1 for c = 3.
    """
    c = product_phase(p, q, n)
    if c == 1:
        return 1
    if c == 3:
        return -1
    raise ValueError("s(p, q) is defined only for anticommuting p, q")
