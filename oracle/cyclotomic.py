"""Exact matrices over Z[omega] / 2^d with omega = e^{i pi/4}.

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

Used only to evaluate the paper's definitions literally at small n:
R(P) = (1 + omega)/2 I + (1 - omega)/2 P (Sec. 4.1) and the channel
representation U_hat_ij = 2^-n Tr(P_i U P_j U^dag) (Sec. 4.1).

A matrix is four integer arrays C[0..3] (coefficients of omega^0..omega^3,
omega^4 = -1) and one denominator exponent d: value = sum_a C[a] omega^a / 2^d.
"""

from __future__ import annotations

import numpy as np

from . import pauli


class CycMat:
    def __init__(self, coeffs, d: int):
        self.c = [np.array(x, dtype=object) for x in coeffs]
        self.d = d

    @property
    def shape(self):
        return self.c[0].shape

    @staticmethod
    def from_pauli(q: int, n: int) -> "CycMat":
        """Pauli matrix: entries 0, +-1, +-i = +-omega^2."""
        m = pauli.matrix(q, n)
        re = np.rint(m.real).astype(int).astype(object)
        im = np.rint(m.imag).astype(int).astype(object)
        zero = np.zeros(m.shape, dtype=object)
        return CycMat([re, zero, im, zero.copy()], 0)

    @staticmethod
    def identity(n: int) -> "CycMat":
        return CycMat.from_pauli(0, n)

    def __matmul__(self, other: "CycMat") -> "CycMat":
        out = [np.zeros((self.shape[0], other.shape[1]), dtype=object) for _ in range(4)]
        for a in range(4):
            for b in range(4):
                prod = np.dot(self.c[a], other.c[b])
                k = a + b
                if k >= 4:
                    out[k - 4] = out[k - 4] - prod
                else:
                    out[k] = out[k] + prod
        return CycMat(out, self.d + other.d)

    def scale(self, coeffs, d: int) -> "CycMat":
        """Multiply every entry by the scalar sum_a coeffs[a] omega^a / 2^d."""
        out = [np.zeros(self.shape, dtype=object) for _ in range(4)]
        for a in range(4):
            for b in range(4):
                if coeffs[b] == 0:
                    continue
                prod = self.c[a] * coeffs[b]
                k = a + b
                if k >= 4:
                    out[k - 4] = out[k - 4] - prod
                else:
                    out[k] = out[k] + prod
        return CycMat(out, self.d + d)

    def __add__(self, other: "CycMat") -> "CycMat":
        d = max(self.d, other.d)
        s1 = 1 << (d - self.d)
        s2 = 1 << (d - other.d)
        return CycMat([self.c[a] * s1 + other.c[a] * s2 for a in range(4)], d)

    def dagger(self) -> "CycMat":
        """Conjugate transpose: conj(omega^a) = omega^-a = -omega^(4-a) for a = 1..3."""
        c0, c1, c2, c3 = (x.T for x in self.c)
        return CycMat([c0, -c3, -c2, -c1], self.d)

    def trace(self):
        return [sum(np.diagonal(x)) for x in self.c], self.d

    def to_complex(self) -> np.ndarray:
        w = np.exp(1j * np.pi / 4)
        m = sum(self.c[a].astype(complex) * w ** a for a in range(4))
        return m / (2.0 ** self.d)

    def equals(self, other: "CycMat") -> bool:
        d = max(self.d, other.d)
        s1 = 1 << (d - self.d)
        s2 = 1 << (d - other.d)
        return all(np.array_equal(self.c[a] * s1, other.c[a] * s2) for a in range(4))


def rotation(p: int, n: int) -> CycMat:
    """R(P_p) = (1 + omega)/2 I + (1 - omega)/2 P_p, exactly (Sec. 4.1)."""
    ident = CycMat.identity(n).scale([1, 1, 0, 0], 1)
    pm = CycMat.from_pauli(p, n).scale([1, -1, 0, 0], 1)
    return ident + pm


def real_to_zsqrt2(coeffs, d: int):
    """A real element of Z[omega]/2^d as (a, b, e) with value (a + b sqrt2)/sqrt2^e.

    Real means c2 = 0 and c3 = -c1; then the value is (c0 + c1 sqrt2)/2^d, since
    omega - omega^3 = sqrt2.
    """
    c0, c1, c2, c3 = coeffs
    if c2 != 0 or c3 != -c1:
        raise ValueError("element is not real")
    return c0, c1, 2 * d


def channel_rep_trace(u: CycMat, n: int):
    """U_hat_ij = 2^-n Tr(P_i U P_j U^dag) (Sec. 4.1), entry by entry.

    Returns (A, B, e) as object arrays with a common exponent e (not reduced).
    """
    r = 4 ** n
    ud = u.dagger()
    paulis = [CycMat.from_pauli(q, n) for q in range(r)]
    conj = [u @ paulis[j] @ ud for j in range(r)]
    entries = {}
    dmax = 0
    for i in range(r):
        for j in range(r):
            tr, d = (paulis[i] @ conj[j]).trace()
            a, b, e = real_to_zsqrt2(tr, d)
            e += 2 * n  # the 2^-n prefactor is sqrt2^-(2n)
            entries[i, j] = (a, b, e)
            dmax = max(dmax, e)
    A = np.zeros((r, r), dtype=object)
    B = np.zeros((r, r), dtype=object)
    for (i, j), (a, b, e) in entries.items():
        # bring to the common exponent dmax: multiply by sqrt2^(dmax - e)
        s = dmax - e
        if s % 2 == 0:
            A[i, j] = a * (1 << (s // 2))
            B[i, j] = b * (1 << (s // 2))
        else:
            # (a + b sqrt2) sqrt2 = 2b + a sqrt2
            A[i, j] = 2 * b * (1 << (s // 2))
            B[i, j] = a * (1 << (s // 2))
    return A, B, dmax
