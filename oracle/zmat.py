"""Exact channel representations over Z[1/sqrt2] (Sec. 4.1).

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

A matrix M is stored as two integer arrays A, B and one exponent e with
M = (A + B sqrt2) / sqrt2^e.  The representation is canonical when e is
minimal (reduce()).  Arithmetic is exact: object arrays of Python ints, or int64
only after a bound check shows no intermediate value can reach 2^62.

The sparse column rule for the channel rep of R(P_p) follows from
R(P) Q R(P)^dag = Q for commuting Q and (Q + s P_{p^q})/sqrt2 for anticommuting Q
(see pauli.rotation_sign); it is pinned against the trace formula in the tests.
"""

from __future__ import annotations

import numpy as np

from . import pauli

_SAFE = 1 << 62


def _as_obj(x):
    return np.array(x, dtype=object)


def _maxabs(x) -> int:
    if x.size == 0:
        return 0
    return int(max(abs(int(v)) for v in x.flat))


def _matmul(x, y):
    """Exact integer matrix product; int64 when a bound check proves it safe."""
    bound = _maxabs(x) * _maxabs(y) * x.shape[1]
    if bound < _SAFE:
        return _as_obj(np.dot(np.array(x, dtype=np.int64), np.array(y, dtype=np.int64)))
    return np.dot(_as_obj(x), _as_obj(y))


class ZMat:
    def __init__(self, A, B, e: int):
        self.A = _as_obj(A)
        self.B = _as_obj(B)
        self.e = int(e)

    # ---- constructors -------------------------------------------------
    @staticmethod
    def identity(n: int) -> "ZMat":
        r = 4 ** n
        A = np.zeros((r, r), dtype=object)
        for i in range(r):
            A[i, i] = 1
        return ZMat(A, np.zeros((r, r), dtype=object), 0)

    @staticmethod
    def signed_perm(perm, sign) -> "ZMat":
        """Column q holds sign[q] in row perm[q] (D P_q D^dag = sign[q] P_perm[q])."""
        r = len(perm)
        A = np.zeros((r, r), dtype=object)
        for q in range(r):
            A[perm[q], q] = int(sign[q])
        return ZMat(A, np.zeros((r, r), dtype=object), 0)

    def copy(self) -> "ZMat":
        return ZMat(self.A.copy(), self.B.copy(), self.e)

    @property
    def size(self) -> int:
        return self.A.shape[0]

    # ---- canonical representation ------------------------------------
    def reduce(self) -> "ZMat":
        """Divide out sqrt2 while every entry stays in Z[sqrt2]: (a + b sqrt2)/sqrt2 = b + (a/2) sqrt2."""
        A, B, e = self.A, self.B, self.e
        while e > 0 and bool(np.all(A % 2 == 0)):
            A, B, e = B, A // 2, e - 1
        return ZMat(A, B, e)

    def raise_to(self, e: int) -> "ZMat":
        """Same value with a larger exponent e: multiply X by sqrt2^(e - self.e)."""
        s = e - self.e
        if s < 0:
            raise ValueError("can only raise the exponent")
        A, B = self.A, self.B
        for _ in range(s):
            A, B = B * 2, A
        return ZMat(A, B, e)

    def equals(self, other: "ZMat") -> bool:
        a, b = self.reduce(), other.reduce()
        return a.e == b.e and np.array_equal(a.A, b.A) and np.array_equal(a.B, b.B)

    # ---- products -----------------------------------------------------
    def __matmul__(self, other: "ZMat") -> "ZMat":
        """(A1 + B1 s)(A2 + B2 s) = (A1A2 + 2 B1B2) + (A1B2 + B1A2) s, s = sqrt2."""
        A = _matmul(self.A, other.A) + 2 * _matmul(self.B, other.B)
        B = _matmul(self.A, other.B) + _matmul(self.B, other.A)
        return ZMat(A, B, self.e + other.e).reduce()

    def T(self) -> "ZMat":
        return ZMat(self.A.T.copy(), self.B.T.copy(), self.e)

    def is_orthogonal(self) -> bool:
        """X X^T = 2^e I exactly, with X = A + B sqrt2."""
        r = self.size
        rat = _matmul(self.A, self.A.T) + 2 * _matmul(self.B, self.B.T)
        irr = _matmul(self.A, self.B.T) + _matmul(self.B, self.A.T)
        eye = np.zeros((r, r), dtype=object)
        for i in range(r):
            eye[i, i] = 1 << self.e  # sqrt2^e * sqrt2^e = 2^e for any e
        return np.array_equal(rat, eye) and all(int(v) == 0 for v in irr.flat)

    def signed_perm_of(self):
        """(perm, sign) if M is a signed permutation matrix, else None."""
        m = self.reduce()
        if m.e != 0 or any(int(v) != 0 for v in m.B.flat):
            return None
        r = m.size
        perm = [-1] * r
        sign = [0] * r
        for q in range(r):
            col = [int(v) for v in m.A[:, q]]
            nz = [i for i, v in enumerate(col) if v != 0]
            if len(nz) != 1 or abs(col[nz[0]]) != 1:
                return None
            perm[q] = nz[0]
            sign[q] = col[nz[0]]
        if sorted(perm) != list(range(r)):
            return None
        return perm, sign

    def is_signed_perm(self) -> bool:
        return self.signed_perm_of() is not None

    # ---- the sparse right-multiplication by R_hat(p) -----------------
    def right_rot(self, p: int, n: int, transpose: bool = False) -> "ZMat":
        """M R_hat(p) (or M R_hat(p)^T) by the column rule, exponent raised by one.

        Column q of R_hat(p): e_q if <p,q> = 0, else (e_q + s(p,q) e_{p^q})/sqrt2.
        Hence (M R_hat)[:, q] = (M[:, q] + s M[:, p^q])/sqrt2 on anticommuting q, and
        M[:, q] (written sqrt2 M[:, q] / sqrt2) elsewhere.  R_hat(p)^T has row q equal to
        (e_q - s(p,q) e_{p^q})/sqrt2, because s(p, p^q) = -s(p, q) (orthogonality).
        """
        r = self.size
        A = np.zeros_like(self.A)
        B = np.zeros_like(self.B)
        for q in range(r):
            if pauli.anticommutes(p, q, n):
                s = pauli.rotation_sign(p, q, n)
                if transpose:
                    s = -s
                A[:, q] = self.A[:, q] + s * self.A[:, p ^ q]
                B[:, q] = self.B[:, q] + s * self.B[:, p ^ q]
            else:
                A[:, q] = 2 * self.B[:, q]
                B[:, q] = self.A[:, q]
        return ZMat(A, B, self.e + 1)


def rot_hat(p: int, n: int) -> ZMat:
    """Channel rep of R(P_p) by the column rule (reduced)."""
    return ZMat.identity(n).right_rot(p, n).reduce()


def product_of_rotations(paulis, n: int, start: ZMat | None = None, transpose: bool = False) -> ZMat:
    """start * R_hat(paulis[0]) * R_hat(paulis[1]) * ... (each optionally transposed), reduced."""
    m = ZMat.identity(n) if start is None else start
    for p in paulis:
        m = m.right_rot(p, n, transpose).reduce()
    return m


def target_from_words(n: int, paulis, clifford) -> ZMat:
    """U_hat = D_hat R_hat(P_k) ... R_hat(P_1) with D_hat = prod_j R_hat(C_j)^2.

    `paulis` is [P_1, ..., P_k]; `clifford` is [C_1, ..., C_m].
    """
    m = ZMat.identity(n)
    for c in clifford:
        m = m.right_rot(c, n).right_rot(c, n).reduce()
    for p in reversed(list(paulis)):
        m = m.right_rot(p, n).reduce()
    return m


def clifford_from_word(n: int, word) -> ZMat:
    return target_from_words(n, [], word)


def sqrt2_valuation(a: int, b: int) -> int:
    """Largest v with (a + b sqrt2)/sqrt2^v in Z[sqrt2]; None for zero."""
    if a == 0 and b == 0:
        return None

    def v2(x):
        if x == 0:
            return 10 ** 9
        return (x & -x).bit_length() - 1

    return min(2 * v2(a), 2 * v2(b) + 1)


def real_sign(a: int, b: int) -> int:
    """Sign of the real number a + b sqrt2, decided exactly."""
    if a >= 0 and b >= 0:
        return 0 if (a == 0 and b == 0) else 1
    if a <= 0 and b <= 0:
        return -1
    # opposite signs: compare a^2 with 2 b^2
    if a > 0:
        return 1 if a * a > 2 * b * b else -1
    return 1 if 2 * b * b > a * a else -1


def canonical_form(m: ZMat):
    """Exact canonical form of the left-Clifford coset {D_hat M : D_hat signed permutation}.

    Left multiplication by a signed permutation permutes and negates rows, so the
    coset is the multiset of rows up to sign.  Form: the minimal common exponent,
    each row negated if its first nonzero entry (lowest column code) is negative,
    rows sorted as integer tuples (a_0, b_0, a_1, b_1, ...).  Returns (e, rows).
    """
    m = m.reduce()
    rows = []
    for r in range(m.size):
        a = [int(v) for v in m.A[r]]
        b = [int(v) for v in m.B[r]]
        sgn = 0
        for q in range(m.size):
            sgn = real_sign(a[q], b[q])
            if sgn != 0:
                break
        if sgn < 0:
            a = [-v for v in a]
            b = [-v for v in b]
        rows.append(tuple(v for pair in zip(a, b) for v in pair))
    rows.sort()
    return m.e, tuple(rows)
