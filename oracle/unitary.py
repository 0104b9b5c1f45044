"""Channel representation of a unitary given exactly over Z[omega] (Sec. 4.1, trace formula).

Test infrastructure only: imported by the tests and the benchmark's CPU baseline, never by the
library.

A unitary is U = V / sqrt2^e with V a d x d array (d = 2^n) of elements of Z[omega],
omega = e^{i pi/4}, each given as four integers (c0, c1, c2, c3) meaning
c0 + c1 omega + c2 omega^2 + c3 omega^3.  Since sqrt2 = omega - omega^3, the factor 1/sqrt2 is
(omega - omega^3)/2, so U is an exact CycMat.  Its channel rep U_hat_ij = 2^-n Tr(P_i U P_j U^dag)
is evaluated entry by entry by cyclotomic.channel_rep_trace and returned as a reduced ZMat.
"""

from __future__ import annotations

import numpy as np

from .cyclotomic import CycMat, channel_rep_trace
from .zmat import ZMat


def cycmat_of(v, e: int) -> CycMat:
    """The exact matrix V / sqrt2^e as a CycMat (denominator a power of 2)."""
    v = np.asarray(v)
    if v.ndim != 3 or v.shape[0] != v.shape[1] or v.shape[2] != 4:
        raise ValueError("V must be d x d x 4")
    m = CycMat([v[:, :, a].astype(object) for a in range(4)], 0)
    if e % 2:
        m = m.scale([0, 1, 0, -1], 1)  # times (omega - omega^3)/2 = 1/sqrt2
    return CycMat(m.c, m.d + e // 2)


def is_unitary(u: CycMat) -> bool:
    d = u.shape[0]
    eye = CycMat([np.eye(d, dtype=int).astype(object)] + [np.zeros((d, d), dtype=object) for _ in range(3)], 0)
    return (u @ u.dagger()).equals(eye)


def channel_of_unitary(n: int, v, e: int) -> ZMat:
    """Reduced exact channel rep of U = V / sqrt2^e; ValueError if U is not unitary."""
    u = cycmat_of(v, e)
    if u.shape[0] != 2 ** n:
        raise ValueError("V must be 2^n x 2^n")
    if not is_unitary(u):
        raise ValueError("U is not unitary")
    A, B, ee = channel_rep_trace(u, n)
    return ZMat(A, B, ee).reduce()
