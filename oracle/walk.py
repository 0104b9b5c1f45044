"""The walk function of the deterministic-walk claw search (Sec. 2, Sec. 3).

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

A point is (x, b): x in [0, N_half) names a half-circuit of h = floor(k/2)
rotations, b in {0, 1} says which half (0: products from the identity, the
paper's z_1 / V side; 1: products from the target side, z_2 / W side).
f(x, b) = z_b(x) decodes x into Paulis (mu), forms the channel-rep product,
derives a string from the matrix entries (nu) and hashes it back to a point
(h followed by a reduction), Sec. 2 and Sec. 3.

This project's reading of the unspecified parts (the paper only asks for "a known
hash function" applied to information about every matrix element):

* Half-circuits.  Digits d_0 (least significant) .. d_{h-1} of x in base
  xi = 4^n - 1 give Paulis p_j = d_j + 1 (identity excluded, Sec. 4.1).
  Side 0: M = R(p_0) R(p_1) ... R(p_{h-1}).
  Side 1: M = S_c R(p_0)^T ... R(p_{h-1})^T with S_c = U R(c)^T for odd k
  (chunk c fixes P_1 = c; Sec. 3 splits the larger half into xi chunks), S = U
  for even k.  (Hats omitted: all matrices are channel representations.)
* Coset.  With the Clifford on the left (U = D R(P_t) ... R(P_1)), a claw is
  M_1 = D M_0, i.e. equal multisets of rows up to sign.  The hash is a function
  of that multiset only.
* Row digest.  phi: Z[1/sqrt2] -> Z/p, p = 2^61 - 1, sends sqrt2 to 2^31 (a
  square root of 2 mod p), hence 1/sqrt2 to 2^30.  S_r = sum_q K[q] phi(M_rq)
  mod p; D_r = min(S_r, p - S_r) (invariant under negating the row).
* Matrix hash.  An additive multiset hash of the digests (MSet-Add-Hash of Clarke,
  Devadas, van Dijk, Gassend, Suh, "Incremental multiset hash functions and their
  application to memory integrity checking", ASIACRYPT 2003):
  H = mix(sum_r g(D_r) mod 2^64), mix being SplitMix64's finaliser and g the element map
  g(D) = ((D mod 2^32 + a) mod 2^32) * ((floor(D / 2^32) + b) mod 2^32), with a and b the low
  and high 32 bits of salt_h: NH of Black, Halevi, Krawczyk, Krovetz and Rogaway (UMAC,
  CRYPTO 1999) on the digest's two 32-bit words.  A sum does not depend on the order of the
  rows, so no canonical sort is needed.
* Reduction.  x' = floor(H N_half / 2^64), b' = H mod 2.
* Distinguished points (Sec. 3, fraction theta = 2^-delta): the top delta bits
  of mix(((x << 1) | b) xor salt_d) are zero.
* Trail starts: g = sm64(salt_s, w 2^32 + j) for walk w, trail j;
  x_0 = floor(g N_half / 2^64), b_0 = g mod 2.  The start is not tested.
* Keys: sm64(s, i) = mix(s + (i+1) GAMMA) is the i-th SplitMix64 output from
  seed s.  From the search seed sigma: s_t = sm64(sigma, t) for t = 0..4;
  K[q] = (sm64(s_0, q) >> 3) mod p (s_1 is not used); with
  ctx = (version << 16) | (k << 8) | c: salt_h = sm64(s_2, ctx),
  salt_d = sm64(s_3, ctx), salt_s = sm64(s_4, ctx).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from . import zmat

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
P61 = (1 << 61) - 1
RHO = 1 << 31          # phi(sqrt2): (2^31)^2 = 2^62 = 2 * 2^61 = 2 (mod p)
RHO_INV = 1 << 30      # phi(1/sqrt2): 2^31 * 2^30 = 2^61 = 1 (mod p)


def mix64(z: int) -> int:
    """SplitMix64 output finaliser (Steele, Lea, Flood 2014)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sm64(seed: int, i: int) -> int:
    return mix64((seed + (i + 1) * GAMMA) & MASK64)


def mulhi64(a: int, b: int) -> int:
    return (a * b) >> 64


def pack(x: int, b: int) -> int:
    return x | (b << 32)


def unpack(pt: int) -> Tuple[int, int]:
    return pt & 0xFFFFFFFF, (pt >> 32) & 1


@dataclass
class Keys:
    K: List[int]
    salt_h: int
    salt_d: int
    salt_s: int


def make_keys(n: int, k: int, chunk: int, seed: int, version: int = 0) -> Keys:
    r = 4 ** n
    s = [sm64(seed, t) for t in range(5)]
    ctx = (version << 16) | (k << 8) | chunk
    return Keys(
        K=[(sm64(s[0], q) >> 3) % P61 for q in range(r)],
        salt_h=sm64(s[2], ctx),
        salt_d=sm64(s[3], ctx),
        salt_s=sm64(s[4], ctx),
    )


def phi(a: int, b: int, e: int) -> int:
    """Image of (a + b sqrt2)/sqrt2^e in Z/p."""
    return ((a + b * RHO) * pow(RHO_INV, e, P61)) % P61


def row_digests(m: zmat.ZMat, K: List[int]) -> List[int]:
    """D_r = min(S_r, p - S_r), S_r = sum_q K[q] phi(M_rq) mod p."""
    scale = pow(RHO_INV, m.e, P61)
    out = []
    for r in range(m.size):
        s = 0
        for q in range(m.size):
            a, b = int(m.A[r, q]), int(m.B[r, q])
            if a or b:
                s += K[q] * (((a + b * RHO) * scale) % P61)
        s %= P61
        out.append(min(s, P61 - s))
    return out


def nh_element(d: int, salt: int) -> int:
    """NH on the two 32-bit words of d, keyed by the two words of salt: a 64-bit product."""
    m32 = 0xFFFFFFFF
    a, b = salt & m32, salt >> 32
    return (((d & m32) + a) & m32) * (((d >> 32) + b) & m32)


def matrix_hash(m: zmat.ZMat, keys: Keys) -> int:
    """H = mix(sum over rows of g(D_r), mod 2^64), g the NH element map: a function of the
    multiset of sign-normalised row digests, i.e. of the left-Clifford coset."""
    acc = 0
    for v in row_digests(m, keys.K):
        acc += nh_element(v, keys.salt_h)
    return mix64(acc & MASK64)


@dataclass
class Spec:
    """One (target, depth k, chunk c) search space with its walk parameters."""

    n: int
    k: int
    chunk: int            # 0 for even k, else 1..xi
    S: zmat.ZMat          # S_c (target side start matrix)
    keys: Keys
    delta: int

    @property
    def xi(self) -> int:
        return 4 ** self.n - 1

    @property
    def h(self) -> int:
        return self.k // 2

    @property
    def n_half(self) -> int:
        return self.xi ** self.h


def chunk_matrix(u: zmat.ZMat, n: int, k: int, chunk: int) -> zmat.ZMat:
    """S_c = U R(c)^T for odd k (chunk c = P_1), S = U for even k."""
    if k % 2 == 1:
        if not 1 <= chunk <= 4 ** n - 1:
            raise ValueError("odd k needs a chunk in 1..xi")
        return u.right_rot(chunk, n, transpose=True).reduce()
    if chunk != 0:
        raise ValueError("even k has the single chunk 0")
    return u.reduce()


def make_spec(u: zmat.ZMat, n: int, k: int, chunk: int, seed: int, delta: int, version: int = 0) -> Spec:
    return Spec(n=n, k=k, chunk=chunk, S=chunk_matrix(u, n, k, chunk),
                keys=make_keys(n, k, chunk, seed, version), delta=delta)


def decode(x: int, n: int, h: int) -> List[int]:
    xi = 4 ** n - 1
    ps = []
    for _ in range(h):
        ps.append(x % xi + 1)
        x //= xi
    return ps


def encode(paulis: List[int], n: int) -> int:
    xi = 4 ** n - 1
    x = 0
    for p in reversed(paulis):
        x = x * xi + (p - 1)
    return x


def half_matrix(spec: Spec, x: int, b: int) -> zmat.ZMat:
    ps = decode(x, spec.n, spec.h)
    if b == 0:
        return zmat.product_of_rotations(ps, spec.n)
    return zmat.product_of_rotations(ps, spec.n, start=spec.S, transpose=True)


def f_with_hash(spec: Spec, pt: int) -> Tuple[int, int]:
    """(f(pt), H): one walk step and the matrix hash it came from."""
    x, b = unpack(pt)
    m = half_matrix(spec, x, b)
    hsh = matrix_hash(m, spec.keys)
    return pack(mulhi64(hsh, spec.n_half), hsh & 1), hsh


def f(spec: Spec, pt: int) -> int:
    return f_with_hash(spec, pt)[0]


def distinguished(spec: Spec, pt: int) -> bool:
    if spec.delta == 0:
        return True
    x, b = unpack(pt)
    return (mix64(((x << 1) | b) ^ spec.keys.salt_d) >> (64 - spec.delta)) == 0


def start_point(spec: Spec, w: int, j: int) -> int:
    g = sm64(spec.keys.salt_s, (w << 32) | j)
    return pack(mulhi64(g, spec.n_half), g & 1)


def trail_cap(delta: int, cap_factor: int = 20) -> int:
    return cap_factor << delta


def trail(spec: Spec, start: int, cap: Optional[int] = None) -> Tuple[Optional[int], int]:
    """Walk from `start` until the next point is distinguished (Sec. 3).

    Returns (dp, d) with d >= 1 the number of steps, or (None, 0) if no
    distinguished point was reached within `cap` steps (trail abandoned).
    """
    cap = trail_cap(spec.delta) if cap is None else cap
    pt = start
    for d in range(1, cap + 1):
        pt = f(spec, pt)
        if distinguished(spec, pt):
            return pt, d
    return None, 0


def planted_points(n: int, k: int, paulis: List[int]) -> Tuple[int, int, int]:
    """(x_V, x_W, chunk) of the claw planted in U = D R(P_k) ... R(P_1).

    V = R(P_k) ... R(P_{k-h+1}) and W = S_c R(P_{1+eps})^T ... R(P_{h+eps})^T = D V,
    eps = k mod 2, chunk = P_1 for odd k.
    """
    h = k // 2
    eps = k % 2
    pv = [paulis[k - 1 - j] for j in range(h)]          # p_j = P_{k-j}
    pw = [paulis[eps + j] for j in range(h)]            # q_j = P_{1+eps+j}
    chunk = paulis[0] if eps else 0
    return encode(pv, n), encode(pw, n), chunk
