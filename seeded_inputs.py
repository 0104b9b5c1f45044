"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This module only draws random numbers and states workload shapes.  It holds none
of the synthesis method's arithmetic: no channel representations, no hashing of
matrices, no walk.  Both the CPU oracle and the HIP library receive what it
produces as plain integer lists.

Random numbers come from SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), used in its
counter form: the i-th output (i = 0, 1, ...) of a generator seeded with s is
mix(s + (i + 1) * GAMMA mod 2^64).

Target recipe (used by every synthetic workload): a seeded product of k
rotations R(P) with P uniform over the 4^n - 1 non-identity Pauli codes, times a
seeded Clifford D built as R(C_1)^2 R(C_2)^2 ... R(C_m)^2 with m = 16 n (each
R(C)^2 is a Clifford; such products reach the whole Clifford group up to phase).
The target unitary is U = D R(P_k) ... R(P_1) up to global phase.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64(seed: int, i: int) -> int:
    """i-th output of SplitMix64 seeded with `seed` (counter form)."""
    return _mix((seed + (i + 1) * GAMMA) & MASK64)


def uniform_below(seed: int, i: int, bound: int) -> int:
    """floor(r * bound / 2^64) for the i-th SplitMix64 output r (Lemire's multiply-high)."""
    return (splitmix64(seed, i) * bound) >> 64


@dataclass
class TargetWords:
    """Integer description of a seeded target: U = D R(P_k) ... R(P_1), D = prod R(C_j)^2."""

    n: int
    k: int
    seed: int
    paulis: List[int]          # [P_1, ..., P_k], each in 1 .. 4^n - 1
    clifford: List[int] = field(default_factory=list)  # [C_1, ..., C_m]


def target_words(n: int, k: int, seed: int, clifford_len: int | None = None) -> TargetWords:
    """Seeded target: k rotation Paulis then m = 16 n Clifford-word Paulis from one stream."""
    if not 1 <= n <= 4:
        raise ValueError("n must be in 1..4")
    xi = 4 ** n - 1
    m = 16 * n if clifford_len is None else clifford_len
    paulis = [uniform_below(seed, i, xi) + 1 for i in range(k)]
    clifford = [uniform_below(seed, k + j, xi) + 1 for j in range(m)]
    return TargetWords(n=n, k=k, seed=seed, paulis=paulis, clifford=clifford)


def random_clifford_word(n: int, seed: int, length: int | None = None) -> List[int]:
    """Paulis C_1..C_m of a seeded Clifford D = R(C_1)^2 ... R(C_m)^2 (used for invariance tests)."""
    xi = 4 ** n - 1
    m = 16 * n if length is None else length
    return [uniform_below(seed ^ 0xC11F, j, xi) + 1 for j in range(m)]


def random_points(n_half: int, count: int, seed: int) -> List[int]:
    """Seeded packed walk points: x in bits 0..31 uniform below n_half, side in bit 32."""
    out = []
    for i in range(count):
        r = splitmix64(seed, i)
        x = (r * n_half) >> 64
        out.append(x | ((r & 1) << 32))
    return out


# Workload shapes of the five benchmark configurations.  Sizes follow the
# paper's search-space definitions: xi = 4^n - 1 rotations per layer, halves of
# floor(k/2) rotations, odd depths split into xi chunks.
WORKLOADS = {
    "n2k4": dict(n=2, k=4, target_seeds=list(range(1, 17)), walks=64, delta=4, log2_table=10,
                 walk_seed_base=1000),
    "n3k6": dict(n=3, k=6, target_seeds=list(range(1, 9)), walks=1 << 16, delta=8, log2_table=20,
                 walk_seed_base=2000),
    "n4k7": dict(n=4, k=7, target_seeds=list(range(1, 5)), walks=1 << 20, delta=12, log2_table=26,
                 walk_seed_base=3000),
    "batch64": dict(count=64, batch_seed=7, n_choices=(2, 3, 4), k_choices=(3, 4, 5, 6, 7),
                    target_seed_base=100, delta_by_n={2: 4, 3: 8, 4: 12}),
    "mlp_n3": dict(n=3, k_range=(1, 10), train_seeds=(0, 1_000_000), eval_seeds=(1_000_000, 1_000_256),
                   batch=4096, init_seed=42, hidden=512, depth=3, classes=11),
}


def batch_targets(count: int = 64, batch_seed: int = 7, seed_base: int = 100):
    """Mixed batch: (n, k) uniform over {2,3,4} x {3..7}, target seeds seed_base + i."""
    out = []
    for i in range(count):
        n = (2, 3, 4)[uniform_below(batch_seed, 2 * i, 3)]
        k = 3 + uniform_below(batch_seed, 2 * i + 1, 5)
        out.append(target_words(n, k, seed_base + i))
    return out


def mlp_init(inp: int, hidden: int, depth: int, classes: int, seed: int):
    """Seeded initial weights of the depth-order network, float32: W_l uniform in
    [-1/sqrt(fan_in), 1/sqrt(fan_in)] (row-major in x out), biases zero.  Values come from the
    SplitMix64 stream of `seed`, 24 bits each: u = (r >> 40) / 2^24."""
    import numpy as np
    sizes = [inp] + [hidden] * depth + [classes]
    params = {}
    idx = 0
    for l in range(depth + 1):
        fi, fo = sizes[l], sizes[l + 1]
        count = fi * fo
        i = np.arange(idx, idx + count, dtype=np.uint64)
        z = (np.uint64(seed) + (i + np.uint64(1)) * np.uint64(GAMMA))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        u = (z >> np.uint64(40)).astype(np.float64) / float(1 << 24)
        bound = 1.0 / np.sqrt(fi)
        params[f"W{l}"] = ((2.0 * u - 1.0) * bound).astype(np.float32).reshape(fi, fo)
        params[f"b{l}"] = np.zeros(fo, dtype=np.float32)
        idx += count
    return params


def mlp_targets(seed_lo: int, seed_hi: int, n: int = 3, k_lo: int = 1, k_hi: int = 10):
    """Seeded circuits for the depth-order network: seed s gives k = k_lo + uniform_below(s', 0,
    k_hi - k_lo + 1) (s' = s xor 0x6B) rotations times a seeded Clifford."""
    out = []
    for s in range(seed_lo, seed_hi):
        k = k_lo + uniform_below(s ^ 0x6B, 0, k_hi - k_lo + 1)
        out.append(target_words(n, k, s))
    return out


def _mix_np(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def uniform_below_np(seeds, i, bound: int):
    """uniform_below over arrays: seeds and i broadcast (uint64 arithmetic wraps mod 2^64 as the scalar
    form's masks do); the 64 x 32-bit multiply-high is taken from the two 32-bit halves of r."""
    if not 1 <= bound < (1 << 32):
        raise ValueError("bound must be in 1 .. 2^32 - 1")
    seeds = np.asarray(seeds, dtype=np.uint64)
    i = np.asarray(i, dtype=np.uint64)
    with np.errstate(over="ignore"):
        r = _mix_np(seeds + (i + np.uint64(1)) * np.uint64(GAMMA))
    b = np.uint64(bound)
    hi, lo = r >> np.uint64(32), r & np.uint64(0xFFFFFFFF)
    return ((hi * b + ((lo * b) >> np.uint64(32))) >> np.uint64(32)).astype(np.int64)


def mlp_target_arrays(seed_lo: int, seed_hi: int, n: int = 3, k_lo: int = 1, k_hi: int = 10):
    """The targets of mlp_targets(seed_lo, seed_hi, n, k_lo, k_hi) as flat arrays: words (uint16,
    every target's k rotation Paulis then its 16 n Clifford Paulis), offsets (int32, count + 1) and
    ks (int32)."""
    seeds = np.arange(seed_lo, seed_hi, dtype=np.uint64)
    ks = (k_lo + uniform_below_np(seeds ^ np.uint64(0x6B), 0, k_hi - k_lo + 1)).astype(np.int32)
    m = 16 * n
    lens = ks.astype(np.int64) + m
    offsets = np.zeros(len(seeds) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    owner = np.repeat(np.arange(len(seeds)), lens)
    pos = np.arange(total, dtype=np.int64) - offsets[:-1][owner]
    words = (uniform_below_np(seeds[owner], pos.astype(np.uint64), 4 ** n - 1) + 1).astype(np.uint16)
    return words, offsets.astype(np.int32), ks


# Named 3-qubit reversible gates (Sec. 5.2, benchmarking known circuits), from their textbook
# definitions as permutations of the computational basis.  Qubit 0 is the leftmost Kronecker
# factor, so a basis index is 4 q0 + 2 q1 + q2.  perm[i] is the image of basis state i.
def _perm3(f):
    out = []
    for i in range(8):
        q0, q1, q2 = (i >> 2) & 1, (i >> 1) & 1, i & 1
        a, b, c = f(q0, q1, q2)
        out.append(4 * a + 2 * b + c)
    return out


NAMED_GATES = {
    # Toffoli: q2 ^= q0 q1
    "toffoli": _perm3(lambda a, b, c: (a, b, c ^ (a & b))),
    # Fredkin: controlled swap of q1 and q2, control q0
    "fredkin": _perm3(lambda a, b, c: (a, c, b) if a else (a, b, c)),
    # Peres: (a, b, c) -> (a, a ^ b, c ^ a b), a Toffoli followed by CNOT q0 -> q1
    "peres": _perm3(lambda a, b, c: (a, a ^ b, c ^ (a & b))),
}


def permutation_unitary(perm):
    """d x d x 4 int64 array of the permutation matrix U|i> = |perm[i]> over Z[omega]: entry
    [r, c] = (c0, c1, c2, c3) for c0 + c1 w + c2 w^2 + c3 w^3; exponent 0."""
    import numpy as np
    d = len(perm)
    if sorted(perm) != list(range(d)):
        raise ValueError("not a permutation")
    v = np.zeros((d, d, 4), dtype=np.int64)
    for c, r in enumerate(perm):
        v[r, c, 0] = 1
    return v
