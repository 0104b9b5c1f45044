"""Distinguished-point storage, trail backtracking, claw checks and the search driver
(Sec. 3 for the claw search, Sec. 4.1 for the T-count problem, Appendix for budgets).

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

Plain, sequential restatement:
* Storage (Sec. 3): a dict from distinguished point to (start, length); the first
  writer stays; a second trail with a different start reaching the same point is
  a merge to trace back.
* Backtracking (Sec. 3, Fig. 2): advance the longer trail by the length
  difference; equal points mean one trail started on the other.  Otherwise step
  both in lockstep until their images coincide: the two predecessors are a
  collision of f.  Same side: useless.  Different sides and equal matrix hash: a
  claw candidate, accepted only when D = W V^T is exactly a signed permutation.
* Driver: depths in the given order; odd depths loop over the xi chunks in
  ascending order; a space with N = 2 xi^h <= enum_max points is enumerated;
  otherwise walks run with a budget of beta N / theta steps, beta = 16 (Appendix:
  order N/theta steps per golden collision when memory exceeds the space), split
  into function versions of max(version_factor * N, 2 m / theta) steps each.  A version changes
  every salt, hence f, and starts from an empty table (re-salting, as in van
  Oorschot-Wiener's golden-collision search; the paper cites it for the method).
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

from . import walk, zmat


class Table:
    def __init__(self):
        self.d: Dict[int, Tuple[int, int]] = {}

    def insert(self, dp: int, start: int, length: int):
        if dp not in self.d:
            self.d[dp] = (start, length)
            return "new", None
        s, l = self.d[dp]
        if s == start:
            return "same", None
        return "collision", (s, l)


def backtrack(spec: walk.Spec, ta: Tuple[int, int], tb: Tuple[int, int]):
    """Locate where two trails with a common distinguished point merged.

    Returns (kind, pair, steps): kind in {"robin_hood", "same_side", "reduction",
    "claw"}; pair = (u_a, u_b), the two distinct predecessors of the merge point.
    "reduction" means different sides whose matrix hashes differ (the points
    merged only through the reduction to N_half).
    """
    (pa, la), (pb, lb) = ta, tb
    steps = 0
    while la > lb:
        pa = walk.f(spec, pa)
        la -= 1
        steps += 1
    while lb > la:
        pb = walk.f(spec, pb)
        lb -= 1
        steps += 1
    if pa == pb:
        return "robin_hood", None, steps
    for _ in range(la):
        na, ha = walk.f_with_hash(spec, pa)
        nb, hb = walk.f_with_hash(spec, pb)
        steps += 2
        if na == nb:
            sa, sb = walk.unpack(pa)[1], walk.unpack(pb)[1]
            if sa == sb:
                return "same_side", (pa, pb), steps
            if ha != hb:
                return "reduction", (pa, pb), steps
            return "claw", (pa, pb), steps
        pa, pb = na, nb
    raise AssertionError("trails with a common end point must merge")


@dataclass
class Decomposition:
    """U_hat = D_hat R_hat(P_t) ... R_hat(P_1) with D P_q D^dag = sign[q] P_perm[q]."""

    t: int
    paulis_desc: List[int]        # [P_t, ..., P_1]
    perm: List[int]
    sign: List[int]


def claw_check(spec: walk.Spec, u0: int, u1: int) -> Optional[Decomposition]:
    """Exact check of a claw candidate: D = W V^T must be a signed permutation."""
    if walk.unpack(u0)[1] == 1:
        u0, u1 = u1, u0
    (xv, bv), (xw, bw) = walk.unpack(u0), walk.unpack(u1)
    if bv != 0 or bw != 1:
        return None
    V = walk.half_matrix(spec, xv, 0)
    W = walk.half_matrix(spec, xw, 1)
    D = W @ V.T()
    sp = D.signed_perm_of()
    if sp is None:
        return None
    pv = walk.decode(xv, spec.n, spec.h)
    pw = walk.decode(xw, spec.n, spec.h)
    desc = list(pv) + list(reversed(pw)) + ([spec.chunk] if spec.k % 2 else [])
    return Decomposition(t=spec.k, paulis_desc=desc, perm=sp[0], sign=sp[1])


def reconstruct(n: int, dec: Decomposition) -> zmat.ZMat:
    """D_hat R_hat(P_t) ... R_hat(P_1)."""
    m = zmat.ZMat.signed_perm(dec.perm, dec.sign)
    return zmat.product_of_rotations(dec.paulis_desc, n, start=m)


@dataclass
class SearchStats:
    steps: int = 0
    dps: int = 0
    abandoned: int = 0
    collisions: Dict[str, int] = field(default_factory=lambda: {"robin_hood": 0, "same_side": 0,
                                                                 "reduction": 0, "claw": 0})
    false_claws: int = 0
    spaces: int = 0
    versions: int = 0


def enumerate_space(spec: walk.Spec, stats: SearchStats) -> Optional[Decomposition]:
    """Every point of a small space: group side-0 points by matrix hash, probe side-1 points."""
    by_hash: Dict[int, List[int]] = {}
    for x in range(spec.n_half):
        _, hsh = walk.f_with_hash(spec, walk.pack(x, 0))
        by_hash.setdefault(hsh, []).append(x)
        stats.steps += 1
    for x in range(spec.n_half):
        _, hsh = walk.f_with_hash(spec, walk.pack(x, 1))
        stats.steps += 1
        for xv in by_hash.get(hsh, []):
            stats.collisions["claw"] += 1
            dec = claw_check(spec, walk.pack(xv, 0), walk.pack(x, 1))
            if dec is not None:
                return dec
            stats.false_claws += 1
    return None


def walk_space(spec: walk.Spec, walks: int, budget: int, cap_factor: int,
               stats: SearchStats) -> Optional[Decomposition]:
    """m walks stepped round-robin, one f per walk per round (Sec. 3)."""
    table = Table()
    cap = walk.trail_cap(spec.delta, cap_factor)
    state = []
    for w in range(walks):
        s = walk.start_point(spec, w, 0)
        state.append([0, s, s, 0])          # trail index j, start, current, length
    used = 0
    while used < budget:
        for w in range(walks):
            j, start, cur, length = state[w]
            nxt = walk.f(spec, cur)
            used += 1
            length += 1
            restart = False
            if walk.distinguished(spec, nxt):
                stats.dps += 1
                kind, other = table.insert(nxt, start, length)
                restart = True
                if kind == "collision":
                    ck, pair, vsteps = backtrack(spec, (start, length), other)
                    used += vsteps
                    stats.collisions[ck] += 1
                    if ck == "claw":
                        dec = claw_check(spec, *pair)
                        if dec is not None:
                            stats.steps += used
                            return dec
                        stats.false_claws += 1
            elif length >= cap:
                stats.abandoned += 1
                restart = True
            if restart:
                j += 1
                s = walk.start_point(spec, w, j)
                state[w] = [j, s, s, 0]
            else:
                state[w] = [j, start, nxt, length]
            if used >= budget:
                break
    stats.steps += used
    return None


@dataclass
class SearchResult:
    found: bool
    decomposition: Optional[Decomposition]
    stats: SearchStats
    seconds: float
    depths_tried: List[int]


def search(u: zmat.ZMat, n: int, k_max: int, seed: int, delta_of_k, walks: int = 64,
           cap_factor: int = 20, beta: int = 16, enum_max: int = 1 << 16,
           depth_order: Optional[List[int]] = None, version: int = 0,
           version_factor: int = 2) -> SearchResult:
    """Find e^{i phi} U = D R(P_t) ... R(P_1) at the first depth in `depth_order` that succeeds."""
    t0 = time.perf_counter()
    stats = SearchStats()
    order = list(range(k_max + 1)) if depth_order is None else list(depth_order)
    tried = []
    xi = 4 ** n - 1
    for k in order:
        tried.append(k)
        if k == 0:
            sp = u.signed_perm_of()
            if sp is not None:
                dec = Decomposition(t=0, paulis_desc=[], perm=sp[0], sign=sp[1])
                return SearchResult(True, dec, stats, time.perf_counter() - t0, tried)
            continue
        chunks = range(1, xi + 1) if k % 2 else [0]
        delta = delta_of_k(k)
        for c in chunks:
            spec = walk.make_spec(u, n, k, c, seed, delta, version)
            stats.spaces += 1
            npts = 2 * spec.n_half
            if npts <= enum_max:
                dec = enumerate_space(spec, stats)
            else:
                # function versions (re-salting): each version is a fresh random f with
                # a fresh table; a fixed f can hide the claw (in-degree-0 points,
                # distinguished-point-free cycles).
                budget = beta * npts * (1 << delta)
                # at least two mean trail lengths per walk, so trails complete in every version
                per_version = max(version_factor * npts, 2 * walks * (1 << delta))
                dec, v, used = None, version, 0
                while dec is None and used < budget:
                    spec = walk.make_spec(u, n, k, c, seed, delta, v)
                    before = stats.steps
                    dec = walk_space(spec, walks, min(per_version, budget - used), cap_factor, stats)
                    used += stats.steps - before
                    stats.versions += 1
                    v += 1
            if dec is not None:
                return SearchResult(True, dec, stats, time.perf_counter() - t0, tried)
    return SearchResult(False, None, stats, time.perf_counter() - t0, tried)
