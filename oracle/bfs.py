"""Brute-force minimal T-count by breadth-first search over left-Clifford cosets
(the brute-force synthesis of Sec. 3, run at tiny n).

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

Level t holds the cosets {D M} whose minimal T-count is exactly t.  Right
multiplication by R_hat(p) is well defined on left cosets, so level t is the set
of new cosets among M R_hat(p) for M in level t-1 and p = 1..xi.  Cosets are
compared through the exact canonical form (zmat.canonical_form).
"""

from __future__ import annotations

from typing import Dict, List, Tuple

from . import zmat


def cosets_by_tcount(n: int, t_max: int) -> Tuple[List[int], Dict[tuple, int], List[List[zmat.ZMat]]]:
    xi = 4 ** n - 1
    ident = zmat.ZMat.identity(n)
    seen: Dict[tuple, int] = {zmat.canonical_form(ident): 0}
    levels = [[ident]]
    for t in range(1, t_max + 1):
        new = []
        for m in levels[-1]:
            for p in range(1, xi + 1):
                m2 = m.right_rot(p, n).reduce()
                key = zmat.canonical_form(m2)
                if key not in seen:
                    seen[key] = t
                    new.append(m2)
        levels.append(new)
    return [len(l) for l in levels], seen, levels


def min_tcount(u: zmat.ZMat, seen: Dict[tuple, int]):
    """Minimal T-count of U if its coset is within the explored levels, else None."""
    return seen.get(zmat.canonical_form(u))
