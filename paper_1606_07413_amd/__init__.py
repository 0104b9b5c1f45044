"""Deterministic-walk optimal T-count synthesis on MI355X (gfx950).

The library (libtcw.so, C ABI in include/tcw.h) runs the walk step, trails,
distinguished-point table, backtracking, claw checks and the search driver;
`tcw` is its ctypes binding.
"""

from . import tcw  # noqa: F401
