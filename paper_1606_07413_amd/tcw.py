"""ctypes binding of libtcw.so (include/tcw.h): argument marshalling only.

Device arrays are torch CUDA tensors (their data_ptr is passed through); streams are
torch streams.  Every computation runs in the HIP library; when the library is not
built this module raises instead of computing anything itself.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcw.so")

TCW_OK = 0
TCW_EINVAL = -1
TCW_EOVERFLOW = -4
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "ESTATE"}
MAX_T = 64
MAX_R = 256
ORDER_PLAIN = 0
ORDER_GIVEN = 1
ORDER_GIVEN_FIRST = 2
STATUS_NOT_FOUND = 0
STATUS_FOUND = 1
STATUS_STOPPED = 2
MAX_TRAIL_CAP = (1 << 30) - 1


class TcwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tcw {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Space(C.Structure):
    _fields_ = [("k", C.c_int32), ("chunk", C.c_int32), ("seed", C.c_uint64), ("version", C.c_uint32),
                ("delta", C.c_int32)]


class WalkStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("steps", "dps", "inserts", "abandoned", "robin_hood", "same_side",
                                          "reduction", "claws", "table_full", "spin_timeouts", "active_walks",
                                          "claws_dropped")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class WalkParams(C.Structure):
    _fields_ = [
        ("k_max", C.c_int32), ("delta", C.c_int32), ("walks", C.c_int64), ("log2_table", C.c_int32),
        ("seed", C.c_uint64), ("version", C.c_uint32), ("trail_cap_factor", C.c_int32),
        ("budget_beta", C.c_int32), ("version_factor", C.c_int32), ("enum_max", C.c_int64),
        ("iters_per_launch", C.c_int32), ("depth_order_kind", C.c_int32), ("depth_order_len", C.c_int32),
        ("depth_order", C.c_int32 * 16), ("chunk_first", C.c_int32), ("chunk_last", C.c_int32),
        ("max_seconds", C.c_double), ("chunk_parallel", C.c_int32), ("launch_limit", C.c_int64),
    ]


class Gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32)]


GATE_NAMES = {1: "h", 2: "s", 3: "sdg", 4: "cx", 5: "t", 6: "tdg", 7: "x", 8: "y", 9: "z"}


class Result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("t", C.c_int32), ("n", C.c_int32), ("chunk", C.c_int32),
        ("paulis", C.c_uint16 * MAX_T), ("clifford_perm", C.c_int32 * MAX_R), ("clifford_sign", C.c_int8 * MAX_R),
        ("stats", WalkStats), ("spaces", C.c_int64), ("versions", C.c_int64), ("launches", C.c_int64),
        ("false_claws", C.c_int64), ("seconds", C.c_double), ("failed_depths", C.c_uint64),
        ("minimal", C.c_int32), ("reserved", C.c_int32),
    ]


_P = C.c_void_p
_SIGS = {
    "tcw_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "tcw_destroy": (C.c_int, [_P]),
    "tcw_last_error": (C.c_char_p, [_P]),
    "tcw_set_stream": (C.c_int, [_P, _P]),
    "tcw_target_from_words": (C.c_int, [_P, C.c_int, C.POINTER(C.c_uint16), C.c_int, C.POINTER(C.c_uint16),
                                        C.c_int, C.POINTER(_P)]),
    "tcw_target_from_channel": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                          C.POINTER(_P)]),
    "tcw_target_from_unitary": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int64), C.c_int32, C.POINTER(_P)]),
    "tcw_target_random": (C.c_int, [_P, C.c_int, C.c_int, C.c_uint64, C.POINTER(_P), C.POINTER(C.c_uint16),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int8)]),
    "tcw_target_free": (C.c_int, [_P]),
    "tcw_target_channel": (C.c_int, [_P, _P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "tcw_target_n": (C.c_int, [_P]),
    "tcw_step": (C.c_int, [_P, _P, C.POINTER(Space), _P, _P, _P, C.c_int64]),
    "tcw_step_noalloc": (C.c_int, [_P, _P, C.POINTER(Space), _P, _P, _P, C.c_int64]),
    "tcw_trails": (C.c_int, [_P, _P, C.POINTER(Space), _P, C.c_int64, C.c_uint32, _P, _P]),
    "tcw_start_points": (C.c_int, [_P, _P, C.POINTER(Space), C.c_int64, C.c_uint32, C.c_int64, _P]),
    "tcw_canon_hash": (C.c_int, [_P, C.c_int, C.POINTER(Space), _P, _P, _P, C.c_int64, _P]),
    "tcw_claw_check": (C.c_int, [_P, _P, C.POINTER(Space), _P, _P, C.c_int64, _P, _P, _P]),
    "tcw_walk_begin": (C.c_int, [_P, _P, C.POINTER(Space), C.c_int64, C.c_int, C.c_uint32, C.c_int,
                                 C.POINTER(_P)]),
    "tcw_walk_run": (C.c_int, [_P, C.c_int]),
    "tcw_walk_stats_get": (C.c_int, [_P, C.POINTER(WalkStats)]),
    "tcw_walk_claws": (C.c_int, [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_int64,
                                 C.POINTER(C.c_int64)]),
    "tcw_walk_reset": (C.c_int, [_P, C.c_uint32]),
    "tcw_walk_last_ms": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "tcw_walk_read_states": (C.c_int, [_P, C.c_int64, C.c_int64, _P]),
    "tcw_walk_write_states": (C.c_int, [_P, C.c_int64, C.c_int64, _P]),
    "tcw_walk_read_table": (C.c_int, [_P, _P]),
    "tcw_walk_write_table": (C.c_int, [_P, _P]),
    "tcw_walk_end": (C.c_int, [_P]),
    "tcw_default_params": (None, [C.POINTER(WalkParams), C.c_int]),
    "tcw_search": (C.c_int, [_P, _P, C.POINTER(WalkParams), C.POINTER(Result)]),
    "tcw_search_stop": (C.c_int, [_P]),
    "tcw_checkpoint": (C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
    "tcw_resume": (C.c_int, [_P, _P, _P, C.c_size_t, C.c_int64, C.POINTER(Result)]),
    "tcw_search_batch": (C.c_int, [_P, C.POINTER(_P), C.c_int, C.POINTER(WalkParams), C.POINTER(Result),
                                   C.POINTER(C.c_double)]),
    "tcw_autotune": (C.c_int, [_P, _P, C.c_int, C.c_int, C.c_int, C.c_uint64, C.POINTER(C.c_int64),
                               C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "tcw_features": (C.c_int, [_P, _P, _P]),
    "tcw_label_batch": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_uint16), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.c_int, C.c_uint64, _P, _P]),
    "tcw_circuit": (C.c_int, [C.POINTER(Result), C.POINTER(Gate), C.c_int32, C.POINTER(C.c_int32)]),
    "tcw_min_tcount": (C.c_int, [_P, _P, C.c_int, C.c_uint64, C.POINTER(C.c_int32)]),
    "tcw_mlp_create": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, _P, C.c_uint64, C.POINTER(_P)]),
    "tcw_mlp_free": (C.c_int, [_P]),
    "tcw_mlp_param_count": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "tcw_mlp_get_params": (C.c_int, [_P, _P]),
    "tcw_mlp_set_params": (C.c_int, [_P, _P]),
    "tcw_mlp_forward": (C.c_int, [_P, _P, C.c_int, _P]),
    "tcw_mlp_gradients": (C.c_int, [_P, _P, _P, C.c_int, _P, C.POINTER(C.c_float)]),
    "tcw_mlp_train_step": (C.c_int, [_P, _P, _P, C.c_int, C.c_float, C.POINTER(C.c_float)]),
    "tcw_mlp_depth_order": (C.c_int, [_P, _P, C.c_int, C.POINTER(WalkParams), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_float)]),
    "tcw_depth_costs": (C.c_int, [_P, _P, C.POINTER(WalkParams), C.c_int, C.POINTER(C.c_double)]),
    "tcw_mlp_train": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int, C.c_int, C.c_float, C.POINTER(C.c_float)]),
}

EXPORTED = sorted(_SIGS)
_lib = None


def load(path: str = LIB_PATH):
    """Load libtcw.so with typed entry points; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError("device arrays must be contiguous CUDA tensors")
    return t.data_ptr()


def _dev(t, esize: int, need: int, what: str, device: int) -> Optional[int]:
    """Device pointer of a contiguous CUDA tensor on `device` whose elements are esize bytes wide and
    which holds at least `need` of them: the library writes `need` elements through the pointer."""
    if t is None:
        return None
    p = _ptr(t)
    if t.device.index != device:
        raise ValueError(f"{what}: tensor on cuda:{t.device.index}, context on cuda:{device}")
    if t.element_size() != esize:
        raise TypeError(f"{what}: elements of {esize} bytes expected, got {t.dtype}")
    if t.numel() < need:
        raise ValueError(f"{what}: at least {need} elements expected, got {t.numel()}")
    return p


def _u16_array(vals: Sequence[int]):
    arr = (C.c_uint16 * max(1, len(vals)))(*vals)
    return arr


@dataclass
class Decomposition:
    t: int
    paulis_desc: List[int]   # P_t .. P_1
    perm: List[int]
    sign: List[int]
    chunk: int


class Context:
    """One library context bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.device = device
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = _P()
        self._check(self.lib.tcw_create(C.byref(h), device, _P(stream.cuda_stream)), None)
        self.h = h

    def _check(self, rc: int, h=None):
        if rc != TCW_OK:
            msg = self.lib.tcw_last_error(h if h is not None else getattr(self, "h", None))
            raise TcwError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.tcw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- targets ----
    def target_from_words(self, n: int, paulis: Sequence[int], clifford: Sequence[int]) -> "Target":
        out = _P()
        self._check(self.lib.tcw_target_from_words(self.h, n, _u16_array(paulis), len(paulis), _u16_array(clifford),
                                                   len(clifford), C.byref(out)))
        return Target(self, out, n)

    def target_from_channel(self, n: int, a, b, e: int) -> "Target":
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.int32)
        b = np.ascontiguousarray(b, dtype=np.int32)
        out = _P()
        self._check(self.lib.tcw_target_from_channel(self.h, n, a.ctypes.data_as(C.POINTER(C.c_int32)),
                                                     b.ctypes.data_as(C.POINTER(C.c_int32)), int(e), C.byref(out)))
        return Target(self, out, n)

    def target_from_unitary(self, n: int, v, e: int) -> "Target":
        """U = V / sqrt2^e, V a 2^n x 2^n x 4 integer array (coefficients of w^0..w^3, w = e^{i pi/4})."""
        import numpy as np
        v = np.ascontiguousarray(v, dtype=np.int64)
        if v.shape != (2 ** n, 2 ** n, 4):
            raise ValueError("V must have shape (2^n, 2^n, 4)")
        out = _P()
        self._check(self.lib.tcw_target_from_unitary(self.h, n, v.ctypes.data_as(C.POINTER(C.c_int64)), int(e),
                                                     C.byref(out)))
        return Target(self, out, n)

    def target_random(self, n: int, k: int, seed: int):
        """Seeded synthetic target; returns (Target, [P_1..P_k], perm, sign) with D P_q D^dag = sign[q] P_perm[q]."""
        r = 4 ** n
        out = _P()
        ps = (C.c_uint16 * max(1, k))()
        perm = (C.c_int32 * r)()
        sign = (C.c_int8 * r)()
        self._check(self.lib.tcw_target_random(self.h, n, k, seed, C.byref(out), ps, perm, sign))
        return Target(self, out, n), list(ps[:k]), list(perm), list(sign)

    def min_tcount(self, target, h_max: int, seed: int = 1) -> int:
        """Minimal T-count by meet in the middle when it is at most 2 h_max, else -1."""
        out = C.c_int32(0)
        self._check(self.lib.tcw_min_tcount(self.h, target.h, h_max, seed, C.byref(out)))
        return out.value

    # ---- parity entry points ----
    def step(self, target, k, chunk, seed, delta, pts_in, pts_out, hash_out=None, version=0):
        sp = Space(k, chunk, seed, version, delta)
        count, d = pts_in.numel(), self.device
        self._check(self.lib.tcw_step(self.h, target.h, C.byref(sp), _dev(pts_in, 8, count, "pts_in", d),
                                      _dev(pts_out, 8, count, "pts_out", d), _dev(hash_out, 8, count, "hash_out", d),
                                      count))

    def step_noalloc(self, target, k, chunk, seed, delta, pts_in, pts_out, hash_out=None, version=0):
        """tcw_step computed with the library's fixed scratch array (no device allocation)."""
        sp = Space(k, chunk, seed, version, delta)
        count, d = pts_in.numel(), self.device
        self._check(self.lib.tcw_step_noalloc(self.h, target.h, C.byref(sp), _dev(pts_in, 8, count, "pts_in", d),
                                              _dev(pts_out, 8, count, "pts_out", d),
                                              _dev(hash_out, 8, count, "hash_out", d), count))

    def trails(self, target, k, chunk, seed, delta, starts, cap, dp_out, len_out, version=0):
        sp = Space(k, chunk, seed, version, delta)
        count, d = starts.numel(), self.device
        self._check(self.lib.tcw_trails(self.h, target.h, C.byref(sp), _dev(starts, 8, count, "starts", d), count,
                                        cap, _dev(dp_out, 8, count, "dp_out", d), _dev(len_out, 4, count, "len_out", d)))

    def start_points(self, target, k, chunk, seed, w0, j, count, out, version=0):
        sp = Space(k, chunk, seed, version, 0)
        self._check(self.lib.tcw_start_points(self.h, target.h, C.byref(sp), w0, j, count,
                                              _dev(out, 8, count, "out", self.device)))

    def canon_hash(self, n, k, chunk, seed, a, b, e, out, version=0):
        sp = Space(k, chunk, seed, version, 0)
        count, rr, d = e.numel(), 16 ** n, self.device
        self._check(self.lib.tcw_canon_hash(self.h, n, C.byref(sp), _dev(a, 4, count * rr, "a", d),
                                            _dev(b, 4, count * rr, "b", d), _dev(e, 4, count, "e", d), count,
                                            _dev(out, 8, count, "out", d)))

    def claw_check(self, target, k, chunk, seed, u0, u1, ok, perm, sign, version=0):
        sp = Space(k, chunk, seed, version, 0)
        count, r, d = u0.numel(), 4 ** target.n, self.device
        self._check(self.lib.tcw_claw_check(self.h, target.h, C.byref(sp), _dev(u0, 8, count, "u0", d),
                                            _dev(u1, 8, count, "u1", d), count, _dev(ok, 4, count, "ok", d),
                                            _dev(perm, 4, count * r, "perm", d), _dev(sign, 1, count * r, "sign", d)))

    # ---- walks and search ----
    def walk(self, target, k, chunk, seed, delta, walks, log2_table, cap, enumerate=False, version=0) -> "Walk":
        sp = Space(k, chunk, seed, version, delta)
        out = _P()
        self._check(self.lib.tcw_walk_begin(self.h, target.h, C.byref(sp), walks, log2_table, cap,
                                            1 if enumerate else 0, C.byref(out)))
        return Walk(self, out)

    def default_params(self, n: int) -> WalkParams:
        p = WalkParams()
        self.lib.tcw_default_params(C.byref(p), n)
        return p

    def depth_costs(self, target, params: WalkParams, k_max: int):
        """Walk steps the driver spends on each depth 0..k_max under params when it holds no
        decomposition (tcw_depth_costs)."""
        out = (C.c_double * (k_max + 1))()
        self._check(self.lib.tcw_depth_costs(self.h, target.h, C.byref(params), k_max, out))
        return list(out)

    def search(self, target, params: WalkParams) -> Result:
        res = Result()
        self._check(self.lib.tcw_search(self.h, target.h, C.byref(params), C.byref(res)))
        return res

    def search_stop(self):
        self._check(self.lib.tcw_search_stop(self.h))

    def checkpoint(self) -> bytes:
        """The stopped search of this context, serialised (host bytes)."""
        n = C.c_size_t(0)
        self._check(self.lib.tcw_checkpoint(self.h, None, C.byref(n)))
        buf = (C.c_uint8 * max(1, n.value))()
        self._check(self.lib.tcw_checkpoint(self.h, buf, C.byref(n)))
        return bytes(buf[:n.value])

    def resume(self, target, blob: bytes, launch_limit: int = 0) -> Result:
        res = Result()
        buf = (C.c_uint8 * max(1, len(blob))).from_buffer_copy(blob if blob else b"\0")
        self._check(self.lib.tcw_resume(self.h, target.h, buf, len(blob), launch_limit, C.byref(res)))
        return res


def _search_batch(self, targets, params):
    """Search many targets together; returns (results, aggregate walk steps/s)."""
    n = len(targets)
    th = (_P * n)(*[t.h for t in targets])
    ps = (WalkParams * n)(*params)
    rs = (Result * n)()
    agg = C.c_double(0)
    self._check(self.lib.tcw_search_batch(self.h, th, n, ps, rs, C.byref(agg)))
    return list(rs), agg.value


def _autotune(self, target, k, chunk, delta, seed):
    w, it, lg, rate = C.c_int64(0), C.c_int(0), C.c_int(0), C.c_double(0)
    self._check(self.lib.tcw_autotune(self.h, target.h, k, chunk, delta, seed, C.byref(w), C.byref(it),
                                      C.byref(lg), C.byref(rate)))
    return {"walks": w.value, "iters": it.value, "log2_table": lg.value, "steps_per_s": rate.value}


Context.search_batch = _search_batch
Context.autotune = _autotune


def circuit_of(res: Result):
    """The decomposition in `res` as gates in application order: [(name, qubits), ...]."""
    lib = load()
    count = C.c_int32(0)
    rc = lib.tcw_circuit(C.byref(res), None, 0, C.byref(count))
    if rc != TCW_OK:
        raise TcwError(rc, "result is not a verified decomposition")
    buf = (Gate * max(1, count.value))()
    rc = lib.tcw_circuit(C.byref(res), buf, count.value, C.byref(count))
    if rc != TCW_OK:
        raise TcwError(rc, "circuit synthesis failed")
    out = []
    for g in buf[:count.value]:
        out.append((GATE_NAMES[g.kind], (g.q0, g.q1) if g.kind == 4 else (g.q0,)))
    return out


def decomposition_of(res: Result) -> Optional[Decomposition]:
    if res.status != 1:
        return None
    r = 4 ** res.n
    return Decomposition(t=res.t, paulis_desc=list(res.paulis[:res.t]), perm=list(res.clifford_perm[:r]),
                         sign=list(res.clifford_sign[:r]), chunk=res.chunk)


class Target:
    def __init__(self, ctx: Context, h, n: int):
        self.ctx, self.h, self.n = ctx, h, n

    def channel(self):
        import numpy as np
        r = 4 ** self.n
        a = np.zeros((r, r), dtype=np.int32)
        b = np.zeros((r, r), dtype=np.int32)
        e = C.c_int32(0)
        self.ctx._check(self.ctx.lib.tcw_target_channel(self.ctx.h, self.h, a.ctypes.data_as(C.POINTER(C.c_int32)),
                                                        b.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(e)))
        return a, b, e.value

    def free(self):
        if self.h:
            self.ctx.lib.tcw_target_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Walk:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def run(self, iters: int):
        self.ctx._check(self.ctx.lib.tcw_walk_run(self.h, iters))

    def stats(self) -> WalkStats:
        st = WalkStats()
        self.ctx._check(self.ctx.lib.tcw_walk_stats_get(self.h, C.byref(st)))
        return st

    def claws(self, max_pairs: int = 4096):
        u0 = (C.c_uint64 * max(1, max_pairs))()
        u1 = (C.c_uint64 * max(1, max_pairs))()
        total = C.c_int64(0)
        self.ctx._check(self.ctx.lib.tcw_walk_claws(self.h, u0, u1, max_pairs, C.byref(total)))
        m = min(total.value, max_pairs, 4096)
        return [(u0[i], u1[i]) for i in range(m)], total.value

    STATE_DTYPE = [("start", "<u8"), ("cur", "<u8"), ("pa", "<u8"), ("pb", "<u8"), ("na", "<u8"), ("ha", "<u8"),
                   ("len", "<u4"), ("trail", "<u4"), ("mode", "<u4"), ("rem", "<u4")]

    def read_states(self, first: int, count: int):
        import numpy as np
        out = np.zeros(count, dtype=self.STATE_DTYPE)
        self.ctx._check(self.ctx.lib.tcw_walk_read_states(self.h, first, count, out.ctypes.data))
        return out

    def write_states(self, first: int, states):
        import numpy as np
        states = np.ascontiguousarray(states, dtype=self.STATE_DTYPE)
        self.ctx._check(self.ctx.lib.tcw_walk_write_states(self.h, first, len(states), states.ctypes.data))

    def read_table(self, log2_table: int):
        import numpy as np
        out = np.zeros((1 << log2_table, 2), dtype=np.uint64)
        self.ctx._check(self.ctx.lib.tcw_walk_read_table(self.h, out.ctypes.data))
        return out

    def write_table(self, table):
        import numpy as np
        table = np.ascontiguousarray(table, dtype=np.uint64)
        self.ctx._check(self.ctx.lib.tcw_walk_write_table(self.h, table.ctypes.data))

    def reset(self, version: int):
        self.ctx._check(self.ctx.lib.tcw_walk_reset(self.h, version))

    def last_ms(self) -> float:
        ms = C.c_float(0)
        self.ctx._check(self.ctx.lib.tcw_walk_last_ms(self.h, C.byref(ms)))
        return ms.value

    def end(self):
        if self.h:
            self.ctx.lib.tcw_walk_end(self.h)
            self.h = None

    def __del__(self):
        try:
            self.end()
        except Exception:
            pass


def _features(self, target, out):
    self._check(self.lib.tcw_features(self.h, target.h, _dev(out, 4, 16 ** target.n, "out", self.device)))


def _label_batch(self, n, words_list, h_max, seed, features_out, labels_out):
    """words_list: [(paulis, clifford), ...]; fills device tensors features_out, labels_out."""
    import numpy as np
    flat, offs, ks = [], [0], []
    for paulis, clifford in words_list:
        flat.extend(paulis)
        flat.extend(clifford)
        offs.append(len(flat))
        ks.append(len(paulis))
    self.label_words(n, np.asarray(flat, dtype=np.uint16), np.asarray(offs, dtype=np.int32),
                     np.asarray(ks, dtype=np.int32), h_max, seed, features_out, labels_out)


def _label_words(self, n, words, offsets, kof, h_max, seed, features_out, labels_out):
    """tcw_label_batch on flat host arrays: words (uint16), offsets (int32, count + 1), kof (int32)."""
    import numpy as np
    words = np.ascontiguousarray(words, dtype=np.uint16)
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    kof = np.ascontiguousarray(kof, dtype=np.int32)
    count = len(kof)
    if len(offsets) != count + 1 or count < 1 or int(offsets[-1]) > len(words):
        raise ValueError("offsets must hold count + 1 entries within words")
    if len(words) == 0:
        words = np.zeros(1, dtype=np.uint16)
    d = self.device
    self._check(self.lib.tcw_label_batch(self.h, n, count, words.ctypes.data_as(C.POINTER(C.c_uint16)),
                                         offsets.ctypes.data_as(C.POINTER(C.c_int32)),
                                         kof.ctypes.data_as(C.POINTER(C.c_int32)), h_max, seed,
                                         _dev(features_out, 4, count * 16 ** n, "features_out", d),
                                         _dev(labels_out, 4, count, "labels_out", d)))


Context.features = _features
Context.label_batch = _label_batch
Context.label_words = _label_words


class Network:
    """The depth-order network (parameters W_0, b_0, W_1, b_1, ... as one float32 vector)."""

    def __init__(self, ctx: Context, inp: int, hidden: int, depth: int, classes: int, init=None, seed: int = 42):
        import numpy as np
        self.ctx = ctx
        self.dims = (inp, hidden, depth, classes)
        h = _P()
        buf = None
        if init is not None:
            buf = np.ascontiguousarray(init, dtype=np.float32)
        ctx._check(ctx.lib.tcw_mlp_create(ctx.h, inp, hidden, depth, classes,
                                          None if buf is None else buf.ctypes.data, seed, C.byref(h)))
        self.h = h
        cnt = C.c_int64(0)
        ctx._check(ctx.lib.tcw_mlp_param_count(self.h, C.byref(cnt)))
        self.count = cnt.value

    def params(self):
        import numpy as np
        out = np.zeros(self.count, dtype=np.float32)
        self.ctx._check(self.ctx.lib.tcw_mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, flat):
        import numpy as np
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self.ctx._check(self.ctx.lib.tcw_mlp_set_params(self.h, flat.ctypes.data))

    def _x(self, x):
        # rows of `inp` float32 features
        return _dev(x, 4, x.shape[0] * self.dims[0], "x", self.ctx.device)

    def _labels(self, labels, b):
        return _dev(labels, 4, b, "labels", self.ctx.device)

    def forward(self, x, probs_out):
        b = x.shape[0]
        self.ctx._check(self.ctx.lib.tcw_mlp_forward(self.h, self._x(x), b,
                                                     _dev(probs_out, 4, b * self.dims[3], "probs_out",
                                                          self.ctx.device)))

    def gradients(self, x, labels):
        import numpy as np
        g = np.zeros(self.count, dtype=np.float32)
        loss = C.c_float(0)
        b = x.shape[0]
        self.ctx._check(self.ctx.lib.tcw_mlp_gradients(self.h, self._x(x), self._labels(labels, b), b,
                                                       g.ctypes.data, C.byref(loss)))
        return g, loss.value

    def train_step(self, x, labels, lr):
        loss = C.c_float(0)
        b = x.shape[0]
        self.ctx._check(self.ctx.lib.tcw_mlp_train_step(self.h, self._x(x), self._labels(labels, b), b, lr,
                                                        C.byref(loss)))
        return loss.value

    def train(self, x, labels, batch, epochs, lr):
        loss = C.c_float(0)
        b = x.shape[0]
        self.ctx._check(self.ctx.lib.tcw_mlp_train(self.h, self._x(x), self._labels(labels, b), b, batch, epochs,
                                                   lr, C.byref(loss)))
        return loss.value

    def depth_order(self, target, k_max, params=None):
        """Depths 0..k_max by descending predicted probability, or with search parameters by
        descending probability per step of each depth's cost (tcw_depth_costs)."""
        order = (C.c_int32 * (k_max + 1))()
        probs = (C.c_float * self.dims[3])()
        self.ctx._check(self.ctx.lib.tcw_mlp_depth_order(self.h, target.h, k_max,
                                                         C.byref(params) if params is not None else None,
                                                         order, probs))
        return list(order), list(probs)

    def free(self):
        if getattr(self, "h", None):
            self.ctx.lib.tcw_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def flatten_params(params: dict, depth: int):
    """W_0, b_0, W_1, b_1, ... concatenated (the library's parameter order)."""
    import numpy as np
    parts = []
    for l in range(depth + 1):
        parts.append(np.asarray(params[f"W{l}"], dtype=np.float32).reshape(-1))
        parts.append(np.asarray(params[f"b{l}"], dtype=np.float32).reshape(-1))
    return np.concatenate(parts)
