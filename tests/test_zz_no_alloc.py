"""The walk step that allocates nothing (tcw_step_noalloc) against tcw_step, through the C ABI: the
same points and matrix hashes bit for bit, on two calls in a row (the second with a smaller input:
fewer points and a smaller space), and no device memory taken by the calls."""

import ctypes

import pytest

import seeded_inputs
from oracle import walk as owalk
from oracle import zmat

pytestmark = pytest.mark.gpu
MASK = (1 << 64) - 1


def _free_device_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _dev(vals):
    import torch
    return torch.tensor([v if v < (1 << 63) else v - (1 << 64) for v in vals], dtype=torch.int64, device="cuda:0")


def test_step_noalloc_matches_step():
    import torch
    from paper_1606_07413_amd import tcw
    assert torch.cuda.is_available()
    ctx = tcw.Context(0)
    cases = [(4, 7, 1, 1000), (3, 5, 2, 77)]
    runs = []
    for n, k, seed, count in cases:
        print("no-alloc step", n, k, seed, count, flush=True)
        tw = seeded_inputs.target_words(n, k, seed)
        tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
        chunk = tw.paulis[0] if k % 2 else 0
        n_half = (4 ** n - 1) ** (k // 2)
        pts = seeded_inputs.random_points(n_half, count, 40 + seed)
        pts[:2] = [n_half - 1, (n_half - 1) | (1 << 32)]
        din = _dev(pts)
        want_o, want_h = torch.empty_like(din), torch.empty_like(din)
        ctx.step(tgt, k, chunk, 900 + seed, 6, din, want_o, want_h, version=3)
        runs.append((n, k, seed, chunk, tgt, tw, pts, din, want_o, want_h))
    outs = [(torch.full_like(r[7], -1), torch.full_like(r[7], -1)) for r in runs]
    torch.cuda.synchronize()
    free_before = _free_device_bytes()
    for (n, k, seed, chunk, tgt, tw, pts, din, want_o, want_h), (got_o, got_h) in zip(runs, outs):
        ctx.step_noalloc(tgt, k, chunk, 900 + seed, 6, din, got_o, got_h, version=3)
    free_after = _free_device_bytes()
    for (n, k, seed, chunk, tgt, tw, pts, din, want_o, want_h), (got_o, got_h) in zip(runs, outs):
        assert torch.equal(got_o, want_o) and torch.equal(got_h, want_h), (n, k)
    # the calls took no device memory (the tensors above were allocated before the first reading)
    assert free_after == free_before
    # and the first points against the oracle
    n, k, seed, chunk, tgt, tw, pts, din, want_o, want_h = runs[1]
    spec = owalk.make_spec(zmat.target_from_words(n, tw.paulis, tw.clifford), n, k, chunk, 900 + seed, delta=6,
                           version=3)
    got = [int(v) & MASK for v in want_o.cpu().tolist()[:8]]
    assert got == [owalk.f(spec, p) for p in pts[:8]]
