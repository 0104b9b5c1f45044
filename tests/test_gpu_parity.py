"""GPU parity of the HIP path (through the C ABI) against the CPU oracle, element by element.

Integer work throughout, so the bar is bit-exactness: targets, step outputs, matrix
hashes, trail end points and lengths, start points, claw checks and decompositions.
"""

import numpy as np
import pytest

import seeded_inputs
from oracle import bfs
from oracle import search as osearch
from oracle import walk as owalk
from oracle import zmat

pytestmark = pytest.mark.gpu
MASK = (1 << 64) - 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_07413_amd import tcw
    assert torch.cuda.is_available()
    return tcw.Context(0)


def dev(vals, dtype=None):
    import torch
    return torch.tensor([v if v < (1 << 63) else v - (1 << 64) for v in vals], dtype=dtype or torch.int64,
                        device="cuda:0")


def host_u64(t):
    return [int(v) & MASK for v in t.cpu().tolist()]


def oracle_target(n, k, seed):
    tw = seeded_inputs.target_words(n, k, seed)
    return tw, zmat.target_from_words(n, tw.paulis, tw.clifford)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n,k,seed", [(1, 5, 1), (2, 4, 2), (2, 7, 3), (3, 6, 4), (4, 7, 1), (4, 3, 2)])
def test_target_build_matches_oracle(ctx, n, k, seed):
    say("target build", n, k, seed)
    tw, u = oracle_target(n, k, seed)
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    a, b, e = tgt.channel()
    assert e == u.e
    assert np.array_equal(a, np.array(u.A, dtype=np.int64)) and np.array_equal(b, np.array(u.B, dtype=np.int64))


def test_target_from_channel_validates(ctx):
    from paper_1606_07413_amd import tcw
    say("target from channel")
    tw, u = oracle_target(2, 5, 9)
    raised = u.raise_to(u.e + 2)
    tgt = ctx.target_from_channel(2, np.array(raised.A, dtype=np.int32), np.array(raised.B, dtype=np.int32),
                                  raised.e)
    a, b, e = tgt.channel()
    assert e == u.e and np.array_equal(a, np.array(u.A, dtype=np.int64))
    bad = np.array(u.A, dtype=np.int32)
    bad[3, 4] += 1
    with pytest.raises(tcw.TcwError):
        ctx.target_from_channel(2, bad, np.array(u.B, dtype=np.int32), u.e)



def test_binding_checks_device_arrays(ctx):
    """The binding refuses output arrays that are too short or of the wrong element width before
    anything is launched (the library writes `count` elements through the pointer it gets)."""
    import torch
    say("binding argument checks")
    tw, u = oracle_target(2, 4, 1)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    din = dev([owalk.pack(0, 0), owalk.pack(1, 1), owalk.pack(2, 0)])
    with pytest.raises(ValueError):
        ctx.step(tgt, 4, 0, 1, 4, din, torch.empty(2, dtype=torch.int64, device="cuda:0"))
    with pytest.raises(TypeError):
        ctx.step(tgt, 4, 0, 1, 4, din, torch.empty(3, dtype=torch.int32, device="cuda:0"))
    with pytest.raises(ValueError):
        ctx.trails(tgt, 4, 0, 1, 4, din, 64, torch.empty_like(din), torch.empty(2, dtype=torch.int32, device="cuda:0"))
    with pytest.raises(TypeError):
        ctx.step(tgt, 4, 0, 1, 4, din, torch.empty_like(din)[::1].cpu())
    # a correct call still works afterwards
    out = torch.empty_like(din)
    ctx.step(tgt, 4, 0, 1, 4, din, out)
    spec = owalk.make_spec(u, 2, 4, 0, 1, delta=4)
    assert host_u64(out) == [owalk.f(spec, p) for p in host_u64(din)]


def test_empty_inputs_are_no_ops(ctx):
    """count = 0: every per-point call returns without error and writes nothing (an empty torch
    tensor may have a null data pointer); the space is still validated."""
    import torch
    from paper_1606_07413_amd import tcw
    say("empty inputs")
    for n, k in ((2, 4), (3, 5), (4, 7)):
        tw, u = oracle_target(n, k, 1)
        tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
        chunk = 0 if k % 2 == 0 else 1
        e64 = torch.empty(0, dtype=torch.int64, device="cuda:0")
        e32 = torch.empty(0, dtype=torch.int32, device="cuda:0")
        e8 = torch.empty(0, dtype=torch.int8, device="cuda:0")
        ctx.step(tgt, k, chunk, 1, 4, e64, e64, e64)
        ctx.trails(tgt, k, chunk, 1, 4, e64, 64, e64, e32)
        ctx.start_points(tgt, k, chunk, 1, 0, 0, 0, e64)
        ctx.canon_hash(n, k, chunk, 1, e32, e32, e32, e64)
        ctx.claw_check(tgt, k, chunk, 1, e64, e64, e32, e32, e8)
        # an invalid space is still refused (odd k needs a chunk in 1..xi)
        with pytest.raises(tcw.TcwError):
            ctx.step(tgt, 5, 0, 1, 4, e64, e64)

STEP_CASES = [(1, 4, 1, 37), (1, 5, 2, 100), (2, 2, 5, 30), (2, 4, 1, 300), (2, 5, 3, 129), (2, 6, 4, 65),
              (3, 3, 5, 64), (3, 5, 2, 77), (3, 6, 1, 200), (4, 1, 4, 16), (4, 2, 1, 33), (4, 3, 2, 20),
              (4, 4, 3, 8), (4, 5, 6, 24), (4, 6, 5, 40), (4, 7, 1, 64)]
# n = 4 covers every start of the rotated-key tables: k = 1 (no rotation: the keys), k = 2, 3 (one
# rotation from the one-rotation table), k = 4, 5 (two from the two-rotation table), k = 6, 7 (two
# from the table, one computed)


@pytest.mark.parametrize("n,k,seed,count", STEP_CASES)
def test_step_parity(ctx, n, k, seed, count):
    import torch
    say("step", n, k, seed, count)
    tw, u = oracle_target(n, k, seed)
    chunk = 0 if k % 2 == 0 else 1 + (seed * 37) % (4 ** n - 1)
    sseed = 1000 + seed
    spec = owalk.make_spec(u, n, k, chunk, sseed, delta=4)
    pts = seeded_inputs.random_points(spec.n_half, count, seed * 7)
    pts[:4] = [owalk.pack(0, 0), owalk.pack(0, 1), owalk.pack(spec.n_half - 1, 0), owalk.pack(spec.n_half - 1, 1)]
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    din = dev(pts)
    dout = torch.empty_like(din)
    dh = torch.empty_like(din)
    ctx.step(tgt, k, chunk, sseed, 4, din, dout, dh)
    got_pts, got_h = host_u64(dout), host_u64(dh)
    want = [owalk.f_with_hash(spec, p) for p in pts]
    assert got_pts == [w[0] for w in want]
    assert got_h == [w[1] for w in want]


def test_rot_keys_cache_many_seeds(ctx):
    """n = 4 steps under more search seeds than the context keeps rotated-key tables for (32), then
    the first seeds again (their tables were evicted and are rebuilt): every step stays exact."""
    import torch
    n, k = 4, 4
    say("rot keys cache")
    tw, u = oracle_target(n, k, 9)
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    seeds = list(range(5000, 5036)) + [5000, 5001, 5035]
    for sseed in seeds:
        spec = owalk.make_spec(u, n, k, 0, sseed, delta=4)
        pts = seeded_inputs.random_points(spec.n_half, 2, sseed)
        din = dev(pts)
        dout = torch.empty_like(din)
        ctx.step(tgt, k, 0, sseed, 4, din, dout)
        assert host_u64(dout) == [owalk.f(spec, p) for p in pts], sseed


@pytest.mark.parametrize("n,k,seed", [(1, 6, 3), (2, 4, 1), (2, 5, 6), (3, 6, 2), (3, 5, 7), (4, 7, 1), (4, 6, 2)])
def test_planted_claw_on_gpu(ctx, n, k, seed):
    import torch
    say("planted", n, k, seed)
    tw, u = oracle_target(n, k, seed)
    xv, xw, c = owalk.planted_points(n, k, tw.paulis)
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    din = dev([owalk.pack(xv, 0), owalk.pack(xw, 1)])
    dout = torch.empty_like(din)
    dh = torch.empty_like(din)
    ctx.step(tgt, k, c, 77, 4, din, dout, dh)
    o, h = host_u64(dout), host_u64(dh)
    assert o[0] == o[1] and h[0] == h[1]


@pytest.mark.parametrize("n,k,delta,count,cap", [(1, 6, 3, 50, 160), (2, 4, 4, 64, 320), (2, 5, 3, 40, 160),
                                                 (3, 6, 3, 24, 160), (2, 4, 6, 40, 4), (4, 3, 2, 6, 80)])
def test_trails_parity(ctx, n, k, delta, count, cap):
    import torch
    say("trails", n, k, delta, count, cap)
    tw, u = oracle_target(n, k, 11)
    chunk = 0 if k % 2 == 0 else 2
    spec = owalk.make_spec(u, n, k, chunk, 5, delta=delta)
    starts = [owalk.start_point(spec, w, 0) for w in range(count)]
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    ds = dev(starts)
    ddp = torch.empty_like(ds)
    dlen = torch.empty(count, dtype=torch.int32, device="cuda:0")
    ctx.trails(tgt, k, chunk, 5, delta, ds, cap, ddp, dlen)
    got_dp, got_len = host_u64(ddp), [int(v) for v in dlen.cpu().tolist()]
    for i, s in enumerate(starts):
        dp, d = owalk.trail(spec, s, cap)
        assert got_len[i] == d
        if d:
            assert got_dp[i] == dp


def test_start_points_parity(ctx):
    import torch
    say("starts")
    for n, k in [(2, 4), (3, 5), (4, 7)]:
        tw, u = oracle_target(n, k, 3)
        chunk = 0 if k % 2 == 0 else 4
        spec = owalk.make_spec(u, n, k, chunk, 99, delta=4, version=3)
        tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
        out = torch.empty(500, dtype=torch.int64, device="cuda:0")
        ctx.start_points(tgt, k, chunk, 99, 1000, 7, 500, out, version=3)
        assert host_u64(out) == [owalk.start_point(spec, 1000 + i, 7) for i in range(500)]


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_canon_hash_parity(ctx, n):
    import torch
    say("canon hash", n)
    mats = []
    rng = np.random.default_rng(n)
    for i in range(4 if n < 4 else 2):
        ps = [int(v) for v in rng.integers(1, 4 ** n, 2 + i)]
        mats.append(zmat.product_of_rotations(ps, n))
    tw, u = oracle_target(n, 5, 2)
    mats.append(u)
    mats.append(zmat.clifford_from_word(n, seeded_inputs.random_clifford_word(n, 4)) @ u)
    mats.append(u.raise_to(u.e + 1))
    a = torch.tensor(np.stack([np.array(m.A, dtype=np.int32) for m in mats]), device="cuda:0")
    b = torch.tensor(np.stack([np.array(m.B, dtype=np.int32) for m in mats]), device="cuda:0")
    e = torch.tensor([m.e for m in mats], dtype=torch.int32, device="cuda:0")
    out = torch.empty(len(mats), dtype=torch.int64, device="cuda:0")
    ctx.canon_hash(n, 5, 3, 31, a, b, e, out, version=1)
    keys = owalk.make_keys(n, 5, 3, 31, version=1)
    got = host_u64(out)
    assert got == [owalk.matrix_hash(m, keys) for m in mats]
    assert got[-1] == got[-3] == got[-2]   # representation and left-Clifford invariance


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_canon_hash_wide_entries(ctx, n):
    """tcw_canon_hash with entries beyond int8 (the 64-bit modular path): random int32 matrices with
    exponents of either sign against the oracle, and a target raised by sqrt2^16 (entries x 256) hashes
    to what the int8 path gives for the target itself."""
    import torch
    say("canon hash wide", n)
    r = 4 ** n
    rng = np.random.default_rng(40 + n)
    mats = []
    for i in range(3 if n < 4 else 2):
        A = rng.integers(-(1 << 31), (1 << 31) - 1, size=(r, r), dtype=np.int64)
        B = rng.integers(-(1 << 31), (1 << 31) - 1, size=(r, r), dtype=np.int64)
        if i == 0:
            A[0, 0], B[0, 0] = -(1 << 31), (1 << 31) - 1
        mats.append(zmat.ZMat(A.astype(object), B.astype(object), int(rng.integers(-7, 40))))
    tw, u = oracle_target(n, 5, 2)
    big = u.raise_to(u.e + 16)
    assert max(abs(int(v)) for v in np.concatenate([big.A.ravel(), big.B.ravel()])) > 127
    mats.append(big)

    def run(ms):
        a = torch.tensor(np.stack([np.array(m.A, dtype=np.int64) for m in ms]).astype(np.int32), device="cuda:0")
        b = torch.tensor(np.stack([np.array(m.B, dtype=np.int64) for m in ms]).astype(np.int32), device="cuda:0")
        e = torch.tensor([m.e for m in ms], dtype=torch.int32, device="cuda:0")
        out = torch.empty(len(ms), dtype=torch.int64, device="cuda:0")
        ctx.canon_hash(n, 5, 3, 31, a, b, e, out, version=1)
        return host_u64(out)

    keys = owalk.make_keys(n, 5, 3, 31, version=1)
    got = run(mats)
    assert got == [owalk.matrix_hash(m, keys) for m in mats]
    assert run([u]) == [got[-1]]     # the int8 path on the target itself


@pytest.mark.parametrize("n,k,seed", [(1, 5, 2), (2, 4, 1), (2, 5, 3), (3, 6, 1), (3, 5, 4), (4, 7, 1)])
def test_claw_check_parity(ctx, n, k, seed):
    import torch
    say("claw check", n, k, seed)
    tw, u = oracle_target(n, k, seed)
    xv, xw, c = owalk.planted_points(n, k, tw.paulis)
    spec = owalk.make_spec(u, n, k, c, 1, delta=4)
    dec = osearch.claw_check(spec, owalk.pack(xv, 0), owalk.pack(xw, 1))
    assert dec is not None
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    bad = (xv + 1) % spec.n_half
    u0 = dev([owalk.pack(xw, 1), owalk.pack(bad, 0), owalk.pack(xv, 0)])
    u1 = dev([owalk.pack(xv, 0), owalk.pack(xw, 1), owalk.pack(xv, 0)])
    r = 4 ** n
    ok = torch.empty(3, dtype=torch.int32, device="cuda:0")
    perm = torch.empty(3 * r, dtype=torch.int32, device="cuda:0")
    sign = torch.empty(3 * r, dtype=torch.int8, device="cuda:0")
    ctx.claw_check(tgt, k, c, 1, u0, u1, ok, perm, sign)
    okh = ok.cpu().tolist()
    want_bad = osearch.claw_check(spec, owalk.pack(bad, 0), owalk.pack(xw, 1))
    assert okh[0] == 1 and okh[1] == (1 if want_bad is not None else 0) and okh[2] == 0
    assert perm.cpu().tolist()[:r] == dec.perm
    assert sign.cpu().tolist()[:r] == dec.sign


def test_walk_session_counters_n2(ctx):
    say("walk session n2")
    tw, u = oracle_target(2, 4, 1)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    w = ctx.walk(tgt, 4, 0, 1001, 4, walks=64, log2_table=10, cap=320)
    for _ in range(4):
        w.run(32)
    st = w.stats()
    assert st.steps == 64 * 32 * 4
    assert st.dps >= st.inserts > 0
    assert st.table_full == 0 and st.spin_timeouts == 0
    w.end()


def test_walk_kernel_full_size_sampled_n4(ctx):
    """n = 4, k = 7 at 2^20 walks, theta = 2^-12, 2^26 slots and 8 steps per walk per launch (the
    benchmark launch): sampled walks still on their first trail hold start = start(w, 0) and
    cur = f^len(start).  The two walks of a wavefront share the pair's 16 evaluations (side-0 steps
    alone, side-1 steps together), so when both are still on their first trail their lengths add up
    to 16."""
    say("walk n4 full size")
    n, k, delta = 4, 7, 12
    tw, u = oracle_target(n, k, 1)
    chunk = tw.paulis[0]
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    w = ctx.walk(tgt, k, chunk, 3001, delta, walks=1 << 20, log2_table=26, cap=20 << delta)
    w.run(8)
    st = w.stats()
    assert st.steps == (1 << 20) * 8
    spec = owalk.make_spec(u, n, k, chunk, 3001, delta=delta)
    sample = [0, 1, 777, 65535, 65536, 131071, 262144, 500000, 700001, 917503, (1 << 20) - 2, (1 << 20) - 1]
    checked = 0
    for wi in sample:
        s = w.read_states(wi, 1)[0]
        if int(s["trail"]) != 0 or int(s["mode"]) != 0:
            continue
        start = owalk.start_point(spec, wi, 0)
        assert int(s["start"]) == start
        pt = start
        for _ in range(int(s["len"])):
            pt = owalk.f(spec, pt)
        assert int(s["cur"]) == pt
        checked += 1
    assert checked >= len(sample) // 2  # at theta = 2^-12 almost every walk is still on its first trail
    for w0 in (0, 65536, 500000, (1 << 20) - 2):
        a, b = w.read_states(w0, 2)
        if all(int(x["trail"]) == 0 and int(x["mode"]) == 0 for x in (a, b)):
            assert int(a["len"]) + int(b["len"]) == 16
    w.end()


@pytest.mark.parametrize("n,k,delta,walks,lg", [(2, 4, 3, 64, 10), (3, 6, 4, 256, 14), (4, 6, 3, 64, 12)])
def test_dp_table_entries(ctx, n, k, delta, walks, lg):
    """The distinguished-point table after a few launches: every key is distinguished, keys are
    unique, and each value (start, length, ready bit) is a trail the oracle walks from that start to
    that key in exactly that many steps, with no distinguished point before."""
    say("dp table", n, k, delta)
    tw, u = oracle_target(n, k, 3)
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    seed = 4200 + n
    w = ctx.walk(tgt, k, 0, seed, delta, walks=walks, log2_table=lg, cap=20 << delta)
    w.run(16)
    w.run(16)
    table = w.read_table(lg)
    w.end()
    empty = (1 << 64) - 1
    keys = [int(key) for key, _ in table if int(key) != empty]
    assert keys and len(keys) == len(set(keys))
    spec = owalk.make_spec(u, n, k, 0, seed, delta=delta)
    entries = [(int(key), int(val)) for key, val in table if int(key) != empty]
    for key, val in entries[:24]:
        assert owalk.distinguished(spec, key)
        assert val >> 63 == 1
        start, length = val & 0x1FFFFFFFF, (val >> 33) & 0x3FFFFFFF
        assert length >= 1
        pt = start
        for i in range(length):
            pt = owalk.f(spec, pt)
            if i < length - 1:
                assert not owalk.distinguished(spec, pt)
        assert pt == key


def test_checkpoint_resume_continues_trails(ctx):
    say("checkpoint")
    tw, u = oracle_target(3, 6, 2)
    tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
    args = dict(k=6, chunk=0, seed=9, delta=8, walks=4096, log2_table=16, cap=20 << 8)
    w1 = ctx.walk(tgt, **args)
    w1.run(16)
    states, table = w1.read_states(0, 4096), w1.read_table(16)
    w1.run(16)
    a = w1.read_states(0, 4096)
    w2 = ctx.walk(tgt, **args)
    w2.write_states(0, states)
    w2.write_table(table)
    w2.run(16)
    b = w2.read_states(0, 4096)
    same_trail = (a["trail"] == states["trail"]) & (a["mode"] == 0)
    assert same_trail.sum() > 3000
    for f in ("start", "cur", "len", "trail"):
        assert np.array_equal(a[f][same_trail], b[f][same_trail])
    w1.end()
    w2.end()


@pytest.mark.parametrize("seed", list(range(1, 17)))
def test_search_n2_cfg1(ctx, seed):
    """n = 2, k = 4 targets; depths 0..3 are enumerated exhaustively, k = 4 by 64 walks at
    theta = 2^-4.  The T-count found equals the brute-force minimum (targets outside the
    brute-forced levels 0..3 have T-count 4); the result is exact.  The budget is 64 N / theta: the
    walk search is randomised (which trail reaches a distinguished point first differs from run to
    run), and with the default 16 N / theta a hard target misses now and then; this test checks
    what is found, not how often the default budget suffices (the bench's n2k4 leg reports that)."""
    say("search n2", seed)
    _, seen, _ = bfs.cosets_by_tcount(2, 3)
    tw, u = oracle_target(2, 4, seed)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    p = ctx.default_params(2)
    p.k_max = 4
    p.seed = 1000 + seed
    p.delta = 4
    p.walks = 64
    p.log2_table = 10
    p.enum_max = 64
    p.budget_beta = 64
    from paper_1606_07413_amd import tcw
    res = ctx.search(tgt, p)
    dec = tcw.decomposition_of(res)
    assert dec is not None
    tmin = bfs.min_tcount(u, seen)
    assert dec.t == (tmin if tmin is not None else 4)
    d = osearch.Decomposition(t=dec.t, paulis_desc=dec.paulis_desc, perm=dec.perm, sign=dec.sign)
    assert osearch.reconstruct(2, d).equals(u)



def test_search_rejects_out_of_range_params(ctx):
    """Parameters outside their documented ranges are refused before any device work, in a single
    search and in a batch; a batch still takes walks = log2_table = 0 as the autotuner's choice."""
    from paper_1606_07413_amd import tcw
    say("search parameter ranges")
    tw, u = oracle_target(2, 3, 4)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    bad = [("delta", 40), ("walks", 0), ("walks", 1 << 32), ("log2_table", 0), ("log2_table", 40),
           ("trail_cap_factor", 0), ("budget_beta", -1), ("version_factor", 0), ("enum_max", -5),
           ("chunk_first", 16), ("chunk_last", -1), ("max_seconds", -1.0), ("k_max", 65)]
    for name, value in bad:
        p = ctx.default_params(2)
        setattr(p, name, value)
        with pytest.raises(tcw.TcwError):
            ctx.search(tgt, p)
        if name not in ("walks", "log2_table") or value > 0:
            with pytest.raises(tcw.TcwError):
                ctx.search_batch([tgt], [p])
    p = ctx.default_params(2)
    p.k_max = 3
    p.walks = 0
    p.log2_table = 0
    results, _ = ctx.search_batch([tgt], [p])
    assert results[0].status == 1 and results[0].t <= 3

def test_search_n1_matches_bfs(ctx):
    from paper_1606_07413_amd import tcw
    say("search n1")
    _, seen, _ = bfs.cosets_by_tcount(1, 8)
    for seed in range(6):
        tw, u = oracle_target(1, 7, seed)
        tgt = ctx.target_from_words(1, tw.paulis, tw.clifford)
        p = ctx.default_params(1)
        p.k_max = 8
        p.seed = seed
        p.delta = 2
        p.walks = 256
        res = ctx.search(tgt, p)
        dec = tcw.decomposition_of(res)
        assert dec is not None and dec.t == bfs.min_tcount(u, seen)
        d = osearch.Decomposition(t=dec.t, paulis_desc=dec.paulis_desc, perm=dec.perm, sign=dec.sign)
        assert osearch.reconstruct(1, d).equals(u)


def test_search_n3_cfg2(ctx):
    """n = 3, k = 6 with 2^16 walks, theta = 2^-8 and 2^20 slots: the decomposition found is exact."""
    from paper_1606_07413_amd import tcw
    say("search n3 k6")
    tw, u = oracle_target(3, 6, 1)
    tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
    p = ctx.default_params(3)
    p.k_max = 6
    p.seed = 2001
    p.max_seconds = 60
    res = ctx.search(tgt, p)
    dec = tcw.decomposition_of(res)
    assert dec is not None and dec.t <= 6
    d = osearch.Decomposition(t=dec.t, paulis_desc=dec.paulis_desc, perm=dec.perm, sign=dec.sign)
    assert osearch.reconstruct(3, d).equals(u)
    say("n3 k6 search", res.seconds, "s", res.stats.steps, "steps", res.versions, "versions")


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_search_n3_default_theta(ctx, seed):
    """n = 3, k = 6 targets of T-count 6 (depths <= 5 are enumerated exhaustively, so 6 is the
    minimum) with the default theta, chosen from the table size: the search reaches depth 6 by walks
    and returns an exact decomposition of T-count 6."""
    from paper_1606_07413_amd import tcw
    say("search n3 k6 default theta", seed)
    tw, u = oracle_target(3, 6, seed)
    tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
    p = ctx.default_params(3)
    p.k_max = 6
    p.seed = 2100 + seed
    p.max_seconds = 60
    res = ctx.search(tgt, p)
    dec = tcw.decomposition_of(res)
    assert dec is not None and dec.t == 6
    d = osearch.Decomposition(t=dec.t, paulis_desc=dec.paulis_desc, perm=dec.perm, sign=dec.sign)
    assert osearch.reconstruct(3, d).equals(u)
    say("n3 k6 default theta", res.seconds, "s", res.stats.steps, "steps", res.versions, "versions")


def test_autotune_choices(ctx):
    say("autotune")
    for n, k, delta in [(2, 4, 4), (3, 6, 8)]:
        tw, u = oracle_target(n, k, 5)
        tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
        cfg = ctx.autotune(tgt, k, 0, delta, 7)
        npts = 2 * (4 ** n - 1) ** (k // 2)
        assert 64 <= cfg["walks"] <= max(64, npts // 4)
        assert 1 <= cfg["iters"] <= 64 and 10 <= cfg["log2_table"] <= 26 and cfg["steps_per_s"] > 0


def test_search_batch_mixed(ctx):
    """Mixed n and k in one batched search (the queue kernels of n = 1..4 in one round): every
    decomposition found reconstructs its target exactly, with T-count at most the generating k;
    n <= 2 minima match brute force; the n = 4 members (depths below 4 enumerated) are certified
    minimal."""
    from paper_1606_07413_amd import tcw
    say("batch")
    _, seen1, _ = bfs.cosets_by_tcount(1, 7)
    _, seen2, _ = bfs.cosets_by_tcount(2, 3)
    specs = [(1, 5, 1), (1, 7, 2), (2, 3, 3), (2, 4, 4), (2, 5, 5), (3, 3, 6), (3, 4, 7), (3, 6, 8), (2, 4, 9),
             (1, 6, 10), (4, 3, 11), (4, 4, 12)]
    targets, params, oracle_u = [], [], []
    for n, k, seed in specs:
        tw, u = oracle_target(n, k, 200 + seed)
        targets.append(ctx.target_from_words(n, tw.paulis, tw.clifford))
        oracle_u.append(u)
        p = ctx.default_params(n)
        p.k_max = k
        p.seed = 300 + seed
        p.walks = 0          # autotuner
        p.log2_table = 0
        p.iters_per_launch = 0
        # a generous budget: this test checks what is found, not how often budget 16 N/theta suffices
        p.budget_beta = 64
        p.max_seconds = 60
        params.append(p)
    results, agg = ctx.search_batch(targets, params)
    assert agg > 0
    for (n, k, seed), u, r in zip(specs, oracle_u, results):
        dec = tcw.decomposition_of(r)
        assert dec is not None, (n, k, seed)
        assert dec.t <= k
        d = osearch.Decomposition(t=dec.t, paulis_desc=dec.paulis_desc, perm=dec.perm, sign=dec.sign)
        assert osearch.reconstruct(n, d).equals(u)
        if n == 1:
            assert dec.t == bfs.min_tcount(u, seen1)
        if n == 2:
            tmin = bfs.min_tcount(u, seen2)
            assert dec.t == (tmin if tmin is not None else dec.t)
        if n == 4:
            assert r.minimal == 1 and r.failed_depths & ((1 << dec.t) - 1) == (1 << dec.t) - 1
