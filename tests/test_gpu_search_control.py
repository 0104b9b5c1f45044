"""GPU tests of the search driver's control surface through the C ABI: seeded targets, the depth
orders and the minimality flag, trail-cap limits, stopping and resuming a search (walk states and
table restored exactly), the exhaustive mode's candidate read-out against the oracle, and the
distinguished-point table under stress (tiny tables, every point distinguished, candidate overflow).
"""

import struct

import numpy as np
import pytest

import seeded_inputs
from oracle import bfs
from oracle import search as osearch
from oracle import walk as owalk
from oracle import zmat

pytestmark = pytest.mark.gpu
MASK = (1 << 64) - 1
EMPTY = MASK


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_07413_amd import tcw
    assert torch.cuda.is_available()
    return tcw.Context(0)


def say(*a):
    print(*a, flush=True)


def oracle_target(n, k, seed):
    tw = seeded_inputs.target_words(n, k, seed)
    return tw, zmat.target_from_words(n, tw.paulis, tw.clifford)


def reconstructs(n, res, u):
    from paper_1606_07413_amd import tcw
    d = tcw.decomposition_of(res)
    return d is not None and osearch.reconstruct(
        n, osearch.Decomposition(t=d.t, paulis_desc=d.paulis_desc, perm=d.perm, sign=d.sign)).equals(u)


@pytest.mark.parametrize("n,k,seed", [(1, 3, 5), (2, 4, 9), (3, 5, 11), (4, 7, 2), (2, 0, 3)])
def test_target_random_matches_seeded_inputs(ctx, n, k, seed):
    """tcw_target_random draws the same words as the seeded-input module, builds the same exact
    channel rep as the oracle, and reports the Clifford factor as the oracle's signed permutation."""
    say("target random", n, k, seed)
    tgt, ps, perm, sign = ctx.target_random(n, k, seed)
    tw, u = oracle_target(n, k, seed)
    assert ps == tw.paulis
    a, b, e = tgt.channel()
    assert e == u.e and np.array_equal(a, np.array(u.A, dtype=np.int64)) and np.array_equal(
        b, np.array(u.B, dtype=np.int64))
    want = zmat.clifford_from_word(n, tw.clifford).signed_perm_of()
    assert want is not None and (perm, sign) == (list(want[0]), list(want[1]))


def test_target_random_rejects_ranges(ctx):
    from paper_1606_07413_amd import tcw
    for n, k in ((0, 3), (5, 3), (2, -1), (2, 65)):
        with pytest.raises(tcw.TcwError):
            ctx.target_random(n, k, 1)


def _given(p, order, kind):
    p.depth_order_kind = kind
    p.depth_order_len = len(order)
    for j, kk in enumerate(order):
        p.depth_order[j] = kk


def _even_tcount_seeds(count):
    _, seen, _ = bfs.cosets_by_tcount(2, 3)
    out = []
    for s in range(1, 200):
        t = bfs.min_tcount(oracle_target(2, 4, s)[1], seen)
        if (4 if t is None else t) % 2 == 0:
            out.append(s)
        if len(out) == count:
            return out
    return out


@pytest.mark.parametrize("seed", _even_tcount_seeds(4))
def test_given_order_returns_the_minimum(ctx, seed):
    """n = 2, k = 4 targets searched with depth 6 first.  TCW_ORDER_GIVEN searches the depths below a
    hit afterwards and returns the lowest: the brute-force minimum, flagged minimal.  With
    TCW_ORDER_GIVEN_FIRST the first verified decomposition comes back (depth 6: R(P)^2 is a Clifford,
    so every target of T-count t also decomposes at t + 2, and these targets have even T-count),
    flagged not minimal.  Every depth here
    is enumerated, so both answers are exact and deterministic."""
    from paper_1606_07413_amd import tcw
    say("given order", seed)
    _, seen, _ = bfs.cosets_by_tcount(2, 3)
    tw, u = oracle_target(2, 4, seed)
    tmin = bfs.min_tcount(u, seen)
    tmin = 4 if tmin is None else tmin
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    out = {}
    for name, kind in (("plain", tcw.ORDER_PLAIN), ("given", tcw.ORDER_GIVEN), ("first", tcw.ORDER_GIVEN_FIRST)):
        p = ctx.default_params(2)
        p.k_max = 6
        p.seed = 60 + seed
        p.enum_max = 1 << 16
        if kind != tcw.ORDER_PLAIN:
            _given(p, [6], kind)
        r = ctx.search(tgt, p)
        assert r.status == tcw.STATUS_FOUND and reconstructs(2, r, u), name
        out[name] = r
    assert out["plain"].t == tmin and out["plain"].minimal == 1
    assert out["given"].t == tmin and out["given"].minimal == 1
    below = (1 << tmin) - 1
    assert out["given"].failed_depths & below == below
    assert out["first"].t == 6 and out["first"].minimal == 0
    # the certified order did the plain order's work plus the depth it tried first
    assert out["given"].spaces > out["plain"].spaces


def test_trail_cap_ranges(ctx):
    """Trail caps that a table value cannot record (30 bits of length) are refused: up front when delta
    is given, in a walk session, and in a batch."""
    from paper_1606_07413_amd import tcw
    say("trail cap ranges")
    tw, u = oracle_target(2, 3, 4)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    p = ctx.default_params(2)
    p.delta = 26            # 20 * 2^26 > 2^30 - 1
    with pytest.raises(tcw.TcwError):
        ctx.search(tgt, p)
    with pytest.raises(tcw.TcwError):
        ctx.search_batch([tgt], [p])
    p.delta = 25            # 20 * 2^25 < 2^30: accepted
    p.k_max = 2
    assert ctx.search(tgt, p).status in (0, 1)
    p = ctx.default_params(2)
    p.trail_cap_factor = 1 << 30
    p.delta = 1
    with pytest.raises(tcw.TcwError):
        ctx.search(tgt, p)
    with pytest.raises(tcw.TcwError):
        ctx.walk(tgt, 4, 0, 1, 4, walks=64, log2_table=10, cap=tcw.MAX_TRAIL_CAP + 1)
    ctx.walk(tgt, 4, 0, 1, 4, walks=64, log2_table=10, cap=tcw.MAX_TRAIL_CAP).end()


# ---- checkpoints -----------------------------------------------------------------------------
STATE = np.dtype([("start", "<u8"), ("cur", "<u8"), ("pa", "<u8"), ("pb", "<u8"), ("na", "<u8"), ("ha", "<u8"),
                  ("len", "<u4"), ("trail", "<u4"), ("mode", "<u4"), ("rem", "<u4")])


def parse_checkpoint(blob):
    """The walk session inside a checkpoint (the layout written by tcw_checkpoint)."""
    import ctypes
    from paper_1606_07413_amd import tcw
    at = 0

    def take(fmt):
        nonlocal at
        v = struct.unpack_from("<" + fmt, blob, at)
        at += struct.calcsize("<" + fmt)
        return v if len(v) > 1 else v[0]

    magic, sp, sr, n, fp = take("QIIiQ")
    assert sp == ctypes.sizeof(tcw.WalkParams) and sr == ctypes.sizeof(tcw.Result)
    at += sp + sr
    cnt = take("Q")
    at += 4 * cnt
    take("i")                                    # oi
    cnt = take("Q")
    at += 4 * cnt
    take("iiQ")                                  # ri, refining, searched
    in_depth, k, cf, cl, chunk, delta, enum, iters, cut = take("9i")
    take("Qd")                                   # npts, elapsed
    has = take("i")
    if not has:
        return {"k": k, "chunk": chunk}
    budget, per_v, used, used_v, version, seen, walks, lg, cap, en, launches = take("QQQQIqqiIiq")
    stats = take("11Q")
    cc = take("Q")
    states = np.frombuffer(blob, dtype=STATE, count=walks, offset=at)
    at += walks * 64
    table = np.frombuffer(blob, dtype="<u8", count=2 << lg, offset=at).reshape(-1, 2)
    at += 16 << lg
    assert at == len(blob)
    return {"k": k, "chunk": chunk, "version": version, "walks": walks, "states": states, "table": table,
            "steps": stats[0]}


def test_checkpoint_resume_continues_trails(ctx):
    """n = 3, depth 6 by walks: a search stopped after 3 launches is resumed twice from its checkpoint
    for 2 more launches, in its own context and in a fresh one.  Every walk that reached no
    distinguished point after the checkpoint holds, in both, the same start, current point and length,
    and the current point is the oracle's f^len(start) (a trail is its start, end and length)."""
    from paper_1606_07413_amd import tcw
    say("checkpoint walk mode")
    tw, u = oracle_target(3, 6, 3)
    tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
    p = ctx.default_params(3)
    p.k_max = 6
    p.seed = 77
    p.delta = 8
    p.walks = 4096
    p.log2_table = 16
    p.iters_per_launch = 16
    p.launch_limit = 3
    _given(p, [6], tcw.ORDER_GIVEN_FIRST)
    r3 = ctx.search(tgt, p)
    assert r3.status == tcw.STATUS_STOPPED and r3.launches == 3
    blob = ctx.checkpoint()
    c = parse_checkpoint(blob)
    assert c["k"] == 6 and c["steps"] == 3 * 16 * 4096
    ra = ctx.resume(tgt, blob, launch_limit=2)
    assert r3.stats.steps == 3 * 16 * 4096
    assert ra.status == tcw.STATUS_STOPPED and ra.launches == 5 and ra.stats.steps == 5 * 16 * 4096
    a = parse_checkpoint(ctx.checkpoint())
    ctx2 = tcw.Context(0)
    tgt2 = ctx2.target_from_words(3, tw.paulis, tw.clifford)
    rb = ctx2.resume(tgt2, blob, launch_limit=2)
    assert rb.status == tcw.STATUS_STOPPED and rb.launches == 5
    b = parse_checkpoint(ctx2.checkpoint())
    assert a["steps"] == b["steps"] == 5 * 16 * 4096
    sa, sb, sc = a["states"], b["states"], c["states"]
    same = ((sa["trail"] == sc["trail"]) & (sb["trail"] == sc["trail"]) & (sa["mode"] == 0) & (sb["mode"] == 0)
            & (sc["mode"] == 0))
    assert same.sum() > 2000
    for f in ("start", "cur", "len"):
        assert np.array_equal(sa[f][same], sb[f][same])
    assert np.array_equal(sa["len"][same], sc["len"][same] + 32)     # 2 launches of 16 steps each
    # resumed walks against the oracle: cur = f^len(start(w, trail))
    spec = owalk.make_spec(u, 3, 6, 0, 77, delta=8)
    for w in np.flatnonzero(same)[:2]:
        s = sb[w]
        pt = owalk.start_point(spec, int(w), int(s["trail"]))
        assert int(s["start"]) == pt
        for _ in range(int(s["len"])):
            pt = owalk.f(spec, pt)
        assert int(s["cur"]) == pt


def test_checkpoint_resume_enumeration_identical(ctx):
    """n = 2, k = 4 with every depth enumerated two points per walk per launch: a search stopped in
    the middle of depth 4 and resumed in a fresh context returns the same decomposition, bit for bit,
    and the same counters as the uninterrupted search (the exhaustive mode's candidates do not depend
    on arrival order)."""
    from paper_1606_07413_amd import tcw
    say("checkpoint enumeration")
    _, seen, _ = bfs.cosets_by_tcount(2, 3)
    seed = next(s for s in range(1, 40) if bfs.min_tcount(oracle_target(2, 4, s)[1], seen) is None)
    tw, u = oracle_target(2, 4, seed)

    def params(limit):
        p = ctx.default_params(2)
        p.k_max = 4
        p.seed = 91
        p.walks = 64
        p.iters_per_launch = 2
        p.launch_limit = limit
        return p

    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    r0 = ctx.search(tgt, params(0))
    assert r0.status == tcw.STATUS_FOUND and r0.t == 4 and r0.minimal == 1 and reconstructs(2, r0, u)
    rs = ctx.search(tgt, params(33))          # 31 launches cover depths 1..3; stop inside depth 4
    assert rs.status == tcw.STATUS_STOPPED
    blob = ctx.checkpoint()
    assert parse_checkpoint(blob)["k"] == 4
    ctx2 = tcw.Context(0)
    tgt2 = ctx2.target_from_words(2, tw.paulis, tw.clifford)
    r1 = ctx2.resume(tgt2, blob)
    assert r1.status == tcw.STATUS_FOUND and r1.t == 4 and r1.minimal == 1
    assert list(r1.paulis[:4]) == list(r0.paulis[:4])
    assert list(r1.clifford_perm[:16]) == list(r0.clifford_perm[:16])
    assert list(r1.clifford_sign[:16]) == list(r0.clifford_sign[:16])
    assert r1.stats.steps == r0.stats.steps and r1.launches == r0.launches
    # another walk count enumerates the same candidates: the same decomposition again
    p = params(0)
    p.walks = 256
    r2 = ctx.search(tgt, p)
    assert list(r2.paulis[:4]) == list(r0.paulis[:4]) and list(r2.clifford_perm[:16]) == list(r0.clifford_perm[:16])


def test_stop_request_and_checkpoint_errors(ctx):
    """A stop request ends the next search at its first launch boundary; the checkpoint resumes to the
    answer.  A checkpoint is refused for another target, when truncated, and when no search stopped."""
    from paper_1606_07413_amd import tcw
    say("stop request")
    tw, u = oracle_target(2, 4, 2)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    p = ctx.default_params(2)
    p.k_max = 4
    p.seed = 5
    ctx.search_stop()
    r = ctx.search(tgt, p)
    assert r.status == tcw.STATUS_STOPPED and r.launches == 0
    blob = ctx.checkpoint()
    other = ctx.target_from_words(2, seeded_inputs.target_words(2, 4, 3).paulis, tw.clifford)
    with pytest.raises(tcw.TcwError):
        ctx.resume(other, blob)
    with pytest.raises(tcw.TcwError):
        ctx.resume(tgt, blob[:-3])
    with pytest.raises(tcw.TcwError):
        ctx.checkpoint()              # the failed resumes dropped the held search; none is stopped now
    r2 = ctx.resume(tgt, blob)
    assert r2.status == tcw.STATUS_FOUND and reconstructs(2, r2, u)
    with pytest.raises(tcw.TcwError):
        ctx.checkpoint()


# ---- exhaustive mode and the table under stress --------------------------------------------------
def test_enumeration_pairs_match_oracle(ctx):
    """Exhaustive mode on the identity at n = 2, k = 6: the candidates read out of the table are
    exactly the oracle's pairs (least x of side 0, least x of side 1) over every matrix hash reached
    from both sides."""
    import torch
    say("enumeration pairs")
    n, k, seed = 2, 6, 5
    u = zmat.ZMat.identity(n)
    tgt = ctx.target_from_words(n, [], [])
    spec = owalk.make_spec(u, n, k, 0, seed, delta=0)
    first = {0: {}, 1: {}}
    for b in (0, 1):
        for x in range(spec.n_half):
            first[b].setdefault(owalk.f_with_hash(spec, owalk.pack(x, b))[1], x)
    want = sorted((first[0][h], first[1][h] | (1 << 32)) for h in set(first[0]) & set(first[1]))
    w = ctx.walk(tgt, k, 0, seed, 0, walks=512, log2_table=15, cap=2, enumerate=True)
    pairs, total = w.claws()
    assert total == 0                  # before the last point nothing is read out
    w.run(64)
    assert w.stats().active_walks == 0
    pairs, total = w.claws()
    st = w.stats()
    w.end()
    assert total == len(want) and st.claws == len(want) and st.claws_dropped == 0
    assert sorted(pairs) == want
    assert st.steps == 2 * spec.n_half and st.table_full == 0


def test_claw_candidates_beyond_the_buffer_are_counted(ctx):
    """n = 2, k = 8 on the identity: more keys are reached from both sides than the 4096-pair buffer
    holds; the overflow is counted in claws_dropped, and the pairs kept are valid candidates."""
    say("claws dropped")
    n, k, seed = 2, 8, 5
    tgt = ctx.target_from_words(n, [], [])
    w = ctx.walk(tgt, k, 0, seed, 0, walks=4096, log2_table=19, cap=2, enumerate=True)
    w.run(32)
    assert w.stats().active_walks == 0
    pairs, total = w.claws()
    st = w.stats()
    w.end()
    assert total > 4096 and len(pairs) == 4096
    assert st.claws_dropped == total - 4096 and st.claws == total
    spec = owalk.make_spec(zmat.ZMat.identity(n), n, k, 0, seed, delta=0)
    for u0, u1 in pairs[:4]:
        assert (u0 >> 32) == 0 and (u1 >> 32) == 1
        assert owalk.f_with_hash(spec, u0)[1] == owalk.f_with_hash(spec, u1)[1]


def _check_entries(spec, table, limit):
    keys = [int(kk) for kk, _ in table if int(kk) != EMPTY]
    assert len(keys) == len(set(keys))
    for kk, val in [(int(kk), int(v)) for kk, v in table if int(kk) != EMPTY][:limit]:
        assert owalk.distinguished(spec, kk) and val >> 63 == 1
        start, length = val & 0x1FFFFFFFF, (val >> 33) & 0x3FFFFFFF
        assert length >= 1
        pt = start
        for i in range(length):
            pt = owalk.f(spec, pt)
            if i < length - 1:
                assert not owalk.distinguished(spec, pt)
        assert pt == kk
    return keys


def test_tiny_table_fills_without_losing_keys(ctx):
    """16- and 32-slot tables at theta = 1/4 and 1/2 overflow: inserts beyond it are counted as table_full, no reader
    times out, the kernel finishes, and every stored entry is a valid trail (oracle)."""
    say("tiny table")
    tw, u = oracle_target(2, 4, 6)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    for lg, delta in ((4, 2), (5, 1)):
        w = ctx.walk(tgt, 4, 0, 123, delta, walks=64, log2_table=lg, cap=20 << delta)
        for _ in range(4):
            w.run(32)
        st = w.stats()
        table = w.read_table(lg)
        w.end()
        assert st.steps == 64 * 32 * 4 and st.table_full > 0 and st.spin_timeouts == 0
        keys = _check_entries(owalk.make_spec(u, 2, 4, 0, 123, delta=delta), table, 64)
        assert len(keys) == 1 << lg                    # full, every slot a distinct key
        assert st.inserts == len(keys)


def test_every_point_distinguished(ctx):
    """theta = 1 (delta = 0): every step ends a trail, so many walks land on the same keys at once; the
    table keeps one entry per key, each a trail of length 1 from its stored start (oracle)."""
    say("delta 0")
    tw, u = oracle_target(2, 4, 8)
    tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
    w = ctx.walk(tgt, 4, 0, 321, 0, walks=256, log2_table=12, cap=20)
    w.run(32)
    st = w.stats()
    table = w.read_table(12)
    w.end()
    assert st.spin_timeouts == 0 and st.table_full == 0 and st.dps > 0
    spec = owalk.make_spec(u, 2, 4, 0, 321, delta=0)
    keys = _check_entries(spec, table, 10 ** 6)
    assert len(keys) == st.inserts and len(keys) <= 2 * spec.n_half
    for kk, val in [(int(kk), int(v)) for kk, v in table if int(kk) != EMPTY]:
        assert (val >> 33) & 0x3FFFFFFF == 1


def test_dp_table_entries_n4(ctx):
    """n = 4, k = 5 at theta = 1/4 with 256 walks: stored entries are distinguished, unique, and reached
    from their stored start in their stored length (oracle, a few entries)."""
    say("dp table n4")
    tw, u = oracle_target(4, 5, 3)
    chunk = tw.paulis[0]
    tgt = ctx.target_from_words(4, tw.paulis, tw.clifford)
    w = ctx.walk(tgt, 5, chunk, 4404, 2, walks=256, log2_table=12, cap=80)
    w.run(4)
    st = w.stats()
    table = w.read_table(12)
    w.end()
    assert st.inserts > 0 and st.table_full == 0 and st.spin_timeouts == 0
    _check_entries(owalk.make_spec(u, 4, 5, chunk, 4404, delta=2), table, 3)


def test_trail_n4k7_to_a_distinguished_point(ctx):
    """n = 4, k = 7 (the benchmark's space) at theta = 1/4: trails from seeded starts end at the
    oracle's distinguished point after the oracle's number of steps."""
    import torch
    say("trail n4k7")
    tw, u = oracle_target(4, 7, 2)
    chunk = tw.paulis[0]
    spec = owalk.make_spec(u, 4, 7, chunk, 31, delta=2)
    starts = [owalk.start_point(spec, w, 0) for w in range(3)]
    tgt = ctx.target_from_words(4, tw.paulis, tw.clifford)
    ds = torch.tensor([s if s < (1 << 63) else s - (1 << 64) for s in starts], dtype=torch.int64, device="cuda:0")
    dp = torch.empty_like(ds)
    ln = torch.empty(3, dtype=torch.int32, device="cuda:0")
    ctx.trails(tgt, 7, chunk, 31, 2, ds, 80, dp, ln)
    got_dp = [int(v) & MASK for v in dp.cpu().tolist()]
    got_len = [int(v) for v in ln.cpu().tolist()]
    for i, s in enumerate(starts):
        want_dp, want_len = owalk.trail(spec, s, 80)
        assert got_len[i] == want_len and want_len >= 1
        assert got_dp[i] == want_dp


def test_batch_exhaustive_matches_single_searches(ctx):
    """Exhaustive mode does not depend on walk count or arrival order (the table keeps each side's
    least point per key, candidates are read after the last point and checked in sorted order), so a
    batch of enumerated members of every qubit count -- the queue kernels of n = 1..4 sharing rounds,
    one target entered twice -- returns, member by member, the decomposition that searching the
    target alone returns, bit for bit."""
    from paper_1606_07413_amd import tcw
    say("batch exhaustive vs single")
    specs = [(1, 3, 21), (1, 7, 22), (2, 4, 23), (2, 5, 24), (3, 4, 25), (3, 5, 26), (4, 3, 27), (4, 4, 28),
             (2, 4, 23)]

    def params(n, k, walks):
        p = ctx.default_params(n)
        p.k_max = k
        p.seed = 610
        p.walks = walks
        p.enum_max = 1 << 18      # every space of these targets is enumerated
        p.max_seconds = 60
        return p

    targets, us = [], []
    for n, k, seed in specs:
        tw, u = oracle_target(n, k, seed)
        targets.append(ctx.target_from_words(n, tw.paulis, tw.clifford))
        us.append(u)
    batch, _ = ctx.search_batch(targets, [params(n, k, 256) for n, k, _ in specs])
    for (n, k, seed), tgt, u, rb in zip(specs, targets, us, batch):
        rs = ctx.search(tgt, params(n, k, 1024))
        assert rs.status == rb.status == tcw.STATUS_FOUND, (n, k, seed)
        assert rs.t == rb.t <= k and rs.minimal == rb.minimal == 1
        t, r = rs.t, 4 ** n
        assert list(rb.paulis[:t]) == list(rs.paulis[:t]) and rb.chunk == rs.chunk, (n, k, seed)
        assert list(rb.clifford_perm[:r]) == list(rs.clifford_perm[:r])
        assert list(rb.clifford_sign[:r]) == list(rs.clifford_sign[:r])
        assert reconstructs(n, rb, u)
