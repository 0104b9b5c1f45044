"""Walk-step throughput of the deterministic-walk claw search at n = 4, k = 7 on one MI355X.

A benchmark step is one launch of the persistent walk kernel in which each of the 2^20
concurrent walks performs `iters` evaluations of the walk function f (decode, rotate,
canonicalise, hash, distinguished-point test, table insert, trail backtracking), on the
seeded synthetic n = 4, k = 7 target of seed 2 (T-count 7; chunk = its planted first
rotation), theta = 2^-12, 2^26 table slots.  value = walk steps per second over the timed
launches.

Also reported by default: the roofline of the walk kernel (VALU-bound), time-to-solution of
whole searches at n = 3, k = 6 and at n = 4, k = 7 (theta = 1/2, seeds 2, 3, 4, capped), the
configured-theta search of one planted chunk (capped, censored), the learned depth order
against the plain order at n = 3, the 64-target mixed batch (solved count and aggregate rate),
and the CPU oracle timed on the host on a bounded sample of the walk workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 32-bit VALU lane-operations per second.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# dense int8 MFMA peak (MI355X): 5.0e15 ops/s
MFMA_I8_PEAK_OPS = 5.0e15
# HBM3E (MI355X): 8 TB/s
HBM_PEAK_BYTES = 8.0e12


# Files the walk kernel is compiled from; the counter summary below records their digest together
# with the hipcc flags.
WALK_KERNEL_SOURCES = ("paper_1606_07413_amd/csrc/walk.hip", "paper_1606_07413_amd/csrc/common.h",
                       "paper_1606_07413_amd/csrc/internal.h")
TRAFFIC_SUMMARY = "profiles/k_walk_n4k7_traffic.md"


def kernel_source_digest() -> str:
    from paper_1606_07413_amd import build
    h = hashlib.sha256()
    for p in WALK_KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    h.update(" ".join(build.HIPCC_FLAGS).encode())
    return h.hexdigest()


def measured_traffic(walks: int, iters: int):
    """HBM bytes per launch of the walk kernel from the committed FETCH_SIZE / WRITE_SIZE summary,
    each counter scaled by what it reads for a plain copy of known size.  None when the summary is
    missing, was taken for another launch shape, or the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        fields = dict(re.findall(r"^- (\w+): (\S+)$", f.read(), re.M))
    try:
        if fields["source_sha256"] != kernel_source_digest():
            return None
        if int(fields["walks"]) != walks or int(fields["iters_per_launch"]) != iters:
            return None
        kib = (float(fields["fetch_kib_per_launch"]) * float(fields["fetch_scale"])
               + float(fields["write_kib_per_launch"]) * float(fields["write_scale"]))
    except (KeyError, ValueError):
        return None
    return kib * 1024.0


def valu_ops_per_step(n: int, h: int) -> float:
    """32-bit VALU lane-operations of one evaluation of f at n = 4 in its phi-linear form (mean over
    the two sides), counted per lane (four rows of the 256-entry key vector per lane, 64 lanes):

      per computed rotation (the first two of a step come from the table of rotated keys): per row
          the partner's sign (64-bit subtract 2, select 2), the add 2, the multiplication by
          1/sqrt2 = 2^30 mod p (shifts and mask 3, add 2) and the anticommutation select 2: 13
      side 0: the digest S_r = u_r folded below p: 4 per row
      both sides: sign fold min(c, p - c) = c ^ (bit 60 ? p : 0): 5 per row; NH element map and
          accumulation (two 32-bit key adds, one 32 x 32 -> 64 multiply-add, 64-bit add): 5 per row;
          the wave sum (four DPP stages and two cross-half swaps of 64-bit adds): 16 per lane
      side 1 (phi(S_c) u on int8 MFMA): digits of u and 2^31 u (the second set 7 per value,
          the bias 2 per value, two 4 x 4 byte transposes of 8 permutes per set, 8 xors per set): 84;
          raw tile sums (2 per tile, 16 tiles): 32; the 8 tile pairs' reduce-scatter and lazy
          weighted residue: 15 each; the final cross-half add, fold and exponent rotation of
          4 rows: 52
    which at h = 3 is 64 x (52 + 8 + 56 + 144) = 16,640 lane-operations (mean of the sides: side 0
    64 x 124, side 1 64 x 396).
    The compiled kernel issues more (address arithmetic, the trail and table logic); the counters
    give that figure separately."""
    if n != 4:
        raise ValueError("the lane-operation count is stated for n = 4")
    rows = 4
    rotations = 13 * rows * max(h - 2, 0)
    side0 = 4 * rows
    both = 5 * rows + 5 * rows + 16
    side1 = 84 + 32 + 8 * 15 + 52
    return 64.0 * (rotations + 0.5 * side0 + both + 0.5 * side1)


# Integer operations per step of the literal method (the 256 x 256 channel representation updated
# by h sparse butterflies, its 65,536 entries normalised and digested, the rows sorted): about 1.3e6
# at n = 4.  The kernel reaches the same f without forming that matrix.
LITERAL_OPS_PER_STEP_N4 = 1.3e6


def mfma_ops_per_step(n: int) -> float:
    """Useful int8 MFMA operations per step (mean over sides): on side 1 the 256 x 256 product
    phi(S_c) u over 8 digit rows for each of the two digit sets (u and 2^31 u), i.e.
    2 sets x 8 digits x 256 x 256 x 2.  Two walks of a wavefront whose next points are both on side 1
    share one pass of the 16 x 8 MFMAs (one walk's digits in A rows 0..7, the other's in rows 8..15),
    which issues exactly these products for both; a side-1 step without a partner issues twice its
    count, and the excess is not counted."""
    return 0.5 * (2 * 8 * 256 * 256 * 2)


COUNTER_SUMMARY = "profiles/k_walk_n4k7_counters.md"


def measured_counters(walks: int, iters: int):
    """Counter values per launch of the walk kernel from the committed summary, or None when it is
    missing, was taken for another launch shape, or the kernel sources changed since."""
    path = os.path.join(ROOT, COUNTER_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        fields = dict(re.findall(r"^- (\w+): (\S+)$", f.read(), re.M))
    try:
        if fields["source_sha256"] != kernel_source_digest():
            return None
        if int(fields["walks"]) != walks or int(fields["iters_per_launch"]) != iters:
            return None
        return {k: float(v) for k, v in fields.items() if k.startswith("SQ_") or k == "kernel_ms"}
    except (KeyError, ValueError):
        return None


def walk_roofline(n, h, steps_per_launch, avg_ms, walks, iters):
    """The walk kernel against the VALU peak (its bound), with the literal method's count, the
    compiled kernel's issued VALU work and busy share (counters), the int8 MFMA rate and HBM bytes."""
    secs = avg_ms * 1e-3
    ops = valu_ops_per_step(n, h)
    achieved = ops * steps_per_launch / secs
    traffic = measured_traffic(walks, iters)
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
           "frac": achieved / VALU_PEAK_OPS, "traffic": traffic, "traffic_unit": "HBM bytes per launch",
           "kernel": "k_walk<4,12>", "kernel_ms": avg_ms, "kernel_source_sha256": kernel_source_digest(),
           "ops_per_step": ops, "ops_unit": "32-bit VALU lane-operations of the phi-linear step",
           "literal_method": {"ops_per_step": LITERAL_OPS_PER_STEP_N4,
                              "frac": LITERAL_OPS_PER_STEP_N4 * steps_per_launch / secs / VALU_PEAK_OPS,
                              "note": "above 1: the kernel does not form the channel representation; it "
                                      "reaches the same f through phi-linearity"}}
    mf = mfma_ops_per_step(n) * steps_per_launch / secs
    out["mfma_i8"] = {"achieved": mf / 1e12, "peak": MFMA_I8_PEAK_OPS / 1e12, "unit": "Tops/s",
                      "frac": mf / MFMA_I8_PEAK_OPS, "counted": "useful products only"}
    out["hbm"] = None if traffic is None else {
        "achieved": traffic / secs / 1e9, "peak": HBM_PEAK_BYTES / 1e9, "unit": "GB/s", "frac": traffic / secs / HBM_PEAK_BYTES}
    c = measured_counters(walks, iters)
    if c is not None:
        mfma_insts = c["SQ_INSTS_VALU_MFMA_MOPS_I8"] * 512 / (16 * 16 * 64 * 2)
        issued = (c["SQ_INSTS_VALU"] - mfma_insts) * 64 / steps_per_launch
        waves_per_simd = c["SQ_WAVES"] / (256 * 4)
        out["counters"] = {
            "issued_valu_lane_ops_per_step": issued,
            "issued_frac": issued * steps_per_launch / secs / VALU_PEAK_OPS,
            "valu_busy": c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"] * waves_per_simd,
            "waves_per_simd": waves_per_simd, "kernel_ms_profiled": c["kernel_ms"], "source": COUNTER_SUMMARY}
    else:
        out["counters"] = None
    return out


def _oracle_worker(args):
    n, k, chunk, target_seed, seed, delta, pts = args
    import seeded_inputs
    from oracle import walk as owalk
    from oracle import zmat
    tw = seeded_inputs.target_words(n, k, target_seed)
    u = zmat.target_from_words(n, tw.paulis, tw.clifford)
    spec = owalk.make_spec(u, n, k, chunk, seed, delta)
    # timed after the target and the space are built
    t0 = time.perf_counter()
    for p in pts:
        owalk.f(spec, p)
    return len(pts), time.perf_counter() - t0


def host_cores() -> int:
    """Worker processes for the oracle: the cores this process may run on, at most 16 (one GPU's
    share of a shared host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


def cpu_baseline(n, k, chunk, target_seed, seed, delta, seconds: float):
    """The oracle's walk step on the host cores over a bounded sample of seeded points: one worker
    process per core, each timing its own evaluations after building the target, rates summed."""
    import seeded_inputs
    cores = host_cores()
    n_half = (4 ** n - 1) ** (k // 2)
    _, dt = _oracle_worker((n, k, chunk, target_seed, seed, delta, seeded_inputs.random_points(n_half, 2, 5)))
    per_proc = max(1, int(seconds / max(dt / 2, 1e-3)))
    jobs = [(n, k, chunk, target_seed, seed, delta, seeded_inputs.random_points(n_half, per_proc, 100 + i))
            for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    rate = sum(c / t for c, t in res)
    return {"value": rate, "unit": "walk steps/s", "cores": cores, "kind": "oracle",
            "os_cpu_count": os.cpu_count(),
            "sample": f"{total} walk steps (f evaluations) on seeded points of the n=4,k=7 planted chunk of target "
                      f"{target_seed}, {per_proc} per process over {cores} processes (rates timed inside each "
                      f"process after its set-up, summed); {wall:.1f} s wall with start-up"}


def _oracle_search_worker(args):
    n, k, target_seed, walk_seed, delta, walks, beta, enum_max = args
    import seeded_inputs
    from oracle import search as osearch
    from oracle import zmat
    tw = seeded_inputs.target_words(n, k, target_seed)
    u = zmat.target_from_words(n, tw.paulis, tw.clifford)
    r = osearch.search(u, n, k, walk_seed, lambda kk: delta, walks=walks, beta=beta, enum_max=enum_max)
    return target_seed, (r.decomposition.t if r.found else None), r.seconds, r.stats.steps


def cpu_configs(seconds: float):
    """The oracle on the host cores at every configuration: walk steps/s in one process and in a
    pool of one process per core (bounded samples of about `seconds` each), and the measured
    time-to-solution of the n = 2, k = 4 searches (16 targets, the same walk parameters as the GPU
    leg), one target per process."""
    import seeded_inputs
    cores = host_cores()
    rates = {}
    for name, n, k in (("n2k4", 2, 4), ("n3k6", 3, 6), ("n4k7", 4, 7)):
        spec = seeded_inputs.WORKLOADS[name]
        tw = seeded_inputs.target_words(n, k, spec["target_seeds"][0])
        chunk = tw.paulis[0] if k % 2 else 0
        n_half = (4 ** n - 1) ** (k // 2)
        ts = spec["target_seeds"][0]
        _, dt = _oracle_worker((n, k, chunk, ts, 5, spec["delta"], seeded_inputs.random_points(n_half, 2, 5)))
        per = max(1, int(seconds / max(dt / 2, 1e-4)))
        cnt, t1 = _oracle_worker((n, k, chunk, ts, 5, spec["delta"], seeded_inputs.random_points(n_half, per, 7)))
        per_proc = max(1, per // 2)
        jobs = [(n, k, chunk, ts, 5, spec["delta"], seeded_inputs.random_points(n_half, per_proc, 100 + i))
                for i in range(cores)]
        with mp.get_context("spawn").Pool(cores) as pool:
            res = pool.map(_oracle_worker, jobs)
        # the processes run side by side: the pool's rate is the sum of each one's own rate
        rates[name] = {"single_process": cnt / t1, "pool": sum(c / dt for c, dt in res), "cores": cores}
        _log(f"oracle {name}: {cnt / t1:.1f} steps/s single, {rates[name]['pool']:.1f} pool")
    spec = seeded_inputs.WORKLOADS["n2k4"]
    jobs = [(2, 4, s, spec["walk_seed_base"] + s, spec["delta"], spec["walks"], 16, 64) for s in spec["target_seeds"]]
    per_target = {}
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        for seed_t, t, secs, steps in pool.imap_unordered(_oracle_search_worker, jobs):
            per_target[seed_t] = {"found_t": t, "seconds": secs, "steps": steps}
            _log(f"oracle n2k4 target {seed_t}: t={t} {secs:.2f} s")
    wall = time.perf_counter() - t0
    secs = [v["seconds"] for v in per_target.values()]
    return {"walk_steps_per_s": rates,
            "tts_n2k4": {"targets": len(jobs), "found": sum(1 for v in per_target.values() if v["found_t"] is not None),
                         "mean_s": sum(secs) / len(secs), "max_s": max(secs), "wall_s": wall, "processes": cores,
                         "per_target": [per_target[s] | {"target_seed": s} for s in sorted(per_target)]}}


def config_legs(ctx):
    """The two smaller configurations on the GPU: time-to-solution of the n = 2, k = 4 searches
    (16 targets, 64 walks, theta = 2^-4, 2^10 slots; depths below 4 enumerated) and of the n = 3,
    k = 6 searches (8 targets x 20 walk seeds, 2^16 walks, theta = 2^-8, 2^20 slots), plus the
    walk-kernel rate at n = 2 and n = 3 for the configured and for 2^20 walks."""
    import statistics

    import seeded_inputs
    from paper_1606_07413_amd import tcw
    out = {}
    spec = seeded_inputs.WORKLOADS["n2k4"]
    per = []
    for s in spec["target_seeds"]:
        tw = seeded_inputs.target_words(2, 4, s)
        tgt = ctx.target_from_words(2, tw.paulis, tw.clifford)
        p = ctx.default_params(2)
        p.k_max = 4
        p.seed = spec["walk_seed_base"] + s
        p.delta = spec["delta"]
        p.walks = spec["walks"]
        p.log2_table = spec["log2_table"]
        p.enum_max = 64
        p.budget_beta = 16
        r = ctx.search(tgt, p)
        per.append({"target_seed": s, "found_t": r.t if r.status else None, "seconds": r.seconds,
                    "steps": r.stats.steps})
    _log(f"n2k4: {sum(1 for v in per if v['found_t'] is not None)}/{len(per)} found")
    out["tts_n2k4"] = {"targets": len(per), "found": sum(1 for v in per if v["found_t"] is not None),
                       "mean_s": statistics.mean(v["seconds"] for v in per),
                       "max_s": max(v["seconds"] for v in per), "per_target": per}
    spec = seeded_inputs.WORKLOADS["n3k6"]
    # the configured theta = 2^-8, then the library's default (theta from the table size)
    for label, delta in (("tts_n3k6", spec["delta"]), ("tts_n3k6_default_theta", -1)):
        rows = []
        for s in spec["target_seeds"]:
            tw = seeded_inputs.target_words(3, 6, s)
            tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
            secs, steps, ts = [], [], []
            for rep in range(20):
                p = ctx.default_params(3)
                p.k_max = 6
                p.seed = spec["walk_seed_base"] + 100 * s + rep
                p.delta = delta
                p.walks = spec["walks"]
                p.log2_table = spec["log2_table"]
                p.max_seconds = 60
                r = ctx.search(tgt, p)
                ts.append(r.t if r.status else None)
                secs.append(r.seconds)
                steps.append(r.stats.steps)
            rows.append({"target_seed": s, "found_t": sorted(set(t for t in ts if t is not None)),
                         "not_found": sum(1 for t in ts if t is None), "mean_s": statistics.mean(secs),
                         "median_s": statistics.median(secs), "max_s": max(secs),
                         "mean_steps": statistics.mean(steps)})
            _log(f"{label} target {s}: t={rows[-1]['found_t']} not found {rows[-1]['not_found']} "
                 f"mean {rows[-1]['mean_s']:.3f} s over 20 walk seeds")
        out[label] = {"targets": len(rows), "reps": 20, "delta": delta, "per_target": rows,
                      "not_found": sum(r["not_found"] for r in rows),
                      "mean_s": statistics.mean(r["mean_s"] for r in rows)}
    rates = {}
    for name, n, k, walks_list in (("n2k4", 2, 4, (64, 1 << 20)), ("n3k6", 3, 6, (1 << 16, 1 << 20))):
        spec = seeded_inputs.WORKLOADS[name]
        tw = seeded_inputs.target_words(n, k, spec["target_seeds"][0])
        tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
        for walks in walks_list:
            # a table that holds the distinguished points of every walk
            w = ctx.walk(tgt, k, 0, 77, spec["delta"], walks=walks, log2_table=max(spec["log2_table"], 22),
                         cap=20 << spec["delta"])
            iters = 64 if walks < 4096 else 8
            w.run(iters)
            ms = []
            before = w.stats().steps
            for _ in range(10):
                w.run(iters)
                ms.append(w.last_ms())
            steps = w.stats().steps - before
            w.end()
            rates[f"{name}_walks{walks}"] = {"walk_steps_per_s": steps / (sum(ms) * 1e-3),
                                             "kernel_ms": sum(ms) / len(ms), "iters_per_launch": iters}
            _log(f"walk {name} {walks} walks: {steps / (sum(ms) * 1e-3):.3g} steps/s")
    out["walk_rates"] = rates
    return out


def batch_leg(ctx, cap: float, configured_theta: bool = True):
    """64 seeded targets, n in {2,3,4}, k in {3..7}, searched together (autotuned walks and tables);
    theta = 2^-4, 2^-8, 2^-12 by n as configured, or the library's default (from the table size)."""
    import seeded_inputs
    from paper_1606_07413_amd import tcw
    spec = seeded_inputs.WORKLOADS["batch64"]
    words = seeded_inputs.batch_targets(spec["count"], spec["batch_seed"], spec["target_seed_base"])
    targets, params = [], []
    for i, tw in enumerate(words):
        targets.append(ctx.target_from_words(tw.n, tw.paulis, tw.clifford))
        p = ctx.default_params(tw.n)
        p.k_max = tw.k
        p.seed = 5000 + i
        p.delta = spec["delta_by_n"][tw.n] if configured_theta else -1
        p.walks = 0
        p.log2_table = 0
        p.iters_per_launch = 0
        p.max_seconds = cap
        params.append(p)
    t0 = time.perf_counter()
    results, agg = ctx.search_batch(targets, params)
    wall = time.perf_counter() - t0
    per = []
    for tw, r in zip(words, results):
        per.append({"n": tw.n, "k": tw.k, "found_t": r.t if r.status else None, "seconds": round(r.seconds, 4),
                    "censored": not r.status, "steps": r.stats.steps})
    _log(f"batch64 ({'configured' if configured_theta else 'default'} theta): "
         f"{sum(1 for r in results if r.status)}/{len(words)} found in {wall:.1f} s")
    return {"targets": len(words), "found": sum(1 for r in results if r.status), "wall_seconds": wall,
            "aggregate_walk_steps_per_s": agg, "per_target_cap_s": cap, "per_target": per}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def tts_n3k6_leg(ctx):
    """The whole optimal-T-count search of the n = 3, k = 6 target of seed 5 (optimum 6, so the depth-6
    walks run) at the configured theta = 2^-8 and at the library's default theta."""
    import seeded_inputs
    tw3 = seeded_inputs.target_words(3, 6, 5)
    t3 = ctx.target_from_words(3, tw3.paulis, tw3.clifford)
    runs = {}
    for name, d3 in (("configured_theta", seeded_inputs.WORKLOADS["n3k6"]["delta"]), ("default_theta", -1)):
        p3 = ctx.default_params(3)
        p3.k_max = 6
        p3.delta = d3
        p3.seed = 2001
        p3.max_seconds = 120
        r3 = ctx.search(t3, p3)
        runs[name] = {"seconds": r3.seconds, "found_t": r3.t if r3.status else None, "steps": r3.stats.steps,
                      "versions": r3.versions}
    t3.free()
    _log(f"tts n3k6: {runs}")
    return {"target_seed": 5, "measured": True, "delta": seeded_inputs.WORKLOADS["n3k6"]["delta"],
            **runs["configured_theta"], "default_theta": runs["default_theta"]}


def tts_n4_leg(ctx, cap: float, slice_s: float = 60.0, seeds=(2, 3, 4)):
    """The whole optimal-T-count search for seeded n = 4, k = 7 targets (seeds 2, 3, 4 have T-count 7)
    at theta = 1/2 (the paper's choice in Sec. 5.2 when the table holds the whole space: 2^27 slots
    >> N = 3.3e7 per chunk), a target not finished within `cap` seconds reported as censored, every
    chunk of an odd depth searched concurrently.  Depths 0..6 run as one call; depth 7 runs in calls
    of at most slice_s seconds, each starting a fresh range of function versions (a version starts
    from an empty table anyway), until a verified decomposition or the cap."""
    import seeded_inputs
    from paper_1606_07413_amd import tcw
    runs = []
    for ts in seeds:
        twn = seeded_inputs.target_words(4, 7, ts)
        tn = ctx.target_from_words(4, twn.paulis, twn.clifford)

        def params(k_max, version, seconds, only=None):
            p4 = ctx.default_params(4)
            p4.k_max = k_max
            p4.delta = 1
            p4.log2_table = 27
            p4.seed = 3100 + ts
            p4.version = version
            p4.chunk_parallel = 0
            p4.max_seconds = seconds
            if only is not None:
                p4.depth_order_kind = tcw.ORDER_GIVEN_FIRST
                p4.depth_order_len = 1
                p4.depth_order[0] = only
            return p4

        t0 = time.perf_counter()
        r = ctx.search(tn, params(6, 0, cap))
        steps, slices = r.stats.steps, 0
        print(f"tts n4k7 target {ts}: depths 0..6 done in {time.perf_counter() - t0:.1f} s, "
              f"t={r.t if r.status else None}", file=sys.stderr, flush=True)
        while not r.status and time.perf_counter() - t0 < cap:
            left = cap - (time.perf_counter() - t0)
            r = ctx.search(tn, params(7, (slices + 1) << 20, max(1e-3, min(slice_s, left)), only=7))
            steps += r.stats.steps
            slices += 1
            print(f"tts n4k7 target {ts}: depth 7 slice {slices} ended at {time.perf_counter() - t0:.1f} s, "
                  f"found={bool(r.status)}", file=sys.stderr, flush=True)
        runs.append({"target_seed": ts, "seconds": time.perf_counter() - t0,
                     "found_t": r.t if r.status else None, "chunk": r.chunk if r.status else None,
                     "censored": not r.status, "steps": steps, "depth7_slices": slices})
        tn.free()
    return {"measured": True, "theta": 0.5, "chunk_parallel": "all", "cap_s": cap, "runs": runs}


def tts_n4_planted_leg(ctx, cap: float, slice_s: float = 120.0, seeds=(2, 3, 4)):
    """The configured n = 4, k = 7 search (theta = 2^-12, 2^20 walks, 2^26 slots) on the planted
    chunk alone (P_1 of the generating word), one target at a time: the time until the exact check
    accepts a decomposition, in calls of at most slice_s seconds (each a fresh range of function
    versions) with a line of progress after each, until the cap."""
    import seeded_inputs
    from paper_1606_07413_amd import tcw
    runs = []
    for ts in seeds:
        twn = seeded_inputs.target_words(4, 7, ts)
        tn = ctx.target_from_words(4, twn.paulis, twn.clifford)
        chunk = twn.paulis[0]
        t0 = time.perf_counter()
        steps, slices, r = 0, 0, None
        while time.perf_counter() - t0 < cap:
            p4 = ctx.default_params(4)
            p4.k_max = 7
            p4.delta = 12
            p4.walks = 1 << 20
            p4.log2_table = 26
            p4.seed = 3200 + ts
            p4.version = slices << 20
            p4.chunk_first = p4.chunk_last = chunk
            p4.depth_order_kind = tcw.ORDER_GIVEN_FIRST
            p4.depth_order_len = 1
            p4.depth_order[0] = 7
            p4.max_seconds = max(1e-3, min(slice_s, cap - (time.perf_counter() - t0)))
            r = ctx.search(tn, p4)
            steps += r.stats.steps
            slices += 1
            print(f"planted chunk {chunk} of n4k7 target {ts}: slice {slices} ended at "
                  f"{time.perf_counter() - t0:.1f} s, {steps:.3g} steps, found={bool(r.status)}",
                  file=sys.stderr, flush=True)
            if r.status:
                break
        n_pts = 2 * 255 ** 3
        runs.append({"target_seed": ts, "chunk": chunk, "seconds": time.perf_counter() - t0,
                     "found_t": r.t if r is not None and r.status else None,
                     "censored": not (r is not None and r.status), "steps": steps,
                     "steps_over_N_per_theta": steps / (n_pts * 4096.0), "slices": slices})
        tn.free()
    return {"measured": True, "theta": 2.0 ** -12, "walks": 1 << 20, "log2_table": 26, "cap_s": cap,
            "runs": runs}


def sweep_leg(ctx, reps: int):
    """The scaling laws of Sec. 5.1 on one GPU, on the Toffoli gate (T-count 7, the whole search:
    depths 0..7, chunks of odd depths in ascending order, 2^20 slots), `reps` walk seeds per point:
      walks m = 2^10 .. 2^20 at theta = 1/2: the paper's runtime falls as 1/(processors); here m
      walks share one GPU, so steps-to-solution should stay about flat in m (until m / theta nears
      N) while the step rate rises until the GPU is full, and wall time = steps / rate;
      theta = 1/2 .. 1/32 at m = 2^16: steps and time rise about as 1/theta while the table holds
      every distinguished point (the appendix)."""
    import statistics

    import seeded_inputs
    v = seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES["toffoli"])
    tgt = ctx.target_from_unitary(3, v, 0)

    def point(walks, delta):
        secs, steps, ts = [], [], []
        for r in range(reps):
            p = ctx.default_params(3)
            p.k_max = 7
            p.delta = delta
            p.walks = walks
            p.log2_table = 20
            p.seed = 7000 + 31 * r
            p.chunk_parallel = 1
            p.max_seconds = 60
            res = ctx.search(tgt, p)
            secs.append(res.seconds)
            steps.append(res.stats.steps)
            ts.append(res.t if res.status == 1 else None)
        out = {"walks": walks, "theta": 2.0 ** -delta, "reps": reps, "found_t": sorted(set(t for t in ts if t)),
               "not_found": sum(1 for t in ts if t is None), "mean_s": statistics.mean(secs),
               "mean_steps": statistics.mean(steps), "steps_per_s": sum(steps) / sum(secs)}
        _log(f"sweep toffoli walks {walks} theta 2^-{delta}: {out['mean_s']:.3f} s, {out['mean_steps']:.3g} steps")
        return out

    res = {"walks_theta_half": [point(1 << lg, 1) for lg in range(10, 21, 2)],
           "theta_walks_2^16": [point(1 << 16, d) for d in range(1, 6)]}
    tgt.free()
    return res


# Sec. 5.2, Table 1: mean synthesis time of the T-count-7 three-qubit gates over 100 trials on
# 4096 Blue Gene/Q cores with half of the points distinguished (another machine: context only).
PAPER_TABLE1_SECONDS = {"toffoli": 25.9870, "fredkin": 25.0031, "peres": 25.4931}


def named_leg(ctx, reps: int, reps_default_theta: int):
    """Optimal T-count synthesis of the named gates: the whole depth loop k = 0..7 (chunks in
    ascending order at odd k) until a verified decomposition, repeated over walk seeds; plus the
    meet-in-the-middle certificate that no decomposition of T-count <= 6 exists."""
    import statistics

    import seeded_inputs
    from paper_1606_07413_amd import tcw
    out = {}
    for name in ("toffoli", "fredkin", "peres"):
        v = seeded_inputs.permutation_unitary(seeded_inputs.NAMED_GATES[name])
        tgt = ctx.target_from_unitary(3, v, 0)
        t0 = time.perf_counter()
        cert = ctx.min_tcount(tgt, 3)
        cert_s = time.perf_counter() - t0
        entry = {"certificate_tcount_gt_6": cert == -1, "certificate_seconds": cert_s}
        for label, delta, cpar, count in (("theta_2^-1", 1, 1, reps), ("theta_2^-1_all_chunks", 1, 0, reps),
                                          ("theta_2^-8", 8, 1, reps_default_theta)):
            secs, steps, ts = [], [], []
            for r in range(count):
                p = ctx.default_params(3)
                p.k_max = 7
                p.delta = delta
                p.seed = 5000 + 97 * r
                p.chunk_parallel = cpar
                p.max_seconds = 120
                res = ctx.search(tgt, p)
                dec = tcw.decomposition_of(res)
                ts.append(dec.t if dec else None)
                secs.append(res.seconds)
                steps.append(res.stats.steps)
            print(f"named {name} {label}: t={ts[0]} mean {statistics.mean(secs):.3f} s over {count}",
                  file=sys.stderr, flush=True)
            entry[label] = {
                "reps": count, "found_t": sorted(set(t for t in ts if t is not None)),
                "not_found": sum(1 for t in ts if t is None),
                "mean_s": statistics.mean(secs), "std_s": statistics.stdev(secs) if count > 1 else 0.0,
                "mean_steps": statistics.mean(steps)}
        # the last search's decomposition as gates (Sec. 5.3)
        if res.status == 1:
            gates = tcw.circuit_of(res)
            entry["circuit"] = {"gates": len(gates), "t": sum(1 for g, _ in gates if g in ("t", "tdg")),
                                "cnot": sum(1 for g, _ in gates if g == "cx")}
        entry["paper_mean_s_4096_bgq_cores"] = PAPER_TABLE1_SECONDS[name]
        out[name] = entry
    return out


def network_leg(ctx, batch: int = 4096, reps: int = 10):
    """The depth-order network at its own shape (4096 -> 512 x 3 -> 11, GELU, BF16 MFMA with FP32
    accumulation): seconds per forward pass and per training step (forward, backward, Adam) on a batch
    of synthetic features, and the rate of the GEMM work against the dense BF16 peak."""
    import torch

    from paper_1606_07413_amd import tcw
    inp, hidden, depth, classes = 4096, 512, 3, 11
    net = tcw.Network(ctx, inp, hidden, depth, classes, seed=42)
    g = torch.Generator(device="cuda:0").manual_seed(5)
    x = torch.randn((batch, inp), device="cuda:0", generator=g) * 0.5
    y = torch.randint(0, classes, (batch,), dtype=torch.int32, device="cuda:0", generator=g)
    probs = torch.empty((batch, classes), device="cuda:0")
    for _ in range(3):
        net.forward(x, probs)
        net.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(x, probs)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / reps
    fwd = 2.0 * batch * (inp * hidden + (depth - 1) * hidden * hidden + hidden * classes)
    net.free()
    # the vendor library on the layer-0 product alone (torch.mm, which calls hipBLASLt: BF16 operands,
    # FP32 accumulation, batch x inp times inp x hidden), a reference point for the network's own GEMM
    a = x.to(torch.bfloat16)
    w = (torch.randn((inp, hidden), device="cuda:0", generator=g) * 0.02).to(torch.bfloat16)
    for _ in range(3):
        torch.mm(a, w)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lib_reps = 20
    e0.record()
    for _ in range(lib_reps):
        torch.mm(a, w)
    e1.record()
    torch.cuda.synchronize()
    t_lib = e0.elapsed_time(e1) / lib_reps * 1e-3
    lib_flops = 2.0 * batch * inp * hidden
    del a, w
    _log(f"network: forward {t_fwd * 1e3:.3f} ms, train step {t_step * 1e3:.3f} ms; "
         f"torch.mm on the layer-0 product {t_lib * 1e6:.1f} us")
    return {"shape": f"{inp}->{hidden}x{depth}->{classes}", "batch": batch,
            "forward_ms": t_fwd * 1e3, "forward_tflops": fwd / t_fwd / 1e12,
            "train_step_ms": t_step * 1e3, "train_step_tflops": 3 * fwd / t_step / 1e12,
            "train_step_bf16_frac": 3 * fwd / t_step / 2.5e15,
            "flops_counted": "GEMMs only: 2 b (in h + (d-1) h^2 + h c) forward, 3x that per training step",
            "library_layer0_mm": {"what": f"torch.mm (hipBLASLt), BF16, {batch} x {hidden} x {inp}",
                                  "us": t_lib * 1e6, "tflops": lib_flops / t_lib / 1e12,
                                  "bf16_frac": lib_flops / t_lib / 2.5e15}}


LEARNED_ORDERS = ("plain", "learned_first")


def mlp_leg(ctx, train_count: int, epochs: int, eval_count: int, cap: float, orders=LEARNED_ORDERS,
            log2_table: int = 24):
    """Learned depth order at n = 3: train on seeded circuits (k uniform in 1..10) labelled by exact
    meet-in-the-middle search, then search each held-out target alone, once per order, with a wall
    clock cap per search (every chunk of an odd depth concurrent, 2^log2_table slots):
      plain              depths in increasing order (the paper's search);
      learned_first      depths by descending p_k / c_k (network probability over the steps the
                         depth costs when it holds no decomposition), the first verified decomposition
                         returned (time to the first exact answer);
      learned_certified  the same order, then every unsearched depth below a hit searched, the lowest
                         returned (certified minimal; it cannot save the failing depths' work);
      learned_prob_first depths by descending p_k alone, first hit (the order without costs).
    A search counts as solved only when its T-count is the target's minimum (the exact label when it
    is <= 6, else the least T-count any order found); a larger T-count is reported and counted as a
    failure, with the cap as its time."""
    import numpy as np
    import torch

    import seeded_inputs
    from paper_1606_07413_amd import tcw
    spec = seeded_inputs.WORKLOADS["mlp_n3"]
    n, classes = spec["n"], spec["classes"]
    h_max = 3

    def dataset(seed_lo, count):
        words, offsets, ks = seeded_inputs.mlp_target_arrays(seed_lo, seed_lo + count, n)
        feats = torch.empty((count, 16 ** n), dtype=torch.float32, device="cuda:0")
        labels = torch.empty(count, dtype=torch.int32, device="cuda:0")
        part = 1 << 18
        for lo in range(0, count, part):
            hi = min(count, lo + part)
            ctx.label_words(n, words[offsets[lo]:offsets[hi]], offsets[lo:hi + 1] - offsets[lo], ks[lo:hi], h_max,
                            777, feats[lo:hi], labels[lo:hi])
        return feats, labels, ks

    t0 = time.perf_counter()
    feats, labels, ks = dataset(spec["train_seeds"][0], train_count)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    gen_k = torch.from_numpy(ks).to("cuda:0")
    unknown = labels < 0
    labels = torch.where(unknown, gen_k, labels)       # T-count > 2 h_max: the generating k (an upper bound)
    del gen_k, ks
    _log(f"generated and labelled {train_count} circuits in {t_label:.1f} s ({int(unknown.sum())} above {2 * h_max})")
    net = tcw.Network(ctx, 16 ** n, spec["hidden"], spec["depth"], classes, seed=spec["init_seed"])
    t1 = time.perf_counter()
    loss = net.train(feats, labels, spec["batch"], epochs, 1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    _log(f"trained {epochs} epochs in {t_train:.1f} s, loss {loss:.3f}")
    flops = 6.0 * train_count * epochs * sum(a * b for a, b in [(16 ** n, 512), (512, 512), (512, 512), (512, classes)])
    del feats, labels

    ev = seeded_inputs.mlp_targets(spec["eval_seeds"][0], spec["eval_seeds"][0] + eval_count)
    ef, el, _ = dataset(spec["eval_seeds"][0], eval_count)
    probs = torch.empty((eval_count, classes), dtype=torch.float32, device="cuda:0")
    net.forward(ef, probs)
    pred = probs.argmax(dim=1).to(torch.int32)
    known = el >= 0
    acc = float((pred[known] == el[known]).float().mean()) if bool(known.any()) else None
    exact = [int(v) for v in el.cpu().tolist()]
    del ef

    runs = {name: [] for name in orders}
    t_eval = time.perf_counter()
    for i, w in enumerate(ev):
        tgt = ctx.target_from_words(n, w.paulis, w.clifford)
        for name in orders:
            p = ctx.default_params(n)
            p.k_max = spec["k_range"][1]
            p.seed = 9000 + i
            p.log2_table = log2_table
            p.chunk_parallel = 0
            p.max_seconds = cap
            if name != "plain":
                order, _ = net.depth_order(tgt, p.k_max, None if name == "learned_prob_first" else p)
                p.depth_order_kind = tcw.ORDER_GIVEN if name == "learned_certified" else tcw.ORDER_GIVEN_FIRST
                p.depth_order_len = len(order)
                for j, kk in enumerate(order):
                    p.depth_order[j] = kk
            r = ctx.search(tgt, p)
            runs[name].append((r.t if r.status == 1 else None, r.seconds, r.stats.steps))
        tgt.free()
        if i % 32 == 31:
            _log(f"learned order: {i + 1}/{eval_count} held-out targets searched, {time.perf_counter() - t_eval:.1f} s")
    # the minimum T-count of each held-out target: the exact label, else the least any order found
    t_min = []
    for i in range(eval_count):
        found = [runs[nm][i][0] for nm in orders if runs[nm][i][0] is not None]
        t_min.append(exact[i] if exact[i] >= 0 else (min(found) if found else None))
    out = {"train_circuits": train_count, "label_seconds": t_label, "unknown_labels": int(unknown.sum()),
           "epochs": epochs, "train_seconds": t_train, "final_loss": loss,
           "train_tflops": flops / t_train / 1e12, "mfma_bf16_frac": flops / t_train / 2.5e15,
           "eval_circuits": eval_count, "eval_accuracy_exact_labels": acc, "cap_s": cap, "log2_table": log2_table,
           "eval_seconds": time.perf_counter() - t_eval,
           "targets_with_known_minimum": sum(1 for v in t_min if v is not None)}
    ok = {nm: [runs[nm][i][0] is not None and runs[nm][i][0] == t_min[i] for i in range(eval_count)] for nm in orders}
    for nm in orders:
        secs = [runs[nm][i][1] if ok[nm][i] else cap for i in range(eval_count)]
        out[nm] = {"solved_minimal": sum(ok[nm]),
                   "larger_t": sum(1 for i in range(eval_count) if runs[nm][i][0] is not None and not ok[nm][i]),
                   "mean_tts_s_censored": float(np.mean(secs)),
                   "mean_steps": float(np.mean([runs[nm][i][2] for i in range(eval_count)]))}
    both = [i for i in range(eval_count) if all(ok[nm][i] for nm in orders)]
    out["solved_minimal_by_all"] = len(both)
    out["on_solved_by_all"] = {nm: {"mean_s": float(np.mean([runs[nm][i][1] for i in both])) if both else None,
                                    "mean_steps": float(np.mean([runs[nm][i][2] for i in both])) if both else None}
                               for nm in orders}
    # by minimum T-count: targets, and the mean seconds and steps of each order where all solved
    by_t = {}
    for tm in sorted(set(v for v in t_min if v is not None)):
        idx = [i for i in both if t_min[i] == tm]
        by_t[str(tm)] = {"targets": sum(1 for v in t_min if v == tm), "solved_by_all": len(idx)}
        for nm in orders:
            by_t[str(tm)][nm] = {"mean_s": float(np.mean([runs[nm][i][1] for i in idx])) if idx else None,
                                 "mean_steps": float(np.mean([runs[nm][i][2] for i in idx])) if idx else None}
    out["by_min_tcount"] = by_t
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=8, help="f evaluations per walk per launch")
    ap.add_argument("--walks", type=int, default=1 << 20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain depth order block")
    ap.add_argument("--no-network", action="store_true", help="skip the network forward / training-step timing")
    ap.add_argument("--batch", action="store_true",
                    help="run the 64-target mixed batch at the configured thetas too (the default theta runs anyway)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-target mixed batch")
    ap.add_argument("--batch-cap", type=float, default=20.0, help="per-target wall-clock cap (s)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration for profiles)")
    ap.add_argument("--tts-n4-cap", type=float, default=40.0, help="wall-clock cap per n = 4 target (s)")
    ap.add_argument("--tts-n4-seeds", default="2,3,4", help="n = 4, k = 7 target seeds (comma-separated)")
    ap.add_argument("--tts-n4-planted-cap", type=float, default=20.0,
                    help="wall-clock cap of the configured-theta planted-chunk search (s)")
    ap.add_argument("--tts-n4-planted-seeds", default="2", help="target seeds (comma-separated)")
    ap.add_argument("--named", action="store_true",
                    help="also synthesise Toffoli, Fredkin and Peres (n = 3, T-count 7) repeatedly")
    ap.add_argument("--named-reps", type=int, default=20)
    ap.add_argument("--sweeps", action="store_true", help="also run the walk-count and theta sweeps on Toffoli")
    ap.add_argument("--sweep-reps", type=int, default=8)
    ap.add_argument("--named-reps-default-theta", type=int, default=3)
    ap.add_argument("--configs", action="store_true",
                    help="also run the n = 2, k = 4 and n = 3, k = 6 searches and walk rates")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="with the CPU baseline, also time the oracle at every configuration")
    ap.add_argument("--mlp-train", type=int, default=1_000_000, help="training circuits of the learned order")
    ap.add_argument("--mlp-epochs", type=int, default=8)
    ap.add_argument("--mlp-eval", type=int, default=256, help="held-out circuits")
    ap.add_argument("--mlp-cap", type=float, default=1.0, help="wall-clock cap (s) of each held-out search")
    ap.add_argument("--mlp-log2-table", type=int, default=24, help="table slots (log2) of the held-out searches")
    ap.add_argument("--mlp-orders", default=",".join(LEARNED_ORDERS),
                    help="orders to compare (plain, learned_first, learned_certified, learned_prob_first)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the walk search here runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import seeded_inputs
    from paper_1606_07413_amd import tcw

    n, k, delta, log2_table = 4, 7, 12, 26
    seed, target_seed = 3001, 2
    tw = seeded_inputs.target_words(n, k, target_seed)
    chunk = tw.paulis[0]
    ctx = tcw.Context(0)
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    w = ctx.walk(tgt, k, chunk, seed, delta, walks=args.walks, log2_table=log2_table, cap=20 << delta)
    for i in range(args.warmup):
        w.run(args.iters)
        _log(f"warmup launch {i} done")
    torch.cuda.synchronize()
    before = w.stats().steps
    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        w.run(args.iters)
        kernel_ms.append(w.last_ms())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = w.stats()
    steps = st.steps - before
    elapsed = t1 - t0
    value = steps / elapsed
    avg_ms = sum(kernel_ms) / len(kernel_ms)
    _log(f"walk kernel: {value:.4g} steps/s, {avg_ms:.3f} ms per launch")
    w.end()
    tgt.free()
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    out = {
        "metric": "walk steps/s + time-to-solution at n=4,k=7; learned depth order vs plain",
        "value": value,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int8 exact (Z/(2^61-1) digests)",
        "data": "synthetic seeded target (product of 7 R(P) times a seeded Clifford; T-count 7)",
        "config": {"workload": "n4k7", "n": n, "k": k, "target_seed": target_seed, "chunk": chunk,
                   "walks": args.walks, "delta": delta, "log2_table": log2_table, "iters_per_launch": args.iters,
                   "parallelism": "1 GPU"},
        "roofline": walk_roofline(n, k // 2, args.walks * args.iters, avg_ms, args.walks, args.iters),
        "walk_stats": st.as_dict(),
    }
    if not args.no_tts:
        out["tts_n3k6"] = tts_n3k6_leg(ctx)
        out["tts_n4k7_theta_half"] = tts_n4_leg(ctx, args.tts_n4_cap,
                                                 seeds=tuple(int(v) for v in args.tts_n4_seeds.split(",")))
        out["tts_n4k7_planted_chunk_configured_theta"] = tts_n4_planted_leg(
            ctx, args.tts_n4_planted_cap, seeds=tuple(int(v) for v in args.tts_n4_planted_seeds.split(",")))
    if not args.no_network:
        out["network"] = network_leg(ctx)
    if not args.no_learned:
        out["learned_order"] = mlp_leg(ctx, args.mlp_train, args.mlp_epochs, args.mlp_eval, args.mlp_cap,
                                       orders=tuple(args.mlp_orders.split(",")), log2_table=args.mlp_log2_table)
    if args.configs:
        out["configs"] = config_legs(ctx)
    if not args.no_batch:
        out["batch64_default_theta"] = batch_leg(ctx, args.batch_cap, configured_theta=False)
        if args.batch:
            out["batch64"] = batch_leg(ctx, args.batch_cap)
    if args.named:
        out["named_n3_t7"] = named_leg(ctx, args.named_reps, args.named_reps_default_theta)
    if args.sweeps:
        out["sweeps_toffoli"] = sweep_leg(ctx, args.sweep_reps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, k, chunk, target_seed, seed, delta, args.cpu_seconds)
        if args.cpu_configs:
            out["cpu_baseline"]["configs"] = cpu_configs(5.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
