"""Host logic of bench.py (no GPU): the algorithmic work counts behind the roofline figures, the
published peaks, and the reading of the committed HBM-traffic summary with its source digest."""

import os
import shutil

import pytest

import bench


def test_work_counts_at_n4k7():
    # 64 lanes x 260 lane-operations per step at n = 4, h = 3 (side 0: 124, side 1: 396; the first
    # two rotations come from the table)
    assert bench.valu_ops_per_step(4, 3) == 64 * 260 == 16640
    # each further rotation adds 13 operations on each of a lane's four rows
    assert bench.valu_ops_per_step(4, 4) - bench.valu_ops_per_step(4, 3) == 64 * 13 * 4
    # the literal method's count exceeds the phi-linear step's by far
    assert bench.LITERAL_OPS_PER_STEP_N4 > 50 * bench.valu_ops_per_step(4, 3)
    # side 1 (half the steps): two digit sets x 8 digit rows x the 256 x 256 product, multiply and add
    assert bench.mfma_ops_per_step(4) == 0.5 * 2 * 8 * 256 * 256 * 2
    # one pass of the 16 N tiles x 8 K steps of 16 x 16 x 64 MFMAs serves two walks' side-1 steps
    assert 2 * bench.mfma_ops_per_step(4) == 0.5 * 2 * 16 * 16 * 64 * 16 * 8
    with pytest.raises(ValueError):
        bench.valu_ops_per_step(3, 3)


def test_host_cores_bounded():
    assert 1 <= bench.host_cores() <= 16


def test_peaks_are_the_published_ones():
    assert bench.VALU_PEAK_OPS == pytest.approx(39.3216e12)
    assert bench.MFMA_I8_PEAK_OPS == 5.0e15
    assert bench.HBM_PEAK_BYTES == 8.0e12


def test_traffic_summary_reading(tmp_path, monkeypatch):
    """bench.measured_traffic reads a summary written for the current kernel sources and launch shape
    (fetch x scale + write, per launch) and gives None for another shape or for changed sources."""
    for p in bench.WALK_KERNEL_SOURCES + ("paper_1606_07413_amd/build.py", "paper_1606_07413_amd/__init__.py"):
        dst = tmp_path / p
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, p), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    summary = tmp_path / bench.TRAFFIC_SUMMARY
    summary.parent.mkdir(parents=True, exist_ok=True)
    summary.write_text("# traffic\n\n"
                       f"- source_sha256: {bench.kernel_source_digest()}\n"
                       "- walks: 1048576\n- iters_per_launch: 8\n"
                       "- fetch_kib_per_launch: 1000.0\n- fetch_scale: 2.0\n"
                       "- write_kib_per_launch: 24.0\n- write_scale: 1.0\n")
    assert bench.measured_traffic(1 << 20, 8) == pytest.approx(2024.0 * 1024)
    # another launch shape is not covered by it
    assert bench.measured_traffic(1 << 19, 8) is None
    # a changed kernel source no longer matches the recorded digest
    with open(tmp_path / bench.WALK_KERNEL_SOURCES[0], "a") as f:
        f.write("\n// changed\n")
    assert bench.measured_traffic(1 << 20, 8) is None


def test_counter_summary_reading(tmp_path, monkeypatch):
    """bench.measured_counters reads the per-launch counter summary for the current kernel sources and
    launch shape; walk_roofline turns it into issued lane-operations per step and the VALU busy share."""
    for p in bench.WALK_KERNEL_SOURCES + ("paper_1606_07413_amd/build.py", "paper_1606_07413_amd/__init__.py"):
        dst = tmp_path / p
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, p), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    steps = (1 << 20) * 8
    summary = tmp_path / bench.COUNTER_SUMMARY
    summary.parent.mkdir(parents=True, exist_ok=True)
    # 300 VALU instructions per step of which 32 are MFMAs (32 x 64 MOPS units of 512 ops each)
    summary.write_text("# counters\n\n"
                       f"- source_sha256: {bench.kernel_source_digest()}\n"
                       "- walks: 1048576\n- iters_per_launch: 8\n- kernel_ms: 10.0\n"
                       f"- SQ_WAVES: 3072\n- SQ_INSTS_VALU: {300 * steps}\n"
                       f"- SQ_INSTS_VALU_MFMA_MOPS_I8: {32 * 64 * steps}\n"
                       f"- SQ_ACTIVE_INST_VALU: {400 * steps}\n- SQ_WAVE_CYCLES: {1600 * steps}\n")
    c = bench.measured_counters(1 << 20, 8)
    assert c["SQ_WAVES"] == 3072 and c["kernel_ms"] == 10.0
    roof = bench.walk_roofline(4, 3, steps, 10.0, 1 << 20, 8)
    assert roof["counters"]["issued_valu_lane_ops_per_step"] == pytest.approx((300 - 32) * 64)
    assert roof["counters"]["valu_busy"] == pytest.approx(400 / 1600 * 3)
    assert roof["frac"] == pytest.approx(16640 * steps / 10e-3 / bench.VALU_PEAK_OPS)
    assert roof["literal_method"]["frac"] > 1
    assert bench.measured_counters(1 << 19, 8) is None
    with open(tmp_path / bench.WALK_KERNEL_SOURCES[0], "a") as f:
        f.write("\n// changed\n")
    assert bench.measured_counters(1 << 20, 8) is None
    assert bench.walk_roofline(4, 3, steps, 10.0, 1 << 20, 8)["counters"] is None
