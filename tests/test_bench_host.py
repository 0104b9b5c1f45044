"""Host logic of bench.py (no GPU): the algorithmic work counts behind the roofline figures, the
published peaks, and the reading of the committed HBM-traffic summary with its source digest."""

import os
import shutil

import pytest

import bench


def test_work_counts_at_n4k7():
    # 23,552 lane-operations per step at n = 4, h = 3 (the first two rotations come from the table)
    assert bench.valu_ops_per_step(4, 3) == 23552
    # each further rotation adds R/2 butterflies of 12 operations
    assert bench.valu_ops_per_step(4, 4) - bench.valu_ops_per_step(4, 3) == 128 * 12
    # side 1: 16 N tiles x 8 K steps of 16 x 16 x 64 int8 MFMAs, half the steps
    assert bench.mfma_ops_per_step(4) == 0.5 * 2 * 16 * 16 * 64 * 16 * 8


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
