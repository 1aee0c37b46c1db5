"""Host-side logic of bench.py (no GPU): the L1 roofline's calibration table
and its interpolation, the counter summaries' sha256 gate, and the refusal of
more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_calibration_table_is_sorted_and_decreasing():
    cal = bench.l1_calibration()
    assert cal is not None and len(cal) >= 4
    miss = [m for m, _ in cal]
    rate = [r for _, r in cal]
    assert miss == sorted(miss) and miss[0] == 0.0 and miss[-1] > 0.9
    # more misses never make the L1 faster
    assert all(a >= b for a, b in zip(rate, rate[1:]))


def test_peak_interpolates_cycles_per_lookup():
    cal = [(0.0, 2.0), (0.5, 1.0), (1.0, 0.5)]
    assert bench.l1_peak_at(cal, 0.0) == pytest.approx(2.0)
    assert bench.l1_peak_at(cal, 0.5) == pytest.approx(1.0)
    # halfway between 0.5 and 1.0 cycles per lookup
    assert bench.l1_peak_at(cal, 0.25) == pytest.approx(1.0 / 0.75)
    assert bench.l1_peak_at(cal, 0.75) == pytest.approx(1.0 / 1.5)
    assert bench.l1_peak_at(cal, 1.5) is None


def test_counter_summary_gated_by_kernel_sources(tmp_path, monkeypatch):
    """Counter-derived fields are reported only while the summary's sha256 is
    that of the kernel sources, and only for the configuration it was taken on."""
    text = ("    traffic_bytes_per_launch = 123\n    l1_accesses_per_launch = 45\n"
            "    l2_requests_per_launch = 6\n    l2_hit_rate = 0.5\n    kernel_source_sha256 = %s\n")
    summary = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    args = type("A", (), dict(layout="tet16", sfc="hilbert", sort=0, block=0, eps=0.0, kernel=0))()
    summary.write_text(text % bench.kernel_source_hash())
    assert bench.measured_counters(args) == (123, 45, 6, 0.5)
    summary.write_text(text % ("0" * 64))
    assert bench.measured_counters(args) == (None, None, None, None)
    summary.write_text(text % bench.kernel_source_hash())
    args.eps = 1e-6
    assert bench.measured_counters(args) == (None, None, None, None)


def test_committed_summary_matches_current_sources():
    """The committed traffic summary describes the kernels as they are."""
    vals = bench.summary_values(bench.TRAFFIC_SUMMARY, ("kernel_source_sha256",))
    assert vals.get("kernel_source_sha256") == bench.kernel_source_hash()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
