"""Host logic of bench.py (no GPU): the one-GPU rule and the committed
counter summaries that the roofline fields read, which are keyed to the
kernel sources they were measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_traffic_summary_matches_the_march_source():
    traffic = bench.load_traffic()
    assert traffic is not None and traffic > 1e11        # bytes per 256^3 sweep


def test_point_roofline_is_algorithmic():
    """The point-source roofline counts the method's FP64 operations per walk
    segment (not the kernel's own instruction count) against the FP64 peak."""
    import inspect
    src = inspect.getsource(bench.bench_point)
    assert "flops_per_seg = 4 + 2 * nb" in src
    assert bench.FP64_VECTOR_PEAK_TFLOPS == pytest.approx(78.6)


def test_summaries_of_other_sources_are_ignored(tmp_path, monkeypatch):
    src = tmp_path / "art_point.hip"
    src.write_text("// another kernel\n")
    monkeypatch.setattr(bench, "POINT_SRC", str(src))
    assert bench.point_valu_per_segment() is None
    msrc = tmp_path / "art_march.hip"
    msrc.write_text("// another march\n")
    monkeypatch.setattr(bench, "MARCH_SRC", str(msrc))
    assert bench.load_traffic() is None
    monkeypatch.setattr(bench, "POINT_VALU_FILE", str(tmp_path / "missing.json"))
    assert bench.point_valu_per_segment() is None


def test_valu_peak_is_the_chip_issue_rate():
    assert bench.VALU_LANE_PEAK == pytest.approx(256 * 4 * 16 * 2.4e9)
    with open(os.path.join(ROOT, "profiles", "point_128_valu.json")) as f:
        t = json.load(f)
    assert t["valu_lane_instructions_per_segment"] == pytest.approx(
        t["sq_insts_valu_per_call"] * 64 / t["segments_per_call"], rel=1e-4)
