"""The benchmark's contract that holds without a GPU: one GPU only, and
profile figures only for the kernel sources and launch shape they were
taken on."""
import os
import subprocess
import sys

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_figures_need_matching_sources_and_shape(tmp_path, monkeypatch):
    src = open(bench.PROFILE_SUMMARY).read()
    digest = bench.kernel_source_digest()
    # a summary written for other sources is not used
    stale = tmp_path / "pmc.txt"
    stale.write_text(src.replace("kernel_source_digest: ", "kernel_source_digest: x", 1))
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(stale))
    assert bench.traffic_from_profile(700000, "benchmarked") is None
    # a summary for these sources is used at its own shape and workload only
    fresh = tmp_path / "pmc2.txt"
    lines = [l if not l.startswith("kernel_source_digest:") else f"kernel_source_digest: {digest}"
             for l in src.splitlines()]
    fresh.write_text("\n".join(lines) + "\n")
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(fresh))
    assert bench.traffic_from_profile(700000, "benchmarked") > 0
    assert bench.traffic_from_profile(700000, "library") is None
    assert bench.traffic_from_profile(700000, None) is None
    assert bench.traffic_from_profile(1000, "benchmarked") is None
