"""Host logic of bench.py (no GPU): the algorithmic flop count of a rollout
step, the one-GPU rule, and that the committed counter summaries are used
only for the kernel source they were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flops_per_rollout_step_at_the_sine_lane():
    # 221 waypoints, 60 obstacle circles, 3 ego circles: 73 + 1326 + 1260
    assert bench.flops_per_rollout_step(221, 60, 3) == 2659
    # no scene terms: the fixed part alone
    assert bench.flops_per_rollout_step(0, 0, 3) == 73
    # each waypoint and each circle pair adds its own share
    assert bench.flops_per_rollout_step(1, 0, 1) - bench.flops_per_rollout_step(0, 0, 1) == 6
    assert bench.flops_per_rollout_step(0, 1, 2) - bench.flops_per_rollout_step(0, 0, 2) == 14


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_summaries_only_for_their_kernel_source(tmp_path, monkeypatch):
    rec = {"kernel_source_sha256_16": bench.kernel_source_hash(), "hbm_bytes_per_launch": 123}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic(1) == 123
    rec["kernel_source_sha256_16"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.load_traffic(1) is None
    f.write_text("not json")
    assert bench.load_traffic(1) is None


def test_trace_record_only_for_its_kernel_source(tmp_path, monkeypatch):
    rec = {"kernel_source_sha256_16": bench.kernel_source_hash(),
           "iteration": {"average_ns": 1.0, "calls": 1}, "combine": {"average_ns": 1.0}}
    f = tmp_path / "trace.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    monkeypatch.setattr(bench, "TRACE_FILE", str(f))
    assert bench.load_trace()["iteration"]["average_ns"] == 1.0
    rec["kernel_source_sha256_16"] = "f" * 16
    f.write_text(json.dumps(rec))
    assert bench.load_trace() is None
