"""Host logic of bench.py (no GPU): the roofline arithmetic of the blend
sweep, the check that the committed traffic counters belong to the current
kernel source, and the refusal of more than one GPU."""

import importlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def bench(monkeypatch):
    # bench.py raises GPU_MAX_HW_QUEUES when imported; keep that in the test
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "4")
    monkeypatch.syspath_prepend(ROOT)
    import bench as b
    return importlib.reload(b)


def test_roofline_constants(bench):
    # 13 plain + 11 FMA + 4 transcendentals per pair (39 FLOP); 256 CUs at
    # 2.4 GHz, 128 lanes/clk for the arithmetic and 32 for transcendentals
    assert bench.BLEND_FLOP == 39 and bench.FAR_FLOP == 9
    cycles = 24 / 128 + 4 / 32
    assert bench.PEAK_PAIRS == pytest.approx(256 * 2.4e9 / cycles)
    assert bench.PEAK_TFLOPS == pytest.approx(39 * 256 * 2.4e9 / cycles / 1e12)
    assert 76.0 < bench.PEAK_TFLOPS < 77.0


def test_roofline_object(bench):
    r = bench.roofline_of({"blend": 1000.0, "far": 10.0}, 1e12, "large")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(39.0)
    assert r["frac"] == pytest.approx(39.0 / bench.PEAK_TFLOPS)
    assert r["frac_of_published_fp32"] == pytest.approx(39.0 / 157.3)
    # the committed counters were taken on the current pts_eval.hip
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_blend_large_traffic.json")))
    assert r["traffic"] == pytest.approx(rec["bytes_per_launch"])


def test_stale_traffic_is_not_reported(bench, tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_blend_large_traffic.json")))
    rec["pts_eval_sha256"] = "0" * 64
    f = tmp_path / "stale.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setitem(bench.TRAFFIC_FILES, "large", str(f))
    assert bench.measured_traffic("large") is None
    assert bench.roofline_of({"blend": 1000.0, "far": 10.0}, 1e12, "large")["traffic"] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, GPU_MAX_HW_QUEUES="4"))
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
