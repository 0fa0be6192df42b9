"""Host-side logic of bench.py (no GPU): the one-GPU guard, and the committed
rocprofv3 counter summaries the bench line's `traffic` field is read from."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    """`--gpus N` with N > 1 exits with status 2 and one JSON line that says so,
    before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("kind", sorted(bench.KERNELS))
def test_counter_summary_is_self_consistent(kind):
    """Each committed summary: read bytes = FETCH_SIZE x 1024 / copy-probe scale,
    write bytes likewise, and the traffic per launch is their sum (FP64)."""
    path = os.path.join(ROOT, "profiles", bench.KERNELS[kind][1])
    d = json.load(open(path))
    probe = d["copy_probe"]
    kib = probe["bytes"] / 1024
    assert probe["fetch_scale"] == pytest.approx(probe["FETCH_SIZE_KiB"] / kib, rel=1e-4)
    assert probe["write_scale"] == pytest.approx(probe["WRITE_SIZE_KiB"] / kib, rel=1e-4)
    f64 = d["f64"]
    rb = f64["FETCH_SIZE_KiB"] * 1024 / probe["fetch_scale"]
    wb = f64["WRITE_SIZE_KiB"] * 1024 / probe["write_scale"]
    assert f64["read_bytes"] == pytest.approx(rb, rel=1e-4)
    assert f64["write_bytes"] == pytest.approx(wb, rel=1e-4)
    assert d["traffic_bytes_per_launch_f64"] == pytest.approx(rb + wb, rel=1e-4)
    # algorithmic bytes of one FP64 launch: 12 populations x 8 B read and written per node
    assert f64["algorithmic_bytes"] == d["n"] ** 2 * 12 * 8 * 2
    assert f64["write_over_alg"] >= 0.99 and f64["read_over_alg"] >= 0.99


def test_headline_traffic_matches_the_current_kernel_source():
    """The wave-strip summary was taken on the kernel source as committed, so the
    bench line carries its traffic; another grid or launch depth gets none."""
    d = json.load(open(os.path.join(ROOT, "profiles", bench.KERNELS["wave_strip"][1])))
    assert d["kernel_source_sha"] == bench._kernel_sha("wave_strip")
    t = bench._measured_traffic(d["n"], "wave_strip", d["steps_per_launch"])
    assert t == d["traffic_bytes_per_launch_f64"]
    assert bench._measured_traffic(d["n"] // 2, "wave_strip", d["steps_per_launch"]) is None
    assert bench._measured_traffic(d["n"], "wave_strip", d["steps_per_launch"] - 1) is None
