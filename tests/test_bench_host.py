"""Host-side logic of bench.py (no GPU): the one-GPU guard, the committed
rocprofv3 counter summaries the bench line's `traffic` field is read from, and
the roofline object built from them and the live launch time."""
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


def test_headline_traffic_is_used_only_for_the_kernel_source_it_was_taken_on():
    """The bench line carries the committed wave-strip traffic only while the kernel
    source hashes to the value recorded with the counters (else null), and never
    for another grid or launch depth."""
    d = json.load(open(os.path.join(ROOT, "profiles", bench.KERNELS["wave_strip"][1])))
    t = bench._measured_traffic(d["n"], "wave_strip", d["steps_per_launch"])
    if d["kernel_source_sha"] == bench._kernel_sha("wave_strip"):
        assert t == d["traffic_bytes_per_launch_f64"]
    else:
        assert t is None
    assert bench._measured_traffic(d["n"] // 2, "wave_strip", d["steps_per_launch"]) is None
    assert bench._measured_traffic(d["n"], "wave_strip", 3) is None
    # a summary taken at another depth (same name with _k<K>) serves that depth only
    stem, tail = bench.KERNELS["wave_strip"][1].rsplit("_", 1)
    for K in range(2, 9):
        path = os.path.join(ROOT, "profiles", f"{stem}_k{K}_{tail}")
        if K == d["steps_per_launch"] or not os.path.exists(path):
            continue
        dk = json.load(open(path))
        assert dk["steps_per_launch"] == K
        t = bench._measured_traffic(dk["n"], "wave_strip", K)
        if dk["kernel_source_sha"] == bench._kernel_sha("wave_strip"):
            assert t == dk["traffic_bytes_per_launch_f64"]
        else:
            assert t is None


def _form(K, launches, full, ms_launch, n=4096, Kd=None):
    return dict(steps_per_launch=K, launches=launches, full_launches=full,
                ms_per_launch=ms_launch, bytes_per_lu=192, dominant_steps=Kd or K,
                periodic=True)


def test_roofline_of_the_dominant_launch_depth(monkeypatch):
    """20 steps at 8 per launch are 3 launches (7 + 7 + 6); the roofline divides the
    algorithmic bytes (and flops: 7 steps) of one launch of the dominant depth by
    those launches' measured duration."""
    monkeypatch.setattr(bench, "_summary", lambda *a: None)
    r = bench.roofline(_form(8, 3, 2, 0.8, Kd=7), 4096, "wave_strip")
    alg = 4096 * 4096 * 192
    assert r["bytes_per_launch"] == alg and r["steps_per_launch"] == 7
    assert r["hbm"]["achieved"] == pytest.approx(alg / 0.8e-3 / 1e9, rel=1e-4)
    flops = bench.ALG_FLOPS_2D * 4096 * 4096 * 7 / 0.8e-3 / 1e12
    assert r["alu"]["achieved"] == pytest.approx(flops, rel=1e-3)
    assert r["bound"] == "alu" and r["frac"] == r["alu"]["frac"]
    assert r["traffic"] is None and r["valu_busy"] is None


def test_roofline_bound_follows_the_counters(monkeypatch):
    """With SQ counters the bound is the roof the kernel uses more of: VALU issue
    busy fraction against the DRAM bandwidth fraction."""
    def fake(kind, which, n, K, busy=0.4):
        if which == 1:
            return {"traffic_bytes_per_launch_f64": 3.6e9}
        return {"f64": {"valu_busy": busy}}

    monkeypatch.setattr(bench, "_summary", lambda k, w, n, K: fake(k, w, n, K, 0.4))
    r = bench.roofline(_form(8, 250, 250, 0.6), 4096, "wave_strip")
    # 3.6e9 B in 0.6 ms = 6 TB/s = 0.75 of the peak, above 0.4 VALU busy
    assert r["bound"] == "hbm" and r["dram_frac"] == pytest.approx(0.75, rel=1e-4)
    assert r["unit"] == "GB/s" and r["traffic"] == 3.6e9
    monkeypatch.setattr(bench, "_summary", lambda k, w, n, K: fake(k, w, n, K, 0.9))
    r = bench.roofline(_form(8, 250, 250, 0.6), 4096, "wave_strip")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["valu_busy"] == 0.9


def test_roofline_of_fp32_storage_uses_the_fp32_counters(monkeypatch):
    """With only FP32 storage timed (``--storage f32``) the roofline takes the FP32
    kernel's bytes, DRAM traffic and VALU busy fraction, and names the float kernel."""
    def fake(kind, which, n, K):
        if which == 1:
            return {"traffic_bytes_per_launch_f64": 3.6e9,
                    "f32": {"read_bytes": 1.0e9, "write_bytes": 0.8e9}}
        return {"f64": {"valu_busy": 0.7}, "f32": {"valu_busy": 0.85}}

    monkeypatch.setattr(bench, "_summary", fake)
    f = dict(_form(8, 250, 250, 0.5), bytes_per_lu=96)
    r = bench.roofline(f, 4096, "wave_strip", "f32")
    assert r["bytes_per_launch"] == 4096 * 4096 * 96
    assert r["traffic"] == pytest.approx(1.8e9)
    # 1.8e9 B in 0.5 ms = 3.6 TB/s = 0.45 of the peak, below 0.85 VALU busy
    assert r["dram_frac"] == pytest.approx(0.45, rel=1e-4) and r["valu_busy"] == 0.85
    assert r["bound"] == "alu" and "<float, 8>" in r["kernel"]
    r64 = bench.roofline(_form(8, 250, 250, 0.5), 4096, "wave_strip")
    assert r64["traffic"] == 3.6e9 and r64["valu_busy"] == 0.7 and "<double, 8>" in r64["kernel"]


def test_batched_counter_summary_is_self_consistent_and_keyed_to_the_sources():
    """The batched kernels' DRAM summary: bytes = counter x 1024 / copy-probe scale,
    compulsory bytes = every instance's state read and written once per pass (FP32:
    48 B per 2D node, 16 B per 1D node each way); carried only for the current
    batched sources."""
    d = json.load(open(os.path.join(ROOT, "profiles", "k_batch_manifest256_traffic.json")))
    assert d["compulsory_bytes_per_pass"] == 2 * (d["nodes_2d"] * 48 + d["nodes_1d"] * 16)
    probe = d["copy_probe"]
    for name, k in d["kernels"].items():
        assert k["read_bytes"] == pytest.approx(k["FETCH_SIZE_KiB"] * 1024 / probe["fetch_scale"],
                                                rel=1e-4)
        assert k["write_bytes"] == pytest.approx(k["WRITE_SIZE_KiB"] * 1024 / probe["write_scale"],
                                                 rel=1e-4)
        assert k["write_over_alg"] >= 0.95, name
    t = bench._batch_traffic()
    if d["kernel_source_sha"] == bench._sources_sha(bench.BATCH_SOURCES):
        assert set(t["kernels"]) == set(d["kernels"])
    else:
        assert t is None


def test_committed_counter_summaries_match_the_present_sources():
    """The counter summaries bench.py carries (DRAM traffic and SQ issue of the
    default-depth and 7-step wave-strip launches, the one-step kernel and the batched
    kernels) were taken on the kernel sources as they are now; a change to those
    sources needs the summaries retaken, else the bench line loses them."""
    prof = os.path.join(ROOT, "profiles")
    names = {"wave_strip": ["k_step2d_xk_fwd_4096_traffic.json", "k_step2d_xk_fwd_4096_sq.json",
                            "k_step2d_xk_fwd_4096_k7_traffic.json",
                            "k_step2d_xk_fwd_4096_k7_sq.json"],
             "one_step": ["k_step2d_fwd_4096_traffic.json", "k_step2d_fwd_4096_sq.json"]}
    for kind, files in names.items():
        for f in files:
            d = json.load(open(os.path.join(prof, f)))
            assert d["kernel_source_sha"] == bench._kernel_sha(kind), f
    d = json.load(open(os.path.join(prof, "k_batch_manifest256_traffic.json")))
    assert d["kernel_source_sha"] == bench._sources_sha(bench.BATCH_SOURCES)
