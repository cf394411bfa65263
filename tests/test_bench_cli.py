"""The benchmark script's command line on the host (no GPU needed).

bench.py measures one GPU: any other --gpus value exits with status 2 and a
message before touching a device; the roofline's traffic figure is read from
the committed counter summary only while its kernel-source hash matches.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=60)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workloads_listed():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("zgemm", "batch", "batch-auto", "learned-n", "vendor-int8", "vendor-complex"):
        assert w in r.stdout


def test_traffic_follows_the_kernel_source_hash(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    key = "ZGEMM 16384x16384x16384 N=14 fast karatsuba"
    with open(os.path.join(ROOT, "profiles", "residue_gemm_traffic.json")) as f:
        entry = json.load(f)[key]
    got = bench.traffic_from_profiles(key)
    if entry["gemm_source_sha"] == bench.gemm_source_hash():
        assert got == entry["hbm_bytes_per_launch"]
    else:
        assert got is None
    monkeypatch.setattr(bench, "gemm_source_hash", lambda: "0" * 16)
    assert bench.traffic_from_profiles(key) is None
    assert bench.traffic_from_profiles("no such workload") is None


def test_performance_model_reproduces_the_worked_example():
    """Section III-C: with 2-4 TB/s of bandwidth and 1500 TOPS of INT8 throughput the
    model puts accurate-mode ZGEMM at m = n = k = 16384 (13 moduli, c = 13) near
    120 TFLOPS."""
    sys.path.insert(0, ROOT)
    import bench

    s = 16384
    tflops = {b: 8.0 * s ** 3 / bench.paper_model_seconds(s, s, s, 13, "accurate", b=b * 1e12,
                                                          p=1.5e15) / 1e12
              for b in (2, 3, 4)}
    assert 110 < tflops[2] < tflops[3] < tflops[4] < 130
    assert abs(tflops[3] - 120) < 5
    # the compute-bound limit: 8 mnk flops against 6 (N + 1) mnk INT8 operations
    limit = 8.0 * 1.5e15 / (6 * 14) / 1e12
    assert tflops[4] < limit
    assert abs(8.0 * s ** 3 / bench.paper_model_seconds(s, s, s, 13, "accurate", b=1e30,
                                                        p=1.5e15) / 1e12 - limit) < 1e-9


def test_performance_model_orders_the_variants():
    """Accurate mode costs one more product and more traffic than fast mode; single
    precision moves fewer bytes than double; the memory terms shrink relative to the
    products as k grows."""
    sys.path.insert(0, ROOT)
    import bench

    s, N = 8192, 13
    t = {(mode, single): bench.paper_model_seconds(s, s, s, N, mode, single, b=3e12, p=1.5e15)
         for mode in ("fast", "accurate") for single in (False, True)}
    assert t[("accurate", False)] > t[("fast", False)]
    assert t[("accurate", True)] > t[("fast", True)]
    assert t[("fast", True)] < t[("fast", False)]
    assert t[("accurate", True)] < t[("accurate", False)]
    # fast mode, double: steps 1-3 of the model summed by hand for m = n = k = 1, N = 1, c = 0
    assert bench.paper_model_seconds(1, 1, 1, 1, "fast", b=1.0, p=1e300, c=0) == (35 + 4) * 2 + 32
    share = [bench.paper_model_seconds(s, s, kk, N, b=3e12, p=1.5e15) / (6.0 * N * s * s * kk / 1.5e15)
             for kk in (1024, 16384, 262144)]
    assert share[0] > share[1] > share[2] > 1.0


def test_phase_rates_count_the_algorithmic_bytes():
    """Split: 16 B read and 3N B written per complex element of both operands; reconstruction:
    2N B of E' read and 16 B written per output; scans: both operands read twice."""
    sys.path.insert(0, ROOT)
    import bench

    prof = {"calls": 2, "scale_ms": 2.0, "split_ms": 4.0, "crt_ms": 6.0}
    r = bench.phase_rates(1000, 2000, 3000, 14, False, "karatsuba", "fast", prof)
    assert r["split"] == round((3000 * 3000 * (16 + 42)) / 2e-3 / 1e12, 3)
    assert r["crt"] == round(1000 * 2000 * (28 + 16) / 3e-3 / 1e12, 3)
    assert r["scale"] == round(2 * 3000 * 3000 * 16 / 1e-3 / 1e12, 3)
    single = bench.phase_rates(1000, 2000, 3000, 6, True, "4m", "accurate", prof)
    assert "scale" not in single
    assert single["split"] == round((3000 * 3000 * (8 + 12)) / 2e-3 / 1e12, 3)
