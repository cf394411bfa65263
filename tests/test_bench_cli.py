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
