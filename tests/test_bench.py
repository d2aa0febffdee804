"""Host-side logic of bench.py (CPU only): the one-GPU refusal, the gate on the
counter-measured GEMM traffic, and the metric's flop count."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_reported_only_for_the_measured_kernel_and_workload():
    b = load_bench()
    with open(os.path.join(ROOT, "paper_2304_10397_amd", "csrc", "gemm.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    t = b.MEASURED_TRAFFIC
    expect = round((t["fetch_gb"] + t["write_gb"]) * 1e9) if sha == t["gemm_sha256_16"] else None
    assert b.measured_traffic(t["n"], t["nb"]) == expect
    assert b.measured_traffic(t["n"], 256) is None
    assert b.measured_traffic(1024, t["nb"]) is None


def test_flop_count_is_the_metric_formula():
    b = load_bench()
    for n in (1, 1024, 163840):
        assert b.hpl_flops(n) == 2.0 * n ** 3 / 3.0 + 2.0 * n ** 2
