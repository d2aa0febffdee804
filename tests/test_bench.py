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
    assert b.measured_traffic(t["n"], t["nb"], t["form"]) == expect
    assert b.measured_traffic(t["n"], 256, t["form"]) is None
    assert b.measured_traffic(1024, t["nb"], t["form"]) is None
    other = "lapack" if t["form"] == "augmented" else "augmented"
    assert b.measured_traffic(t["n"], t["nb"], other) is None


def test_flop_count_is_the_metric_formula():
    b = load_bench()
    for n in (1, 1024, 163840):
        assert b.hpl_flops(n) == 2.0 * n ** 3 / 3.0 + 2.0 * n ** 2


def simulate(b, requested, startup_s, step_s, budget=420.0, timed_budget=100.0):
    """Steps the benchmark's loop would run: (count, seconds since start at the end)."""
    done, timed, est, clock = 0, 0.0, 0.0, startup_s
    while b.may_start_step(done, requested, clock, timed, est, budget, timed_budget):
        clock += step_s + 0.05      # generation + factor + solve
        timed += step_s
        est = step_s + 0.05
        done += 1
    return done, clock + b.RESERVE_S


def test_step_budget_fits_the_driver_command():
    """--steps 20 at about 46 s per full-size step: a bounded number of steps,
    the whole run well inside 600 s even after a slow start."""
    b = load_bench()
    for startup in (20.0, 60.0, 150.0, 300.0):
        for step in (40.0, 46.0, 60.0):
            k, end = simulate(b, 20, startup, step)
            assert k >= 1
            assert end <= 420.0 + step + b.RESERVE_S
            assert end < 560.0
            assert k * step <= 100.0 + step    # the timed work stops near its budget
    assert simulate(b, 20, 40.0, 46.0)[0] == 2
    assert simulate(b, 1, 40.0, 46.0)[0] == 1
    assert simulate(b, 0, 40.0, 46.0)[0] == 0
    # short steps: the requested count is the limit
    assert simulate(b, 20, 10.0, 1.0)[0] == 20


def test_first_step_always_runs_and_later_ones_respect_the_process_budget():
    b = load_bench()
    assert b.may_start_step(0, 5, 10_000.0, 0.0, 0.0, 420.0, 100.0)
    assert not b.may_start_step(1, 5, 380.0, 46.0, 46.0, 420.0, 1000.0)
    assert b.may_start_step(1, 5, 300.0, 46.0, 46.0, 420.0, 1000.0)


def test_projection_is_cubic_through_the_largest_point():
    b = load_bench()
    p = b.project_n3([(1024, 0.2), (4096, 12.8)], [8192, 163840])
    assert p["8192"] == 102.4
    assert abs(p["163840"] - 12.8 * 40.0 ** 3) < 0.1


def test_cpu_baseline_fields_on_tiny_sizes():
    b = load_bench()
    base, x = b.cpu_baseline([64, 128], 2304, 3)
    assert base["kind"] == "oracle" and base["unit"] == "TFLOP/s"
    assert base["cores"] == 3 and base["threads"] == 3
    assert [r["n"] for r in base["serial"]] == [64, 128] == [r["n"] for r in base["parallel"]]
    assert set(base["projection"]["serial_seconds"]) == {"8192", "65536", "163840"}
    assert "PROJECTION" in base["projection"]["note"]
    assert x.shape == (64,)


def test_tuner_table_round_trip(tmp_path):
    """The batched tuner's table writer: the file it writes holds every cost
    of the (systems per CU, variant, bucket) array it was given, in the shape
    the library compiles (host only, no GPU)."""
    import re
    import numpy as np
    from paper_2304_10397_amd import tune_batched
    cost = np.arange(2 * 4 * 16, dtype=np.float64).reshape(2, 4, 16) / 7.0 + 0.5
    out = tmp_path / "table.inc"
    tune_batched.write_table(str(out), cost, "gfx950 (256 CUs)", 4, [4096] * 16)
    text = out.read_text()
    assert "static const int kBatchTableTuned = 1;" in text
    assert "kBatchCostUs[2][4][16]" in text
    body = text[text.index("= {"):]
    vals = np.array([float(v) for v in re.findall(r"-?\d+\.\d+", body)])
    assert vals.size == cost.size
    assert np.allclose(vals, cost.ravel(), atol=5e-5)
