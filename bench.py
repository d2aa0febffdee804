#!/usr/bin/env python3
"""HPL benchmark on one MI355X: FP64 LU with partial pivoting + solve.

One step = generate the random system (untimed), then factor + solve (timed):
    HPL TFLOP/s = (2 N^3 / 3 + 2 N^2) / t(factor + solve)
By default the step is HPL's own formulation (Sec. II): b is carried through
the LU as column N of [A | b], each panel's row interchanges reach only the
columns right of it, and x follows from U x = L^-1 P^-1 b by back
substitution (hpl_solve_augmented).  --form lapack times hpl_factor (LAPACK
form: the interchanges applied across all columns) + hpl_solve instead.
The default workload is N = 163840, NB = 512, look-ahead depth 1 (A fills
about 215 GB of HBM), seeded synthetic input.  Prints ONE JSON line on stdout;
progress goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--n 163840] [--nb 512]

One full-size step takes about 46 s, so the number of timed steps is bounded
by wall-clock budgets: at least one step runs; another starts only while the
timed work stays within --timed-budget seconds and the whole process within
--budget seconds (from its start).  The JSON line reports the steps actually
timed and the steps requested.  Warm-up steps (--warmup) are factor + solve
runs at N = 4096: they load the code objects and the workspace, which is all
a full-size warm-up would add.
"""
import time

T_PROCESS_START = time.time()

import argparse  # noqa: E402
import json  # noqa: E402
import os  # noqa: E402
import subprocess  # noqa: E402
import sys  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HPL TFLOP/s (2N³/3+2N²) & % FP64 MFMA peak; MxP+IR speed-up at FP64 residual"
PEAK_FP64_MFMA_TFLOPS = 78.6   # MI355X datasheet, dense FP64 matrix
PEAK_HBM_GBS = 8000.0
PEAK_FP16_MFMA_TFLOPS = 2500.0   # MI355X datasheet, dense FP16/BF16 matrix (no sparsity)
PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X, FP64 vector (256 CUs x 128 flop/clk x 2.4 GHz); FP64 MFMA is rated the same

# HBM bytes per trailing-GEMM launch measured with rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by a 2048 MiB copy: x2.000 and x1.000) at the default
# workload, valid only for the GEMM source with this SHA-256 prefix.
MEASURED_TRAFFIC = {"gemm_sha256_16": "e73c0f582a69228e", "n": 163840, "nb": 512, "form": "augmented",
                    "fetch_gb": 96.24, "write_gb": 35.74}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hpl_flops(n):
    return 2.0 * n ** 3 / 3.0 + 2.0 * n ** 2


def host_description():
    """(CPU model, nproc) of this host."""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        model = [l.split(":", 1)[1].strip() for l in txt.splitlines() if l.startswith("Model name")]
        model = model[0] if model else "unknown"
    except OSError:
        model = "unknown"
    return model, os.cpu_count()


def host_threads():
    """Threads for the parallel oracle: the host share the environment grants
    (OMP_NUM_THREADS when set), else every core."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    return int(v) if v.isdigit() and int(v) > 0 else (os.cpu_count() or 1)


def project_n3(measured, sizes):
    """t proportional to N^3 fitted through the largest measured point (the one
    nearest the projected sizes' out-of-cache regime): {str(N): seconds}."""
    n0, t0 = max(measured, key=lambda r: r[0])
    return {str(n): round(t0 * (n / n0) ** 3, 1) for n in sizes}


def cpu_baseline(sizes, seed, threads):
    """The oracle (plain C: unblocked LU with partial pivoting + substitution) on
    this host: single-threaded, then its threaded form (bitwise the same result)
    on `threads` threads, LU + solve of the same seeded system at each N.
    Returns (baseline dict, oracle x at the smallest N)."""
    import numpy as np
    import oracle
    serial, parallel = [], []
    x_small = None
    used = threads
    for n in sizes:
        b0 = oracle.gen(seed, 1, n, 1)[:, 0].copy()
        for form in ("serial", "parallel"):
            A = oracle.gen(seed, 0, n, n).copy(order="F")
            b = b0.copy()
            t0 = time.perf_counter()
            if form == "serial":
                ipiv, info = oracle.lu(A)
            else:
                ipiv, info, used = oracle.lu_par(A, threads)
            oracle.solve(A, ipiv, b)
            dt = time.perf_counter() - t0
            row = {"n": n, "seconds": round(dt, 4), "tflops": round(hpl_flops(n) / dt / 1e12, 6)}
            (serial if form == "serial" else parallel).append(row)
            if form == "serial" and n == min(sizes):
                x_small = b.copy()
            log(f"oracle {form} N={n}: {dt:.3f} s, {hpl_flops(n) / dt / 1e9:.2f} GFLOP/s")
    model, nproc = host_description()
    top = max(parallel, key=lambda r: r["n"])
    proj = [8192, 65536, 163840]
    out = {
        "value": top["tflops"],
        "unit": "TFLOP/s",
        "cores": used,
        "kind": "oracle",
        "sample": (f"oracle LU + solve of the benchmark's seeded system (seed {seed}) at N = "
                   f"{', '.join(str(n) for n in sizes)}; value = the threaded form at N={top['n']} on "
                   f"{used} threads ({top['seconds']:.2f} s); host CPU: {model}, nproc={nproc}"),
        "host_cpu": model,
        "nproc": nproc,
        "threads": used,
        "serial": serial,
        "parallel": parallel,
        "projection": {
            "note": "PROJECTION, not measured: t proportional to N^3 through the largest measured N",
            "serial_seconds": project_n3([(r["n"], r["seconds"]) for r in serial], proj),
            "parallel_seconds": project_n3([(r["n"], r["seconds"]) for r in parallel], proj),
        },
    }
    return out, x_small


def measured_traffic(n, nb, form):
    """Counter-measured bytes per trailing-GEMM launch, or None if the kernel or workload differs."""
    import hashlib
    src = os.path.join(ROOT, "paper_2304_10397_amd", "csrc", "gemm.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    t = MEASURED_TRAFFIC
    if sha != t["gemm_sha256_16"] or n != t["n"] or nb != t["nb"] or form != t["form"]:
        return None
    return round((t["fetch_gb"] + t["write_gb"]) * 1e9)


GA_REPS = 5


def bench_diffsolve(args, torch, h):
    """Differentiable solve: X = A^{-1} B (forward: factor + solve) and the
    backward (transposed solve + grad_A = -grad_B X^T), A = U[-0.5,0.5) + 8I,
    B uniform, loss = sum(W * X) with W standard normal."""
    n = 8192 if args.n == 163840 else args.n
    nb = 256 if args.nb == 512 else args.nb
    nrhs = 16
    A = h.colmajor(n, n)
    h.hpl_generate(args.seed, 0, A)
    h.hpl_add_diagonal(A, 8.0)
    B = h.colmajor(n, nrhs)
    h.hpl_generate(args.seed, 1, B)
    W = h.colmajor(n, nrhs)
    h.hpl_generate_normal(args.seed, 2, W)
    A.requires_grad_(True)
    B.requires_grad_(True)
    fw, bw, ga = [], [], []
    for step in range(args.warmup + args.steps):
        A.grad = None
        B.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = h.hpl_solve_diff(A, B, nb=nb)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X.backward(W)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # the fused grad_A kernel alone (it rewrites the same A.grad), timed by
        # the library's HIP events enqueued around the launch on its stream
        GB, Xd = B.grad.detach(), X.detach()
        h.hpl_reset_stats()
        h.hpl_set_option(h.HPL_OPT_TIMING, 1)
        for _ in range(GA_REPS):
            h.hpl_solve_grad_a(GB, Xd, A.grad)
        h.hpl_set_option(h.HPL_OPT_TIMING, 0)
        g = h.hpl_get_stats()["grad_a"]
        if step >= args.warmup:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
            ga.append(g["ms"] * 1e-3 / g["launches"])
        log(f"step {step}: forward {1e3 * (t1 - t0):.2f} ms, backward {1e3 * (t2 - t1):.2f} ms")
    k = len(fw)
    t_fw, t_bw, t_ga = sum(fw) / k, sum(bw) / k, sum(ga) / k
    lu_flops = 2.0 * n ** 3 / 3.0
    solve_flops = 2.0 * n * n * nrhs
    ga_bytes = 8.0 * n * n + 16.0 * n * nrhs   # grad_A written once, grad_B and X read
    out = {
        "metric": "differentiable FP64 solve: forward + backward time",
        "value": round(1e3 * (t_fw + t_bw), 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * (t_fw + t_bw), 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"differentiable solve, N={n}, NB={nb}, {nrhs} right-hand sides, A ~ U[-0.5,0.5) + 8I, "
                        f"B ~ U[-0.5,0.5), loss = sum(W*X), W ~ N(0,1), seed {args.seed}",
            "n": n, "nb": nb, "nrhs": nrhs,
            "forward_ms": round(1e3 * t_fw, 3), "backward_ms": round(1e3 * t_bw, 3),
            "forward_tflops": round((lu_flops + solve_flops) / t_fw / 1e12, 3),
        },
        "roofline": {
            "kernel": "grad_a_kernel (grad_A = -grad_B X^T)",
            "bound": "hbm",
            "achieved": round(ga_bytes / t_ga / 1e9, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(ga_bytes / t_ga / 1e9 / PEAK_HBM_GBS, 4),
            "avg_launch_ms": round(1e3 * t_ga, 4),
            "algorithmic_bytes_per_launch": ga_bytes,
            "traffic": None,
        },
    }
    print(json.dumps(out), flush=True)


def bench_mxp(args, torch, h):
    """HPL-MxP: time from the diagonally dominant A (in HBM) to an x that passes
    the FP64 scaled-residual test, mixed precision (FP16 and BF16 LU + FP64
    refinement) against the FP64 path (partial-pivoting LU + solve) on the same
    matrix; speed-up = t_fp64 / t_mxp."""
    n = 65536 if args.n == 163840 else args.n
    nb = args.nb            # FP64 path (its best panel width)
    mnb = args.mxp_nb       # mixed-precision path: FP32 panels of mnb columns, joint updates of 2048
    A = h.colmajor(n, n)
    h.hpl_mxp_generate(args.seed, A)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.hpl_generate(args.seed, 1, b)
    flops = hpl_flops(n)
    res = {}
    # FP64 path on a copy of the same matrix: the benchmark's FP64 method, the
    # augmented [A | b] LU + back substitution (hpl_solve_augmented)
    AB64 = h.colmajor(n, n + 1)
    LU64, x64 = AB64[:, :n], AB64[:, n]
    t64 = []
    for step in range(args.warmup + args.steps):
        LU64.copy_(A)
        x64.copy_(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ipiv, info = h.hpl_solve_augmented(AB64, n, nb)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        log(f"fp64 step {step}: {dt:.3f} s, info={info}")
        if step >= args.warmup:
            t64.append(dt)
    r64 = h.hpl_residual(A, x64.reshape(n, 1), b.reshape(n, 1))
    del LU64, x64, AB64
    torch.cuda.empty_cache()
    t_fp64 = sum(t64) / len(t64)
    LU = h.colmajor32(n, n)
    x = torch.empty_like(b)
    gemm_stats = None
    for fmt, name in ((h.MXP_FP16, "fp16"), (h.MXP_BF16, "bf16")):
        ts = []
        for step in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            timed = step >= args.warmup
            if timed and fmt == h.MXP_FP16:
                h.hpl_reset_stats()
                h.hpl_set_option(h.HPL_OPT_TIMING, 1)
            t0 = time.perf_counter()
            _, info = h.hpl_mxp_factor(A, nb=mnb, fmt=fmt, LU=LU)
            _, out = h.hpl_mxp_solve(A, LU, b, x=x, max_iter=50)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h.hpl_set_option(h.HPL_OPT_TIMING, 0)
            if timed and fmt == h.MXP_FP16:
                gemm_stats = h.hpl_get_stats()
            log(f"{name} step {step}: {dt:.3f} s, {int(out[0])} corrections, scaled residual {out[1]:.3g}, "
                f"info={info}")
            if timed:
                ts.append(dt)
        rr = h.hpl_residual(A, x.reshape(n, 1), b.reshape(n, 1))
        res[name] = {"seconds": round(sum(ts) / len(ts), 4), "corrections": int(out[0]),
                     "scaled_residual": float(rr[0]), "residual_pass": bool(rr[0] < 16.0),
                     "speedup_vs_fp64": round(t_fp64 / (sum(ts) / len(ts)), 3),
                     "effective_tflops": round(flops / (sum(ts) / len(ts)) / 1e12, 2)}
    g = gemm_stats["mxp_gemm"]
    f = gemm_stats["mxp_fact"]
    # the updates' bound: their arithmetic intensity (algorithmic flops per
    # algorithmic byte, over all launches) against the ridge point peak FP16
    # flop/s / peak HBM byte/s = 312.5; the joint updates of two panels (k =
    # 2 NB = 2048: 512 flop/B) are above it, single-panel ones (256) below
    ai = g["flops"] / g["bytes"] if g["bytes"] else 0.0
    ridge = PEAK_FP16_MFMA_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    gbs = g["bytes"] / (g["ms"] * 1e-3) / 1e9 if g["ms"] else None
    tfs = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] else None
    if ai >= ridge:
        rl = {"bound": "mfma", "achieved": round(tfs, 2) if tfs else None, "peak": PEAK_FP16_MFMA_TFLOPS,
              "unit": "TFLOP/s", "frac": round(tfs / PEAK_FP16_MFMA_TFLOPS, 4) if tfs else None}
    else:
        rl = {"bound": "hbm", "achieved": round(gbs, 1) if gbs else None, "peak": PEAK_HBM_GBS,
              "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4) if gbs else None}
    out = {
        "metric": "HPL-MxP: speed-up of FP16 LU + FP64 refinement over the FP64 path, to FP64 residual < 16",
        "value": res["fp16"]["speedup_vs_fp64"],
        "unit": "x",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * res["fp16"]["seconds"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16/bf16 MFMA, fp32 accumulate; fp64 refinement",
        "data": "synthetic",
        "config": {
            "workload": f"HPL-MxP, N={n}, NB={mnb} (FP64 path: augmented [A | b] LU + back substitution, NB={nb}), A ~ U[-0.5,0.5) with "
                        f"a_ii = sum_j |a_ij|, b ~ U[-0.5,0.5), seed {args.seed}",
            "n": n, "nb": mnb, "fp64_nb": nb,
            "fp64_path": {"seconds": round(t_fp64, 4), "tflops": round(flops / t_fp64 / 1e12, 2),
                          "scaled_residual": float(r64[0])},
            "fp16": res["fp16"], "bf16": res["bf16"],
            "fp16_phase_ms": {"trailing_update": round(g["ms"], 2), "panel_u12_convert": round(f["ms"], 2)},
        },
        "roofline": {
            "kernel": "hgemm256_update_kernel (256x128 tiles) and hgemm_update_kernel (128x128, small updates): A22 += (-L21) U12, FP16 MFMA, FP32 C",
            **rl,
            "arithmetic_intensity": round(ai, 1),
            "hbm_gbs": round(gbs, 1) if gbs else None,
            "hbm_frac": round(gbs / PEAK_HBM_GBS, 4) if gbs else None,
            "tflops": round(tfs, 2) if tfs else None,
            "launches": g["launches"],
            "avg_launch_ms": round(g["ms"] / g["launches"], 4) if g["launches"] else None,
            "traffic": None,
        },
    }
    print(json.dumps(out), flush=True)


def bench_batched(args, torch, h):
    """Batched uneven solves: 4096 systems, n ~ U{32..512} (stream 3), A and B uniform,
    4 right-hand sides, W standard normal; one persistent launch for factor + solve
    (the metric) and one for factor + solve + adjoint, against one launch per system
    (timed on every 8th system)."""
    import numpy as np
    count, nrhs = 4096, 4
    sizes = h.hpl_batched_sizes(args.seed, count, 32, 512)
    _, _, na, nb = h.batch_layout(sizes, nrhs)
    A0 = torch.empty(na, dtype=torch.float64, device="cuda")
    B0 = torch.empty(nb, dtype=torch.float64, device="cuda")
    W = torch.empty(nb, dtype=torch.float64, device="cuda")
    h.hpl_generate(args.seed, 0, A0)
    h.hpl_generate(args.seed, 1, B0)
    h.hpl_generate_normal(args.seed, 2, W)
    A, B = torch.empty_like(A0), torch.empty_like(B0)
    GB, GA = torch.empty_like(B0), torch.empty_like(A0)
    ipiv = torch.empty(int(np.sum(sizes)), dtype=torch.int32, device="cuda")
    n3 = sizes.astype(np.float64)
    f_fwd = float(np.sum(2.0 * n3 ** 3 / 3.0 + 2.0 * n3 ** 2 * nrhs))

    def run(mode, reps, label):
        wall, dev = [], []
        for step in range(args.warmup + reps):
            A.copy_(A0)
            B.copy_(B0)
            torch.cuda.synchronize()
            h.hpl_reset_stats()
            h.hpl_set_option(h.HPL_OPT_TIMING, 1)
            t0 = time.perf_counter()
            info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, W=W, GB=GB, GA=GA, mode=mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h.hpl_set_option(h.HPL_OPT_TIMING, 0)
            st = h.hpl_get_stats()["batched"]
            if int(np.count_nonzero(info)):
                raise RuntimeError(f"{label}: singular system in the batch")
            log(f"{label} step {step}: {1e3 * dt:.3f} ms wall, kernel {st['ms']:.3f} ms")
            if step >= args.warmup:
                wall.append(dt)
                dev.append(st["ms"] * 1e-3)
        return sum(wall) / len(wall), sum(dev) / len(dev)

    t_fwd, k_fwd = run(h.BATCH_FORWARD, args.steps, "factor+solve")
    t_both, k_both = run(h.BATCH_BOTH, args.steps, "factor+solve+adjoint")
    # one launch per system, every 8th system of the batch
    sample = np.arange(0, count, 8)
    _, voff_all, _, _ = h.batch_layout(sizes, nrhs)
    aoff_all = h.batch_layout(sizes, nrhs)[0]
    A.copy_(A0)
    B.copy_(B0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in sample:
        n = int(sizes[i])
        a0, v0 = int(aoff_all[i]), int(voff_all[i])
        h.hpl_batched_solve(sizes[i:i + 1], A[a0:a0 + n * n], ipiv[v0:v0 + n], B[nrhs * v0:nrhs * v0 + n * nrhs],
                            nrhs, mode=h.BATCH_FORWARD)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    loop_rate = sample.size / t_loop
    out = {
        "metric": "batched uneven FP64 solves (LU with partial pivoting + solve), one persistent launch",
        "value": round(count / t_fwd, 1),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_fwd, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{count} systems, n ~ U{{32..512}} (seed {args.seed}, stream 3), A_i, B_i ~ U[-0.5,0.5), "
                        f"{nrhs} right-hand sides, W ~ N(0,1) for the adjoint",
            "systems": count, "nrhs": nrhs, "sum_n": int(np.sum(sizes)),
            "factor_solve_tflops": round(f_fwd / t_fwd / 1e12, 3),
            "factor_solve_adjoint_ms": round(1e3 * t_both, 3),
            "factor_solve_adjoint_systems_per_s": round(count / t_both, 1),
            "adjoint_ms": round(1e3 * (t_both - t_fwd), 3),
            "per_system_launch_loop_systems_per_s": round(loop_rate, 1),
            "speedup_vs_per_system_loop": round((count / t_fwd) / loop_rate, 2),
            "per_system_loop_sample": f"every 8th system ({sample.size} launches, sizes as in the batch)",
        },
        "roofline": {
            "kernel": "batched_solve_kernel (factor + solve; trailing updates on the FP64 matrix cores, "
                      "panels and solves on the VALU, both rated 78.6 TFLOP/s)",
            "bound": "mfma",
            "achieved": round(f_fwd / k_fwd / 1e12, 3),
            "peak": PEAK_FP64_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(f_fwd / k_fwd / 1e12 / PEAK_FP64_VALU_TFLOPS, 4),
            "avg_launch_ms": round(1e3 * k_fwd, 4),
            "algorithmic_flops_per_launch": f_fwd,
            "traffic": None,
        },
    }
    print(json.dumps(out), flush=True)


def bench_hostpanel(args, torch, h):
    """The paper's host FACT (T threads over NB-row tiles) against the GPU panel:
    (1) FACT of an M x 512 panel for M = 512 .. 32768 (the tail of a run has the
    small M); (2) factor + solve at N = 32768, NB = 512, once with each FACT,
    the host one overlapping the trailing update as in the paper."""
    import numpy as np
    nb = 512
    threads = [1, 4, 16]
    Ms = [512, 1024, 2048, 4096, 8192, 16384, 32768]
    rows = []
    last = {}
    for M in Ms:
        G = h.colmajor(M, nb)
        h.hpl_generate(args.seed, 0, G)
        P0 = np.asfortranarray(G.cpu().numpy())
        flops = M * nb * nb - nb ** 3 / 3.0
        row = {"M": M}
        for T in threads:
            if T in last and last[T] * 2.2 > 5.0:   # keep the host part of the run short
                row[f"host_T{T}_gflops"] = None
                continue
            P = P0.copy(order="F")
            t0 = time.perf_counter()
            h.hpl_host_panel(P, T)
            dt = time.perf_counter() - t0
            last[T] = dt
            row[f"host_T{T}_gflops"] = round(flops / dt / 1e9, 2)
        best = 1e30
        for _ in range(3):
            A = G.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.hpl_panel_factor(A)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        row["gpu_gflops"] = round(flops / best / 1e9, 2)
        rows.append(row)
        log(f"FACT M={M}: {row}")
    n = 32768
    runs = {}
    for label, T in (("gpu_panel", 0), ("host_panel_T16", 16)):
        h.hpl_set_option(h.HPL_OPT_HOST_PANEL, T)
        A = h.colmajor(n, n)
        h.hpl_generate(args.seed, 0, A)
        b = h.colmajor(n, 1)
        h.hpl_generate(args.seed, 1, b)
        torch.cuda.synchronize()
        h.hpl_reset_stats()
        h.hpl_set_option(h.HPL_OPT_TIMING, 1)
        t0 = time.perf_counter()
        ipiv, info = h.hpl_factor(A, nb)
        h.hpl_solve(A, ipiv, b)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h.hpl_set_option(h.HPL_OPT_TIMING, 0)
        st = h.hpl_get_stats()
        A0 = h.colmajor(n, n)
        h.hpl_generate(args.seed, 0, A0)
        b0 = h.colmajor(n, 1)
        h.hpl_generate(args.seed, 1, b0)
        res = h.hpl_residual(A0, b, b0)
        del A0, A
        runs[label] = {"seconds": round(dt, 4), "tflops": round(hpl_flops(n) / dt / 1e12, 3),
                       "fact_ms_total": round(st["panel"]["ms"], 2), "fact_launches": st["panel"]["launches"],
                       "gemm_ms": round(st["gemm"]["ms"], 2), "scaled_residual": float(res[0]), "info": int(info)}
        log(f"{label}: {runs[label]}")
    h.hpl_set_option(h.HPL_OPT_HOST_PANEL, 0)
    g = runs["host_panel_T16"]
    out = {
        "metric": "HPL with the paper's host FACT (16 threads, NB-row tiles): TFLOP/s at N=32768, against the GPU panel",
        "value": g["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(1e3 * g["seconds"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"HPL FP64 LU+solve, N={n}, NB={nb}, look-ahead 1, A,b ~ U[-0.5,0.5) seed {args.seed}; "
                        "FACT of M x 512 panels on the host (T threads) and on the GPU",
            "n": n, "nb": nb, "runs": runs, "fact_gflops_by_M": rows,
            "host_threads_note": "the host FACT runs on the box's CPU share (16 cores)",
        },
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


# The small configuration timed next to the oracle (N = 1024, NB = 64): median
# of CONFIG1_RUNS factor + solve runs after CONFIG1_WARM warm-ups.
CONFIG1_N, CONFIG1_NB, CONFIG1_RUNS, CONFIG1_WARM = 1024, 64, 20, 3
RESERVE_S = 15.0   # after the last step: residual, statistics, JSON


def may_start_step(done, requested, elapsed_s, timed_s, est_step_s, budget_s, timed_budget_s,
                   reserve_s=RESERVE_S):
    """Whether another full-size step may start.  The first always does (when
    one was requested); a later one only if, at the last step's duration, the
    timed work stays within timed_budget_s and the process, with reserve_s
    left for the residual and the report, within budget_s."""
    if done >= requested:
        return False
    if done == 0:
        return True
    if timed_s + est_step_s > timed_budget_s:
        return False
    return elapsed_s + est_step_s + reserve_s <= budget_s


def config1_run(torch, h, seed, x_oracle):
    """Factor + solve at N = 1024, NB = 64 on the GPU: median time, TFLOP/s,
    scaled residual, and x against the oracle's x of the same system."""
    import numpy as np
    n, nb = CONFIG1_N, CONFIG1_NB
    A0 = h.colmajor(n, n)
    h.hpl_generate(seed, 0, A0)
    b0 = h.colmajor(n, 1)
    h.hpl_generate(seed, 1, b0)
    A, x = torch.empty_like(A0), torch.empty_like(b0)
    ts = []
    for r in range(CONFIG1_WARM + CONFIG1_RUNS):
        A.copy_(A0)
        x.copy_(b0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ipiv, info = h.hpl_factor(A, nb)
        h.hpl_solve(A, ipiv, x)
        torch.cuda.synchronize()
        if r >= CONFIG1_WARM:
            ts.append(time.perf_counter() - t0)
    res = h.hpl_residual(A0, x, b0)
    med = float(np.median(ts))
    out = {"n": n, "nb": nb, "runs": CONFIG1_RUNS, "gpu_median_s": round(med, 6),
           "gpu_tflops": round(hpl_flops(n) / med / 1e12, 4), "scaled_residual": float(res[0])}
    if x_oracle is not None:
        xg = x.cpu().numpy()[:, 0]
        out["x_rel_err_vs_oracle"] = float(np.max(np.abs(xg - x_oracle)) / np.max(np.abs(x_oracle)))
    return out


def bench_hpl(args, torch, h, dev):
    n, nb = args.n, args.nb
    log(f"device {torch.cuda.get_device_name(dev)}; N={n} NB={nb} look-ahead={args.lookahead}")
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, args.lookahead)
    if args.laswp_wgs is not None:
        h.hpl_set_option(h.HPL_OPT_LASWP_WGS, args.laswp_wgs)

    # Warm-up (not timed): factor + solve at N = 4096 loads the code objects and
    # the workspace; a full-size warm-up would add nothing else.
    for _ in range(max(1, args.warmup)):
        A_s = h.colmajor(4096, 4097)
        h.hpl_generate(1, 0, A_s)
        if args.form == "augmented":
            h.hpl_solve_augmented(A_s, 4096, nb)
        else:
            piv_s, _ = h.hpl_factor(A_s[:, :4096], nb)
            h.hpl_solve(A_s[:, :4096], piv_s, A_s[:, 4096:])
        del A_s
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    peak_measured, _ = h.hpl_mfma_peak(200000)
    log(f"measured FP64 MFMA peak (pure 16x16x4 loop): {peak_measured:.2f} TFLOP/s")

    # CPU baseline (the oracle on this host's cores) and the small configuration
    # next to it, before the full-size matrix takes the GPU memory.
    base, x_small = None, None
    if args.cpu_sample > 0:
        sizes = [m for m in (1024, 2048, 4096, 8192) if m <= args.cpu_sample] or [args.cpu_sample]
        log(f"oracle CPU baseline at N = {sizes} ...")
        base, x_small = cpu_baseline(sizes, args.seed, host_threads())
    cfg1 = config1_run(torch, h, args.seed, x_small if base and base["serial"][0]["n"] == CONFIG1_N else None)
    log(f"N={CONFIG1_N} NB={CONFIG1_NB}: {cfg1}")
    if base is not None:
        s1 = base["serial"][0]
        p1 = base["parallel"][0]
        cfg1["oracle_serial_s"] = s1["seconds"]
        cfg1["oracle_threaded_s"] = p1["seconds"]
        cfg1["gpu_speedup_vs_oracle_serial"] = round(s1["seconds"] / cfg1["gpu_median_s"], 1)
        base["config_n1024_nb64"] = cfg1

    augmented = args.form == "augmented"
    if augmented:
        # [A | b] in one allocation: b is column n, carried through the factorization
        AB = h.colmajor(n, n + 1, ld=n + args.pad)
        A, x = AB[:, :n], AB[:, n:]
    else:
        A = h.colmajor(n, n, ld=n + args.pad)
        x = h.colmajor(n, 1)
    b = h.colmajor(n, 1)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    log(f"allocated A: {A.stride(1) * n * 8 / 1e9:.1f} GB ({args.form} form)")

    times = []
    info = 0
    est = 0.0
    h.hpl_set_option(h.HPL_OPT_PROGRESS, args.progress)
    while may_start_step(len(times), args.steps, time.time() - T_PROCESS_START, sum(times), est,
                         args.budget, args.timed_budget):
        step = len(times)
        t_gen = time.perf_counter()
        h.hpl_generate(args.seed, 0, A)
        h.hpl_generate(args.seed, 1, b)
        x.copy_(b)
        torch.cuda.synchronize()
        h.hpl_reset_stats()
        h.hpl_set_option(h.HPL_OPT_TIMING, 1)
        t0 = time.perf_counter()
        if augmented:
            _, info = h.hpl_solve_augmented(AB, n, nb, ipiv=ipiv)
        else:
            _, info = h.hpl_factor(A, nb, ipiv=ipiv)
            h.hpl_solve(A, ipiv, x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h.hpl_set_option(h.HPL_OPT_TIMING, 0)
        times.append(dt)
        est = time.perf_counter() - t_gen   # generation + factor + solve
        log(f"step {step} (timed): {dt:.3f} s, {hpl_flops(n) / dt / 1e12:.2f} TFLOP/s, info={info}; "
            f"{time.time() - T_PROCESS_START:.0f} s since start")
    h.hpl_set_option(h.HPL_OPT_PROGRESS, 0)
    stats = h.hpl_get_stats()  # last timed step

    res = h.hpl_residual_gen(args.seed, n, x, b)
    log(f"scaled residual {res[0]:.4g} ({'PASS' if res[0] < 16 else 'FAIL'})")

    total = sum(times)
    tflops = hpl_flops(n) * len(times) / total / 1e12
    g = stats["gemm"]
    gemm_tflops = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else None
    phases = {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in stats.items()}
    out = {
        "metric": METRIC,
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": len(times),
        "steps_requested": args.steps,
        "warmup": args.warmup,
        "warmup_note": "warm-up steps are the same factor + solve at N = 4096 (code objects, workspace)",
        "ms_per_step": round(1e3 * total / len(times), 3),
        "step_seconds": [round(t, 3) for t in times],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "pct_fp64_mfma_peak": round(100.0 * tflops / PEAK_FP64_MFMA_TFLOPS, 2),
        "fp64_mfma_peak_measured": round(peak_measured, 3),
        "pct_measured_fp64_mfma_peak": round(100.0 * tflops / peak_measured, 2) if peak_measured > 0 else None,
        "config": {
            "workload": f"HPL FP64 LU+solve, N={n}, NB={nb}, look-ahead {args.lookahead}, "
                        f"A,b ~ U[-0.5,0.5) seed {args.seed}",
            "n": n, "nb": nb, "lda": n + args.pad, "lookahead": args.lookahead,
            "form": ("augmented [A | b]: LU with b carried as column N, row swaps right of each panel only, "
                     "then back substitution (hpl_solve_augmented)" if augmented else
                     "LAPACK: hpl_factor (swaps across all columns) + hpl_solve"),
            "interchange_workgroups": h.hpl_get_option(h.HPL_OPT_LASWP_WGS), "seed": args.seed,
            "scaled_residual": float(res[0]), "residual_pass": bool(res[0] < 16.0), "info": info,
            "budget_s": args.budget, "timed_budget_s": args.timed_budget,
            "phase_ms_last_step": phases,
        },
        "roofline": {
            "kernel": "gemm_stream_kernel (trailing-update DGEMM, FP64 MFMA 16x16x4)",
            "bound": "mfma",
            "achieved": round(gemm_tflops, 3) if gemm_tflops else None,
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(gemm_tflops / PEAK_FP64_MFMA_TFLOPS, 4) if gemm_tflops else None,
            "launches": g["launches"],
            "avg_launch_ms": round(g["ms"] / g["launches"], 4) if g["launches"] else None,
            "avg_launch_gflop": round(g["flops"] / g["launches"] / 1e9, 3) if g["launches"] else None,
            "traffic": measured_traffic(n, nb, args.form),
            "traffic_unit": "bytes per launch (L2-miss fetch + write, rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated; includes MALL hits)",
            "algorithmic_bytes_per_launch": round(g["bytes"] / g["launches"]) if g["launches"] else None,
        },
    }
    if base is not None:
        out["cpu_baseline"] = base
    else:
        out["config_n1024_nb64"] = cfg1
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="full-size steps requested (hpl: bounded by --timed-budget and --budget)")
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed warm-up steps (hpl: factor + solve at N = 4096)")
    ap.add_argument("--timed-budget", type=float, default=100.0,
                    help="hpl: seconds of timed full-size work after which no further step starts")
    ap.add_argument("--budget", type=float, default=420.0,
                    help="hpl: seconds from process start after which no further step starts")
    ap.add_argument("--n", type=int, default=163840)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--mxp-nb", type=int, default=256,
                    help="panel width of the mixed-precision LU (--workload mxp); panels are grouped 2048 columns "
                         "at a time for the joint trailing update")
    ap.add_argument("--lookahead", type=int, default=1)
    ap.add_argument("--laswp-wgs", type=int, default=None,
                    help="hpl: workgroups of the trailing interchanges (HPL_OPT_LASWP_WGS; default: the library's)")
    ap.add_argument("--form", choices=["augmented", "lapack"], default="augmented",
                    help="hpl: augmented = the HPL formulation (b carried through the LU as column N, "
                         "row swaps only right of each panel, then U x = b'); lapack = hpl_factor + hpl_solve")
    ap.add_argument("--seed", type=int, default=2304)
    ap.add_argument("--pad", type=int, default=0, help="lda = n + pad")
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="largest N of the oracle timings (N = 1024, 2048, ... up to it; 0: skip)")
    ap.add_argument("--progress", type=int, default=32, help="progress line every k panels (stderr)")
    ap.add_argument("--workload", choices=["hpl", "diffsolve", "mxp", "batched", "hostpanel"], default="hpl",
                    help="hpl: the HPL factor + solve (default); diffsolve: the differentiable FP64 "
                         "solve, N=8192 NB=256 16 right-hand sides, forward + backward; mxp: mixed-precision "
                         "LU + FP64 refinement at N=65536 against the FP64 path on the same matrix")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (reference for the HBM byte "
                         "counters FETCH_SIZE / WRITE_SIZE) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2304_10397_amd.hpl as h

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nbytes} bytes ({nbytes >> 10} KiB read + written each)")
        return
    if args.workload == "diffsolve":
        return bench_diffsolve(args, torch, h)
    if args.workload == "mxp":
        return bench_mxp(args, torch, h)
    if args.workload == "batched":
        return bench_batched(args, torch, h)
    if args.workload == "hostpanel":
        return bench_hostpanel(args, torch, h)
    return bench_hpl(args, torch, h, dev)

if __name__ == "__main__":
    main()
