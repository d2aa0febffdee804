"""Offline tuner of hpl_batched_solve's schedule.

    python -m paper_2304_10397_amd.tune_batched [--out PATH] [--nrhs 4]

For every number of systems in flight per CU (occ = 1, 2), every variant of
the per-system factorization (HPL_BATCH_VARIANTS: panel width and U12 stage
width) and every size bucket (n - 1) / 32 of n = 1..512, it times one
persistent launch (factor + solve) of a batch of systems whose sizes are
uniform in the bucket, with that schedule forced through HPL_OPT_BATCH_CONFIG,
and records the kernel time per system, amortized over the device, in
microseconds (the fastest of --reps launches, from the library's HIP events).
The table is written as csrc/batched_tuned.inc (by default); rebuilding the
library makes hpl_batched_solve choose from it (hpl_batched_config).

The systems are the benchmark's kind (entries uniform in [-0.5, 0.5), seeded);
every launch must report info = 0 for all systems.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "csrc", "batched_tuned.inc")


def batch_for_bucket(h, torch, q, count, nrhs, seed):
    lo, hi = 32 * q + 1, 32 * q + 32
    sizes = h.hpl_batched_sizes(seed + q, count, lo, hi)
    _, _, na, nb = h.batch_layout(sizes, nrhs)
    A0 = torch.empty(na, dtype=torch.float64, device="cuda")
    B0 = torch.empty(nb, dtype=torch.float64, device="cuda")
    h.hpl_generate(seed, 0, A0)
    h.hpl_generate(seed, 1, B0)
    return sizes, A0, B0


def measure(h, torch, sizes, A0, B0, nrhs, config, reps):
    A, B = torch.empty_like(A0), torch.empty_like(B0)
    ipiv = torch.empty(int(np.sum(sizes)), dtype=torch.int32, device="cuda")
    h.hpl_set_option(h.HPL_OPT_BATCH_CONFIG, config)
    best = float("inf")
    try:
        for _ in range(reps + 1):   # the first launch is a warm-up
            A.copy_(A0)
            B.copy_(B0)
            torch.cuda.synchronize()
            h.hpl_reset_stats()
            h.hpl_set_option(h.HPL_OPT_TIMING, 1)
            info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, mode=h.BATCH_FORWARD)
            h.hpl_set_option(h.HPL_OPT_TIMING, 0)
            if np.count_nonzero(info):
                raise RuntimeError("singular system in a tuning batch")
            best = min(best, h.hpl_get_stats()["batched"]["ms"])
    finally:
        h.hpl_set_option(h.HPL_OPT_TIMING, 0)
        h.hpl_set_option(h.HPL_OPT_BATCH_CONFIG, 0)
    return best


def write_table(path, cost, device, nrhs, counts):
    """cost[occ-1][v][q] in microseconds per system."""
    lines = [
        "// Tuned schedule table of hpl_batched_solve: microseconds per system (amortized",
        "// over the device) of every (systems per CU, variant, size bucket), indexed",
        "// [occ - 1][variant][(n - 1) / 32].  Written by",
        "// paper_2304_10397_amd/tune_batched.py -- do not edit by hand.",
        f"// device: {device}; {nrhs} right-hand sides; systems per measurement by bucket: "
        + ", ".join(str(c) for c in counts),
        "static const int kBatchTableTuned = 1;",
        f"static const double kBatchCostUs[2][{cost.shape[1]}][{cost.shape[2]}] = {{",
    ]
    for o in range(cost.shape[0]):
        lines.append("    {")
        for v in range(cost.shape[1]):
            vals = ", ".join(f"{x:.4f}" for x in cost[o, v])
            lines.append(f"        {{{vals}}},")
        lines.append("    },")
    lines.append("};")
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=2304)
    args = ap.parse_args()

    import torch
    import importlib
    h = importlib.import_module(__package__ + ".hpl")

    torch.cuda.set_device(0)
    variants, buckets = h.HPL_BATCH_VARIANTS, h.HPL_BATCH_BUCKETS
    cost = np.zeros((2, variants, buckets))
    counts = []
    t0 = time.time()
    for q in range(buckets):
        # enough systems to fill every workgroup slot (2 per CU) several times,
        # fewer for the large buckets to bound the time
        count = 4096 if q < 4 else (2048 if q < 10 else 1536)
        counts.append(count)
        sizes, A0, B0 = batch_for_bucket(h, torch, q, count, args.nrhs, args.seed)
        for o in (1, 2):
            for v in range(variants):
                ms = measure(h, torch, sizes, A0, B0, args.nrhs, 1 + (o - 1) * variants + v, args.reps)
                cost[o - 1, v, q] = 1e3 * ms / count
        best = np.unravel_index(np.argmin(cost[:, :, q]), cost[:, :, q].shape)
        print(f"[tune] bucket {q} (n {32 * q + 1}..{32 * q + 32}, {count} systems): "
              f"occ1 {np.round(cost[0, :, q], 3).tolist()} occ2 {np.round(cost[1, :, q], 3).tolist()} "
              f"us/system; best occ {best[0] + 1} variant {best[1]}; {time.time() - t0:.0f} s",
              file=sys.stderr, flush=True)
        del A0, B0
        torch.cuda.empty_cache()
    props = torch.cuda.get_device_properties(0)
    write_table(args.out, cost, f"{props.gcnArchName} ({props.multi_processor_count} CUs)", args.nrhs, counts)
    print(f"[tune] wrote {args.out}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
