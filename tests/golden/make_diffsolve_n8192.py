"""Writes tests/golden/diffsolve_n8192_oracle.txt: the oracle's X = A^{-1} B,
grad_B = A^{-T} W and grad_A = -grad_B X^T for the differentiable-solve
workload at its full size (N = 8192, 16 right-hand sides, A = U[-0.5, 0.5)
+ 8 I from stream 0, B from stream 1, W standard normal from stream 2, seed
2304), reduced to what a GPU test can compare against cheaply: the largest
magnitudes, the column sums and absolute column sums of X and grad_B, and
entries of X, grad_B and grad_A at seeded sample positions.

Calls only oracle/ (the factorization on host threads: bitwise the serial
oracle's factors).   python tests/golden/make_diffsolve_n8192.py [threads]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

N, NRHS, SEED, SHIFT = 8192, 16, 2304, 8.0
N_X, N_GB, N_GA = 256, 256, 64
OUT = os.path.join(HERE, "diffsolve_n8192_oracle.txt")


def sample_positions():
    """Seeded sample positions (independent of every value): rows/columns of X,
    of grad_B, and (row, column) pairs of grad_A."""
    rng = np.random.default_rng(81920)
    px = np.stack([rng.integers(0, N, N_X), rng.integers(0, NRHS, N_X)], axis=1)
    pb = np.stack([rng.integers(0, N, N_GB), rng.integers(0, NRHS, N_GB)], axis=1)
    pa = np.stack([rng.integers(0, N, N_GA), rng.integers(0, N, N_GA)], axis=1)
    return px, pb, pa


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    A = oracle.gen(SEED, 0, N, N).copy(order="F")
    A[np.arange(N), np.arange(N)] += SHIFT
    B = oracle.gen(SEED, 1, N, NRHS).copy(order="F")
    W = oracle.gen_normal(SEED, 2, N, NRHS).copy(order="F")
    X, GB, GA, info = oracle.solve_grad(A, B, W, threads=threads)
    assert info == 0
    px, pb, pa = sample_positions()
    lines = [
        "# oracle X = A^-1 B, grad_B = A^-T W, grad_A = -grad_B X^T; N=8192, 16 right-hand sides,",
        "# A = U[-0.5,0.5) (stream 0) + 8 I, B stream 1, W standard normal stream 2, seed 2304",
        "# written by tests/golden/make_diffsolve_n8192.py (oracle only)",
        f"maxabs X {float(np.max(np.abs(X))).hex()}",
        f"maxabs GB {float(np.max(np.abs(GB))).hex()}",
        f"maxabs GA {float(np.max(np.abs(GA))).hex()}",
    ]
    for name, M in (("X", X), ("GB", GB)):
        for r in range(NRHS):
            lines.append(f"colsum {name} {r} {float(np.sum(M[:, r])).hex()} {float(np.sum(np.abs(M[:, r]))).hex()}")
    for name, P, M in (("X", px, X), ("GB", pb, GB), ("GA", pa, GA)):
        for i, j in P:
            lines.append(f"entry {name} {int(i)} {int(j)} {float(M[i, j]).hex()}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {OUT} ({len(lines)} lines, {threads} threads)")


if __name__ == "__main__":
    main()
