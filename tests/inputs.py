"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module only builds inputs (numpy, seeded); it holds none of the arithmetic of
LU, the solves or the residual.  Large random HPL matrices are not built here: the
oracle draws them from its own SplitMix64 generator and the GPU library from its
own, and a test checks that the two agree bit for bit.

All matrices are returned as float64 arrays in Fortran (column-major) order.
"""
import numpy as np


def fortran(a, ld=None):
    """Column-major copy of a (n x m); with ld > n the copy sits in an ld x m buffer."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return np.array(a, dtype=np.float64)
    n, m = a.shape
    ld = n if ld is None else ld
    buf = np.full((ld, m), np.nan, dtype=np.float64, order="F")  # padding poisoned
    buf[:n, :] = a
    return buf[:n, :]


def dyadic_factors(n, seed):
    """Exact construction A = P^T L U.

    L: unit lower triangular, off-diagonal entries multiples of 1/8 in [-7/8, 7/8]
       (|l| < 1 strictly, so partial pivoting must pick the row holding L's 1).
    U: upper triangular, integers in [-8, 8], nonzero diagonal.
    perm: a random permutation; A[perm[i], :] = (L U)[i, :], i.e. row i of L U
          sits at row perm[i] of A.
    Every product and partial sum is a multiple of 1/8 far below 2^50, so A is
    exact in fp64 and the factorization of A is exact in any summation order.
    Returns (A, L, U, perm).
    """
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-7, 8, size=(n, n)).astype(np.float64) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-8, 9, size=(n, n)).astype(np.float64), 1)
    d = rng.integers(1, 9, size=n) * rng.choice([-1, 1], size=n)
    U += np.diag(d.astype(np.float64))
    perm = rng.permutation(n)
    LU = L @ U  # exact: multiples of 1/8, |.| < 2^20
    A = np.empty_like(LU)
    A[perm, :] = LU
    return A, L, U, perm


def integer_system(n, seed, lo=-9, hi=9, nrhs=1):
    """Integer A in [lo, hi], integer X in [-9, 9], B = A X computed exactly in int64."""
    rng = np.random.default_rng(seed)
    Ai = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int64)
    Xi = rng.integers(-9, 10, size=(n, nrhs)).astype(np.int64)
    Bi = Ai @ Xi
    return Ai.astype(np.float64), Xi.astype(np.float64), Bi.astype(np.float64)


def uniform_matrix(n, m, seed):
    """i.i.d. U[-0.5, 0.5) via numpy (small tests only; HPL matrices use the generators)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, m)) - 0.5


def column_dominant(n, seed):
    """Strictly column diagonally dominant matrix: partial pivoting never interchanges."""
    A = uniform_matrix(n, n, seed)
    A[np.arange(n), np.arange(n)] = 0.0
    colsum = np.abs(A).sum(axis=0)
    A[np.arange(n), np.arange(n)] = (colsum + 1.0) * np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return A


def permutation_matrix(n, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    return P, perm


def upper_triangular(n, seed):
    rng = np.random.default_rng(seed)
    U = np.triu(rng.random((n, n)) - 0.5)
    U[np.arange(n), np.arange(n)] += np.where(rng.random(n) < 0.5, -2.0, 2.0)
    return U


# Exponents of the scaled mixed-precision construction below.
MXP_L21_EXP = -30      # L21 entries are odd multiples of 2^-30
MXP_U12_EXP = 27       # U12 entries are odd multiples of 2^27
MXP_BIG = 2047         # the largest odd multiple (11 significant bits)


def mxp_scaled_lu(n, w, seed):
    """A = L U whose first panel (columns [0, w)) has multipliers far below FP16's
    normal range and a U block row far above its largest value, so that FP16
    copies of L21 and U12 are exact only after a power-of-two exchange of scale
    between them.

    L: unit lower.  L21 = rows >= w of columns < w: odd multiples of 2^-30 in
    {+-1, +-3, +-5, +-7} * 2^-30, one entry 2047 * 2^-30 (at (i*, k*)); every
    other strictly lower entry a multiple of 1/8 in [-1/2, 1/2].
    U: upper, power-of-two diagonal (1, 2 or 4).  U12 = rows < w of columns >= w:
    odd multiples of 2^27 in {+-1, ..., +-7} * 2^27, one entry 2047 * 2^27 (at
    (k*, j*), the same k* as L's large entry, so the product 2047^2 * 2^-3
    occurs); every other strictly upper entry an integer in [-7, 7].

    FP32 holds every entry of A, of the panel's intermediate values and of the
    trailing update's partial sums exactly (A12: multiples of 2^24 below 2^40;
    A21: multiples of 2^-30 below 2^-14; A22: multiples of 1/8 below 2^21).
    FP16 (11 significant bits, largest 65504, smallest subnormal 2^-24) holds
    2^s L21 and 2^-s U12 exactly iff 22 <= s <= 35: 2^(s-30) >= 2^-24 and
    2047 * 2^(s-30) <= 65504 for L21, 2047 * 2^(27-s) <= 65504 = 2047 * 2^5 and
    2^(27-s) >= 2^-24 for U12.  Returns (A, L, U) as float64 Fortran arrays."""
    rng = np.random.default_rng(seed)
    odd = np.array([-7, -5, -3, -1, 1, 3, 5, 7], dtype=np.float64)
    L = np.tril(rng.integers(-4, 5, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-7, 8, (n, n)).astype(np.float64), 1) + np.diag(2.0 ** rng.integers(0, 3, n))
    m = n - w
    if m > 0 and w > 0:
        L[w:, :w] = rng.choice(odd, size=(m, w)) * 2.0 ** MXP_L21_EXP
        U[:w, w:] = rng.choice(odd, size=(w, m)) * 2.0 ** MXP_U12_EXP
        ib, kb, jb = w + int(rng.integers(0, m)), int(rng.integers(0, w)), w + int(rng.integers(0, m))
        L[ib, kb] = MXP_BIG * 2.0 ** MXP_L21_EXP
        U[kb, jb] = MXP_BIG * 2.0 ** MXP_U12_EXP
    A = np.asfortranarray(L @ U)   # exact in fp64: see above
    return A, L, U


def fp16_exact(x):
    """Whether every entry of the float64 array x is exactly an IEEE binary16 value."""
    with np.errstate(over="ignore"):
        h = x.astype(np.float16).astype(np.float64)
    return bool(np.all(h == x))
