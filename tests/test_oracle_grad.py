"""Pins of the oracle's differentiable-solve pieces (CPU only).

oracle.gen_normal (Box-Muller) is pinned to the standard normal law by its
moments and a Kolmogorov-Smirnov test against scipy's normal CDF.
oracle.solve_grad (X = A^{-1}B, grad_B = A^{-T}W, grad_A = -grad_B X^T for the
loss sum(W * X)) is pinned to: the closed form for diagonal A, central finite
differences of the oracle's own forward solve on tiny systems, and exact
rational arithmetic (fractions) on a 4 x 4 system.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_normal_moments_and_ks():
    z = oracle.gen_normal(2304, 2, 500_000, 1)[:, 0]
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    skew = np.mean(z ** 3)
    kurt = np.mean(z ** 4)
    assert abs(skew) < 5 * np.sqrt(15.0 / n)
    assert abs(kurt - 3.0) < 5 * np.sqrt(96.0 / n)
    from scipy import stats
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert 0.49 < np.mean(z < 0) < 0.51


def test_normal_streams_independent_and_deterministic():
    a = oracle.gen_normal(7, 2, 20_000, 1)[:, 0]
    b = oracle.gen_normal(7, 3, 20_000, 1)[:, 0]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(a.size)
    again = oracle.gen_normal(7, 2, 20_000, 1)[:, 0]
    assert np.array_equal(a.view(np.int64), again.view(np.int64))
    # index = i + j*rows, independent of the leading dimension
    M = oracle.gen_normal(7, 2, 100, 3, ld=117)
    flat = oracle.gen_normal(7, 2, 300, 1)[:, 0]
    assert np.array_equal(M.flatten(order="F"), flat)


def test_grad_diagonal_closed_form():
    rng = np.random.default_rng(11)
    n, k = 37, 5
    d = rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n)
    A = np.asfortranarray(np.diag(d))
    B = np.asfortranarray(rng.standard_normal((n, k)))
    W = np.asfortranarray(rng.standard_normal((n, k)))
    X, GB, GA, info = oracle.solve_grad(A, B, W)
    assert info == 0
    Xc = B / d[:, None]
    GBc = W / d[:, None]
    GAc = -np.einsum("ir,jr->ij", GBc, Xc)
    assert np.array_equal(X, Xc)
    assert np.array_equal(GB, GBc)
    assert np.max(np.abs(GA - GAc)) <= 1e-14 * np.max(np.abs(GAc))


def _loss(A, B, W):
    LU = np.asfortranarray(A.copy())
    ipiv, info = oracle.lu(LU)
    X = np.asfortranarray(B.copy())
    oracle.solve(LU, ipiv, X)
    return float(np.sum(W * X))


@pytest.mark.parametrize("n,k,seed", [(3, 1, 1), (5, 2, 2), (6, 3, 3)])
def test_grad_central_differences(n, k, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.uniform(-0.5, 0.5, (n, n)) + 2.0 * np.eye(n))
    B = np.asfortranarray(rng.uniform(-0.5, 0.5, (n, k)))
    W = np.asfortranarray(rng.standard_normal((n, k)))
    _, GB, GA, info = oracle.solve_grad(A, B, W)
    assert info == 0
    h = 1e-6
    for i in range(n):
        for j in range(n):
            Ap, Am = A.copy(order="F"), A.copy(order="F")
            Ap[i, j] += h
            Am[i, j] -= h
            fd = (_loss(Ap, B, W) - _loss(Am, B, W)) / (2 * h)
            assert abs(fd - GA[i, j]) <= 1e-6 * (1.0 + abs(GA[i, j])), (i, j, fd, GA[i, j])
        for r in range(k):
            Bp, Bm = B.copy(order="F"), B.copy(order="F")
            Bp[i, r] += h
            Bm[i, r] -= h
            fd = (_loss(A, Bp, W) - _loss(A, Bm, W)) / (2 * h)
            assert abs(fd - GB[i, r]) <= 1e-6 * (1.0 + abs(GB[i, r]))


def _exact_solve(A, B):
    """Gauss-Jordan in exact rationals (brute force for tiny n)."""
    n = len(A)
    M = [[Fraction(A[i][j]) for j in range(n)] + [Fraction(B[i][r]) for r in range(len(B[0]))] for i in range(n)]
    for c in range(n):
        p = next(i for i in range(c, n) if M[i][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for i in range(n):
            if i != c and M[i][c] != 0:
                f = M[i][c]
                M[i] = [vi - f * vc for vi, vc in zip(M[i], M[c])]
    return [row[n:] for row in M]


def test_grad_exact_rationals():
    A = [[2, -1, 0, 3], [1, 4, -2, 0], [0, 1, 5, -1], [-3, 0, 1, 2]]
    B = [[1, 0], [2, -1], [0, 3], [-1, 1]]
    W = [[1, 2], [0, -1], [3, 1], [-2, 0]]
    X = _exact_solve(A, B)
    AT = [[A[j][i] for j in range(4)] for i in range(4)]
    GB = _exact_solve(AT, W)
    GA = [[-sum(GB[i][r] * X[j][r] for r in range(2)) for j in range(4)] for i in range(4)]
    Xo, GBo, GAo, info = oracle.solve_grad(np.asfortranarray(np.array(A, float)),
                                           np.asfortranarray(np.array(B, float)),
                                           np.asfortranarray(np.array(W, float)))
    assert info == 0
    for i in range(4):
        for r in range(2):
            assert abs(Xo[i, r] - float(X[i][r])) <= 1e-14
            assert abs(GBo[i, r] - float(GB[i][r])) <= 1e-14
        for j in range(4):
            assert abs(GAo[i, j] - float(GA[i][j])) <= 1e-14


@pytest.mark.parametrize("n,k,threads", [(1, 1, 4), (97, 3, 3), (300, 16, 8)])
def test_grad_threaded_bitwise(n, k, threads):
    """The threaded form (factorization on several host threads) gives the
    serial oracle's X, grad_B and grad_A bit for bit."""
    A = oracle.gen(11, 0, n, n).copy(order="F")
    A[np.arange(n), np.arange(n)] += 8.0
    B = oracle.gen(11, 1, n, k).copy(order="F")
    W = oracle.gen_normal(11, 2, n, k).copy(order="F")
    ref = oracle.solve_grad(A, B, W)
    got = oracle.solve_grad(A, B, W, threads=threads)
    for r, g in zip(ref[:3], got[:3]):
        assert np.array_equal(r.view(np.int64), g.view(np.int64))
    assert ref[3] == got[3]
