"""Pins of the oracle's batched pieces (CPU only).

oracle.batched_sizes is pinned to its definition's range and to uniformity
(chi-square); oracle.batched_solve's packing (offsets of A_i, B_i, W_i, ipiv_i)
and per-system results are pinned to closed forms: diagonal systems
(X = B / d, grad_B = W / d, grad_A = -grad_B X^T) and permutation systems
(X = P^T B, the interchanges that partial pivoting must choose).
"""
import numpy as np
import pytest

import oracle


def test_sizes_range_uniform_deterministic():
    s = oracle.batched_sizes(2304, 200_000, 32, 512)
    assert s.dtype == np.int32 and s.min() == 32 and s.max() == 512
    counts = np.bincount(s - 32, minlength=481)
    assert np.all(counts > 0)
    from scipy import stats
    assert stats.chisquare(counts).pvalue > 1e-4
    assert np.array_equal(s, oracle.batched_sizes(2304, 200_000, 32, 512))
    assert not np.array_equal(s[:1000], oracle.batched_sizes(2305, 1000, 32, 512))
    assert np.all(oracle.batched_sizes(1, 50, 7, 7) == 7)


def _pack(mats):
    return np.concatenate([m.reshape(-1, order="F") for m in mats]) if mats else np.zeros(0)


def test_batched_diagonal_closed_form():
    rng = np.random.default_rng(3)
    sizes = np.array([3, 1, 5, 2, 7], dtype=np.int32)
    nrhs = 3
    ds = [rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n) for n in sizes]
    Bs = [rng.standard_normal((n, nrhs)) for n in sizes]
    Ws = [rng.standard_normal((n, nrhs)) for n in sizes]
    out = oracle.batched_solve(sizes, _pack([np.diag(d) for d in ds]), _pack(Bs), nrhs, W=_pack(Ws))
    aoff, voff = oracle.batch_offsets(sizes, nrhs)
    assert np.all(out["info"] == 0)
    for i, n in enumerate(sizes):
        X = oracle.batch_rhs(sizes, out["X"], voff, nrhs, i)
        GB = oracle.batch_rhs(sizes, out["GB"], voff, nrhs, i)
        GA = oracle.batch_system(sizes, out["GA"], aoff, i)
        Xc, GBc = Bs[i] / ds[i][:, None], Ws[i] / ds[i][:, None]
        assert np.array_equal(X, Xc) and np.array_equal(GB, GBc)
        assert np.max(np.abs(GA + GBc @ Xc.T)) <= 1e-15 * max(1.0, np.max(np.abs(GA)))
        assert np.array_equal(out["ipiv"][voff[i]:voff[i] + n], np.arange(n))
        assert np.array_equal(oracle.batch_system(sizes, out["LU"], aoff, i), np.diag(ds[i]))


def test_batched_permutation_systems():
    rng = np.random.default_rng(4)
    sizes = np.array([4, 6, 1, 3], dtype=np.int32)
    nrhs = 2
    perms = [rng.permutation(n) for n in sizes]
    As = [np.eye(n)[p] for n, p in zip(sizes, perms)]          # A x = b  ->  x = A^T b
    Bs = [rng.integers(-9, 10, (n, nrhs)).astype(float) for n in sizes]
    Ws = [rng.integers(-9, 10, (n, nrhs)).astype(float) for n in sizes]
    out = oracle.batched_solve(sizes, _pack(As), _pack(Bs), nrhs, W=_pack(Ws))
    aoff, voff = oracle.batch_offsets(sizes, nrhs)
    for i, n in enumerate(sizes):
        X = oracle.batch_rhs(sizes, out["X"], voff, nrhs, i)
        GB = oracle.batch_rhs(sizes, out["GB"], voff, nrhs, i)
        GA = oracle.batch_system(sizes, out["GA"], aoff, i)
        assert np.array_equal(X, As[i].T @ Bs[i])
        assert np.array_equal(GB, As[i] @ Ws[i])                  # A^{-T} = A for a permutation
        assert np.array_equal(GA, -(As[i] @ Ws[i]) @ (As[i].T @ Bs[i]).T)
        # partial pivoting on a permutation matrix: U = I, the interchanges bring row p(k) up
        assert np.array_equal(oracle.batch_system(sizes, out["LU"], aoff, i), np.eye(n))


def test_batched_singular_info():
    sizes = np.array([3, 4], dtype=np.int32)
    A1 = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 9.5]])
    A2 = np.eye(4)
    A2[:, 2] = 0.0
    out = oracle.batched_solve(sizes, _pack([A1, A2]), np.ones(7), 1)
    assert out["info"][0] == 0 and out["info"][1] == 3
