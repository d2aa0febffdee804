"""Pins for the oracle's triangular solves and residual."""
import numpy as np
import pytest

import oracle
import inputs

EPS = 2.0**-53


def lu(A):
    A = inputs.fortran(A)
    ipiv, info = oracle.lu(A)
    return A, ipiv


@pytest.mark.parametrize("n,nrhs", [(10, 1), (40, 3), (120, 2)])
def test_integer_system_known_x(n, nrhs):
    A, X, B = inputs.integer_system(n, 31 * n, nrhs=nrhs)
    LU, ipiv = lu(A)
    Bf = inputs.fortran(B)
    oracle.solve(LU, ipiv, Bf)
    cond = np.linalg.cond(A)
    assert np.max(np.abs(Bf - X)) <= 50 * cond * EPS * np.max(np.abs(X))


@pytest.mark.parametrize("n", [3, 64, 250])
def test_dyadic_solve_exact(n):
    A, L, U, perm = inputs.dyadic_factors(n, seed=3 * n)
    rng = np.random.default_rng(n)
    x = rng.integers(-9, 10, size=n).astype(np.float64)
    b = A @ x  # exact (multiples of 1/8, small)
    LU, ipiv = lu(A)
    y = b.copy()
    oracle.solve(LU, ipiv, y)
    assert np.array_equal(y, x)
    # transposed: A^T x = c with c = A^T x exact
    c = A.T @ x
    oracle.solve(LU, ipiv, c, trans=1)
    assert np.array_equal(c, x)


@pytest.mark.parametrize("n", [17, 200])
def test_against_numpy_solve(n):
    A = inputs.uniform_matrix(n, n, n + 1)
    B = inputs.uniform_matrix(n, 4, n + 2)
    LU, ipiv = lu(A)
    X = inputs.fortran(B)
    oracle.solve(LU, ipiv, X)
    ref = np.linalg.solve(A, B)
    assert np.max(np.abs(X - ref)) <= 1e-10 * np.max(np.abs(ref))
    XT = inputs.fortran(B)
    oracle.solve(LU, ipiv, XT, trans=1)
    refT = np.linalg.solve(A.T, B)
    assert np.max(np.abs(XT - refT)) <= 1e-10 * np.max(np.abs(refT))


def test_residual_closed_form():
    n = 6
    A = inputs.fortran(np.eye(n))
    b = np.arange(1.0, n + 1)
    delta = 0.25
    x = b.copy()
    x[3] += delta
    out = oracle.residual(A, x, b)
    assert out[1] == delta  # ||r||inf
    assert out[2] == 1.0    # ||A||inf
    assert out[3] == np.max(np.abs(x))
    assert out[4] == n
    assert out[0] == delta / (EPS * (1.0 * np.max(np.abs(x)) + n) * n)


def test_residual_row_sums():
    A = inputs.fortran(np.array([[1.0, -2.0], [-3.0, 0.5]]))
    x = np.array([1.0, 1.0])
    b = np.array([-1.0, -2.5])
    out = oracle.residual(A, x, b)
    assert out[2] == 3.5 and out[1] == 0.0 and out[0] == 0.0


def test_residual_gen_matches_explicit():
    n = 50
    A = oracle.gen(99, 0, n, n)
    x = inputs.uniform_matrix(n, 1, 1)[:, 0]
    b = inputs.uniform_matrix(n, 1, 2)[:, 0]
    assert np.array_equal(oracle.residual(A, x, b), oracle.residual_gen(99, n, x, b))


@pytest.mark.parametrize("n", [100, 512])
def test_hpl_pass_on_random_system(n):
    A = oracle.gen(2304, 0, n, n)
    b = oracle.gen(2304, 1, n, 1)[:, 0].copy()
    LU, ipiv = lu(A)
    x = b.copy()
    oracle.solve(LU, ipiv, x)
    out = oracle.residual_gen(2304, n, x, b)
    assert out[0] < 16.0
    # a wrong solution must fail the test
    x[0] += 1e-6
    assert oracle.residual_gen(2304, n, x, b)[0] > 16.0


def test_residual_nan_fails():
    n = 8
    A = oracle.gen(1, 0, n, n)
    x = np.ones(n)
    x[2] = np.nan
    out = oracle.residual(A, x, np.ones(n))
    assert np.isnan(out[0]) or out[0] >= 16.0
