"""Pins for the oracle's LU with partial pivoting (FACT/RS/UPDATE reduced to one column)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
import inputs
from golden.load import keyed_fractions

EPS = 2.0**-53


def factor(A):
    A = inputs.fortran(A)
    ipiv, info = oracle.lu(A)
    return A, ipiv, info


def split(LU):
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return L, U


def perm_from_ipiv(ipiv, n):
    """Row order after applying the interchanges in sequence: (P A)[i] = A[order[i]]."""
    order = np.arange(n)
    for k, p in enumerate(ipiv):
        order[[k, p]] = order[[p, k]]
    return order


def leibniz_det(A):
    n = A.shape[0]
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = Fraction(1)
        for i in range(n):
            prod *= Fraction(A[i, perm[i]])
        total += -prod if inv % 2 else prod
    return total


def bareiss_det(M):
    """Exact integer determinant (fraction-free elimination, Bareiss 1968)."""
    M = [[int(x) for x in row] for row in M]
    n = len(M)
    sign, prev = 1, 1
    for k in range(n - 1):
        if M[k][k] == 0:
            for i in range(k + 1, n):
                if M[i][k] != 0:
                    M[k], M[i] = M[i], M[k]
                    sign = -sign
                    break
            else:
                return 0
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = (M[i][j] * M[k][k] - M[i][k] * M[k][j]) // prev
        prev = M[k][k]
    return sign * M[n - 1][n - 1]


def test_worked_3x3_example():
    g = keyed_fractions("lu3x3_worked.txt")
    A = np.array([[float(x) for x in r] for r in g["A"]])
    LU, ipiv, info = factor(A)
    assert info == 0
    assert list(ipiv) == [int(x) for x in g["ipiv"][0]]
    L, U = split(LU)
    np.testing.assert_allclose(L, [[float(x) for x in r] for r in g["L"]], rtol=0, atol=4e-16)
    np.testing.assert_allclose(U, [[float(x) for x in r] for r in g["U"]], rtol=0, atol=4e-15)
    s, l2, ex = oracle.det(LU, ipiv)
    assert ex == pytest.approx(float(g["det"][0][0]), rel=1e-14)
    b = np.array([float(x) for x in g["b"][0]])
    oracle.solve(LU, ipiv, b)
    np.testing.assert_allclose(b, [float(x) for x in g["x"][0]], rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_determinant_vs_leibniz(n):
    for seed in range(3):
        A = inputs.uniform_matrix(n, n, 100 * n + seed)
        want = float(leibniz_det(A))
        LU, ipiv, _ = factor(A)
        _, _, got = oracle.det(LU, ipiv)
        assert got == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("n", [8, 12, 20])
def test_determinant_vs_bareiss(n):
    for seed in range(3):
        Ai, _, _ = inputs.integer_system(n, 7 * n + seed)
        want = bareiss_det(Ai)
        LU, ipiv, _ = factor(Ai)
        sgn, l2, got = oracle.det(LU, ipiv)
        assert got == pytest.approx(float(want), rel=1e-11)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 200])
def test_dyadic_exact_factorization(n):
    A, L, U, perm = inputs.dyadic_factors(n, seed=n)
    LU, ipiv, info = factor(A)
    assert info == 0
    Lg, Ug = split(LU)
    assert np.array_equal(Lg, L) and np.array_equal(Ug, U)  # bit-exact
    order = perm_from_ipiv(ipiv, n)
    assert np.array_equal(order, perm)


def test_identity():
    LU, ipiv, info = factor(np.eye(9))
    assert info == 0 and list(ipiv) == list(range(9))
    assert np.array_equal(LU, np.eye(9))


def test_permutation_matrix():
    P, perm = inputs.permutation_matrix(17, 3)
    LU, ipiv, info = factor(P)
    assert info == 0
    assert np.array_equal(LU, np.eye(17))  # L = U = I
    # P @ x permutes: (P A)[i] = A[perm_inverse...]; rows of P: row i has its 1 at perm[i]
    order = perm_from_ipiv(ipiv, 17)
    assert np.array_equal(P[order], np.eye(17))


def test_upper_triangular_no_pivoting():
    Ut = inputs.upper_triangular(23, 4)
    LU, ipiv, info = factor(Ut)
    assert list(ipiv) == list(range(23))
    assert np.array_equal(LU, Ut)


def test_column_dominant_no_pivoting():
    A = inputs.column_dominant(60, 5)
    LU, ipiv, _ = factor(A)
    assert list(ipiv) == list(range(60))


@pytest.mark.parametrize("n", [50, 257, 600])
def test_backward_error_bound(n):
    # |P A - L U| <= gamma_n |L| |U| elementwise (Higham, Thm 9.3), gamma_n = n eps/(1 - n eps)
    A = inputs.uniform_matrix(n, n, n)
    LU, ipiv, _ = factor(A)
    L, U = split(LU)
    order = perm_from_ipiv(ipiv, n)
    R = np.abs(A[order] - L @ U)
    gamma = n * EPS / (1 - n * EPS)
    bound = gamma * (np.abs(L) @ np.abs(U))
    assert np.all(R <= bound * 1.0001 + 1e-300)
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)  # partial pivoting bounds multipliers


@pytest.mark.parametrize("n", [64, 300, 1024])
def test_matches_lapack(n):
    A = oracle.gen(2304, 0, n, n)
    lu_s, piv_s = scipy.linalg.lu_factor(A.copy(order="F"))
    LU, ipiv, _ = factor(A)
    assert np.array_equal(ipiv, piv_s)
    assert np.max(np.abs(LU - lu_s)) <= 1e-11 * max(1.0, np.max(np.abs(lu_s)))


def test_zero_column_sets_info_and_completes():
    A = inputs.uniform_matrix(12, 12, 9)
    A[:, 4] = 0.0
    A0 = A.copy()
    LU, ipiv, info = factor(A)
    assert info == 5
    L, U = split(LU)
    order = perm_from_ipiv(ipiv, 12)
    np.testing.assert_allclose(L @ U, A0[order], atol=1e-13)


def test_n_zero_and_padding():
    LU, ipiv, info = factor(np.zeros((0, 0)))
    assert info == 0 and ipiv.size == 0
    A = inputs.uniform_matrix(33, 33, 1)
    A1, p1, _ = factor(A)
    A2 = inputs.fortran(A, ld=40)
    p2, _ = oracle.lu(A2)
    assert np.array_equal(A1, A2) and np.array_equal(p1, p2)


@pytest.mark.parametrize("n", [16, 90])
def test_ties_take_first_row_like_lapack(n):
    # integer entries in [-2, 2] give many equal |a| candidates; LAPACK's idamax
    # returns the first, which is the reading used for ties
    Ai, _, _ = inputs.integer_system(n, 5 + n, lo=-2, hi=2)
    lu_s, piv_s = scipy.linalg.lu_factor(Ai.copy(order="F"))
    LU, ipiv, info = factor(Ai)
    assert info == 0
    assert np.array_equal(ipiv, piv_s)
    np.testing.assert_allclose(LU, lu_s, atol=1e-12)


def test_tie_explicit_column():
    A = np.array([[1.0, 2.0, 0.5], [-1.0, 1.0, 3.0], [1.0, 0.0, 1.0]])
    _, ipiv, _ = factor(A)
    assert ipiv[0] == 0


@pytest.mark.parametrize("n,threads", [(1, 4), (37, 3), (300, 8), (301, 16), (520, 5)])
def test_parallel_form_bitwise(n, threads):
    """The threaded form (used only to time the oracle on every host core) gives
    the bits of the serial oracle, pivots and info included; with a padded lda."""
    A0 = inputs.fortran(oracle.gen(17, 0, n, n), ld=n + 3)
    A1 = inputs.fortran(A0, ld=n + 3)
    A2 = inputs.fortran(A0, ld=n + 3)
    p1, i1 = oracle.lu(A1)
    p2, i2, used = oracle.lu_par(A2, threads)
    assert used == threads
    assert i1 == i2 == 0
    assert np.array_equal(p1, p2)
    assert np.array_equal(A1.view(np.int64), A2.view(np.int64))


def test_parallel_form_singular_and_dyadic():
    # zero columns: info and the skipped steps as in the serial form
    A = inputs.fortran(oracle.gen(3, 0, 60, 60))
    A[:, 7] = 0.0
    A[:, 40] = 0.0
    B = inputs.fortran(A)
    p1, i1 = oracle.lu(A)
    p2, i2, _ = oracle.lu_par(B, 6)
    assert i1 == i2 == 8
    assert np.array_equal(p1, p2) and np.array_equal(A.view(np.int64), B.view(np.int64))
    # exact factors of a dyadic construction
    Ad, L, U, perm = inputs.dyadic_factors(200, 5)
    F = inputs.fortran(Ad)
    ipiv, info, _ = oracle.lu_par(F, 7)
    assert info == 0
    assert np.array_equal(np.tril(F, -1) + np.eye(200), L) and np.array_equal(np.triu(F), U)
