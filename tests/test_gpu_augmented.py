"""GPU parity of hpl_solve_augmented (the HPL formulation, paper Sec. II: the
augmented system [A | B] is reduced to U X = L^{-1} P^{-1} B by the blocked LU
with partial pivoting, whose row interchanges reach only the columns right of
each panel, then X follows by back substitution) against the CPU oracle.

The oracle factors in LAPACK form (every interchange applied across all n
columns).  The augmented form differs only in the multipliers of each panel:
they stay in the row order of that panel's own factorization.  hpl_form_L turns
the oracle's L into that form by undoing, on each panel's columns, the
interchanges of the later panels (last applied first)."""
import numpy as np
import pytest

import inputs
import oracle
from gpu_util import hpl, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

SEED = 2304
XTOL = 1e-10


def hpl_form_L(L_lapack, ipiv, nb):
    """Strictly lower part of a LAPACK-form L, with each nb-column panel's rows
    put back in the order of that panel's own factorization."""
    n = L_lapack.shape[0]
    Lh = np.tril(L_lapack, -1).copy()
    for i in range(n - 1, -1, -1):
        p = int(ipiv[i])
        c0 = (i // nb) * nb  # columns of the panels before interchange i's panel
        if p != i and c0 > 0:
            Lh[[i, p], :c0] = Lh[[p, i], :c0]
    return Lh


def augmented_system(n, nrhs, ld, seed=SEED):
    h = hpl()
    AB = h.colmajor(n, n + nrhs, ld=ld, fill=float("nan"))
    h.hpl_generate(seed, 0, AB[:, :n])
    if nrhs:
        h.hpl_generate(seed, 1, AB[:, n:])
    return AB


@pytest.mark.parametrize("n", [1, 2, 65, 1000, 1031])
@pytest.mark.parametrize("nb", [32, 128])
@pytest.mark.parametrize("nrhs,pad", [(1, 0), (3, 5)])
def test_augmented_vs_oracle(n, nb, nrhs, pad):
    h = hpl()
    A0 = oracle.gen(SEED, 0, n, n).copy(order="F")
    B0 = oracle.gen(SEED, 1, n, nrhs).copy(order="F")
    LU_o = A0.copy(order="F")
    ipiv_o, info_o = oracle.lu(LU_o)
    X_o = B0.copy(order="F")
    for r in range(nrhs):
        col = X_o[:, r].copy()
        oracle.solve(LU_o, ipiv_o, col)
        X_o[:, r] = col
    AB = augmented_system(n, nrhs, n + pad)
    ipiv, info = h.hpl_solve_augmented(AB, n, nb)
    assert info == info_o == 0
    piv = ipiv.cpu().numpy()
    assert np.array_equal(piv, ipiv_o)
    got = to_host(AB)
    scale = max(1.0, np.max(np.abs(LU_o)))
    assert np.max(np.abs(np.triu(got[:, :n]) - np.triu(LU_o))) <= 1e-11 * scale
    assert np.max(np.abs(np.tril(got[:, :n], -1) - hpl_form_L(LU_o, ipiv_o, nb))) <= 1e-11 * scale
    X = got[:, n:]
    assert np.max(np.abs(X - X_o)) <= XTOL * np.max(np.abs(X_o))
    res = h.hpl_residual(to_gpu(A0), AB[:, n:], to_gpu(B0))
    assert res[0] < 16.0


@pytest.mark.parametrize("n,nb", [(200, 32), (1031, 128), (2100, 512)])
def test_augmented_dyadic_bit_exact(n, nb):
    h = hpl()
    A, L, U, perm = inputs.dyadic_factors(n, seed=n + nb + 1)
    rng = np.random.default_rng(n)
    x = rng.integers(-9, 10, size=(n, 2)).astype(np.float64)
    AB = to_gpu(np.hstack([A, A @ x]), ld=n + 3)
    ipiv, info = h.hpl_solve_augmented(AB, n, nb)
    assert info == 0
    piv = ipiv.cpu().numpy()
    order = np.arange(n)
    for k, p in enumerate(piv):
        order[[k, p]] = order[[p, k]]
    assert np.array_equal(order, perm)
    got = to_host(AB)
    assert np.array_equal(np.triu(got[:, :n]), U)
    assert np.array_equal(np.tril(got[:, :n], -1), hpl_form_L(L, piv, nb))
    assert np.array_equal(got[:, n:], x)


@pytest.mark.parametrize("n,nb", [(1031, 64), (2500, 128), (1500, 512)])
def test_augmented_lookahead_bitwise_and_same_U_as_factor(n, nb):
    h = hpl()
    t = torch()
    results = []
    try:
        for la, ser in [(1, 0), (0, 0), (2, 0), (1, 1)]:
            h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, la)
            h.hpl_set_option(h.HPL_OPT_SERIALIZE, ser)
            AB = augmented_system(n, 2, n, seed=11)
            ipiv, info = h.hpl_solve_augmented(AB, n, nb)
            assert info == 0
            results.append((to_host(AB), ipiv.cpu().numpy()))
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 1)
        h.hpl_set_option(h.HPL_OPT_SERIALIZE, 0)
        A = h.colmajor(n, n)
        h.hpl_generate(11, 0, A)
        ipiv_f, _ = h.hpl_factor(A, nb)
    finally:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 3)
        h.hpl_set_option(h.HPL_OPT_SERIALIZE, 0)
    ref = results[0]
    for got, piv in results[1:]:
        assert np.array_equal(piv, ref[1])
        assert np.array_equal(got.view(np.int64), ref[0].view(np.int64))
    # the pivots and U of hpl_factor on the same matrix, bit for bit
    assert np.array_equal(ipiv_f.cpu().numpy(), ref[1])
    U_f = np.triu(to_host(A))
    assert np.array_equal(np.triu(ref[0][:, :n]).view(np.int64), U_f.view(np.int64))
    del A
    t.cuda.empty_cache()


def test_augmented_host_panel_vs_oracle():
    h = hpl()
    n, nb = 700, 64
    A0 = oracle.gen(SEED, 0, n, n).copy(order="F")
    b0 = oracle.gen(SEED, 1, n, 1)[:, 0].copy()
    LU_o = A0.copy(order="F")
    ipiv_o, _ = oracle.lu(LU_o)
    x_o = b0.copy()
    oracle.solve(LU_o, ipiv_o, x_o)
    h.hpl_set_option(h.HPL_OPT_HOST_PANEL, 2)
    try:
        AB = augmented_system(n, 1, n)
        ipiv, info = h.hpl_solve_augmented(AB, n, nb)
    finally:
        h.hpl_set_option(h.HPL_OPT_HOST_PANEL, 0)
    assert info == 0
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_o)
    x = to_host(AB)[:, n]
    assert np.max(np.abs(x - x_o)) <= XTOL * np.max(np.abs(x_o))


def test_augmented_no_rhs_and_singular():
    h = hpl()
    n, nb = 300, 32
    # nrhs = 0: the factorization alone, in the augmented (HPL) form
    AB = augmented_system(n, 0, n)
    ipiv, info = h.hpl_solve_augmented(AB, n, nb)
    assert info == 0
    A0 = oracle.gen(SEED, 0, n, n).copy(order="F")
    LU_o = A0.copy(order="F")
    ipiv_o, _ = oracle.lu(LU_o)
    got = to_host(AB)
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_o)
    assert np.max(np.abs(np.tril(got, -1) - hpl_form_L(LU_o, ipiv_o, nb))) <= 1e-11 * np.max(np.abs(LU_o))
    # an all-zero column: info names it; the back substitution is skipped
    AB = augmented_system(n, 1, n)
    AB[:, 137] = 0.0
    _, info = h.hpl_solve_augmented(AB, n, nb)
    assert info == 138


def test_augmented_zero_order():
    h = hpl()
    AB = h.colmajor(0, 1)
    ipiv = torch().empty(1, dtype=torch().int32, device="cuda")
    _, info = h.hpl_solve_augmented(AB, 0, 64, ipiv=ipiv)
    assert info == 0
