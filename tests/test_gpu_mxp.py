"""GPU parity tests of the mixed-precision LU and FP64 refinement (C ABI:
hpl_mxp_generate, hpl_mxp_factor, hpl_mxp_solve) against the oracle
(oracle.mxp_gen, oracle.lu_mxp, the FP64 oracle solve and residual)."""
import numpy as np
import pytest

import oracle
from gpu_util import hpl, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

UNIT = {0: 2.0 ** -11, 1: 2.0 ** -8}   # unit roundoff of FP16, BF16


def gpu_mxp_system(n, seed):
    h = hpl()
    A = h.colmajor(n, n)
    h.hpl_mxp_generate(seed, A)
    b = h.colmajor(n, 1)
    h.hpl_generate(seed, 1, b)
    return A, b[:, 0]


@pytest.mark.parametrize("n", [1, 7, 300, 1000])
def test_mxp_generate_bitwise(n):
    A, _ = gpu_mxp_system(n, 11)
    assert np.array_equal(to_host(A).view(np.int64), oracle.mxp_gen(11, n).view(np.int64))


def dyadic_lu(n, seed):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-4, 5, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-7, 8, (n, n)).astype(float), 1) + np.diag(2.0 ** rng.integers(0, 3, n))
    return np.asfortranarray(L @ U), L, U


@pytest.mark.parametrize("n,nb", [(64, 64), (200, 64), (300, 128), (517, 256), (2100, 2048)])
@pytest.mark.parametrize("fmt", [0, 1])
def test_mxp_factor_dyadic_exact(n, nb, fmt):
    h = hpl()
    A, L, U = dyadic_lu(n, n + nb + fmt)
    LU, info = h.hpl_mxp_factor(to_gpu(A), nb=nb, fmt=fmt)
    assert info == 0
    LUh = LU.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.tril(LUh, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(LUh), U)


@pytest.mark.parametrize("fmt", [0, 1])
def test_mxp_factor_zero_pivot_info(fmt):
    """A = L U (dyadic) with u_kk = 0: after eliminating columns < k, column k is
    exactly zero on and below the diagonal, so info = k + 1 whatever the
    schedule; k = 300 lies in a leaf whose rows span two workgroups."""
    h = hpl()
    n, nb, k = 700, 128, 300
    rng = np.random.default_rng(12)
    L = np.tril(rng.integers(-4, 5, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-7, 8, (n, n)).astype(float), 1) + np.diag(2.0 ** rng.integers(0, 3, n))
    U[k, k] = 0.0
    A = np.asfortranarray(L @ U)
    _, info_o = oracle.lu_mxp(A, nb, fmt)
    assert info_o == k + 1
    old = h.hpl_get_option(h.HPL_OPT_LOOKAHEAD)
    try:
        for la in (1, 0):
            h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, la)
            LU, info = h.hpl_mxp_factor(to_gpu(A), nb=nb, fmt=fmt)
            assert info == k + 1, (la, info)
            # the columns before k are the exact factors
            LUh = LU.cpu().numpy().astype(np.float64)
            assert np.array_equal(np.tril(LUh, -1)[:, :k], np.tril(L, -1)[:, :k])
            assert np.array_equal(np.triu(LUh)[:k, :], U[:k, :])
    finally:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, old)


@pytest.mark.parametrize("n,nb", [(64, 64), (130, 64), (1000, 128), (3000, 512), (4160, 1024), (2500, 64),
                                  (8192, 256)])
@pytest.mark.parametrize("fmt", [0, 1])
def test_mxp_factor_lookahead_bitwise(n, nb, fmt):
    """The look-ahead schedule (the next pair's columns and rows first, its panel
    work on the panel stream beside the rest of the joint update) gives the bits
    of the plain schedule.  At n = 8192 the plain schedule's joint updates run
    on the 256 x 128 kernel alone, the look-ahead's narrow pieces on the
    128 x 128 one: the two kernels must round alike."""
    h = hpl()
    A, _ = gpu_mxp_system(n, 9)
    old = h.hpl_get_option(h.HPL_OPT_LOOKAHEAD)
    try:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 0)
        LU0, info0 = h.hpl_mxp_factor(A, nb=nb, fmt=fmt)
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 1)
        LU1, info1 = h.hpl_mxp_factor(A, nb=nb, fmt=fmt)
    finally:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, old)
    assert info0 == info1 == 0
    assert np.array_equal(LU0.cpu().numpy().view(np.int32), LU1.cpu().numpy().view(np.int32))


@pytest.mark.parametrize("n,nb", [(256, 64), (1000, 128), (1536, 512)])
@pytest.mark.parametrize("fmt", [0, 1])
def test_mxp_factor_vs_oracle(n, nb, fmt):
    h = hpl()
    A, _ = gpu_mxp_system(n, 5)
    LU, info = h.hpl_mxp_factor(A, nb=nb, fmt=fmt)
    assert info == 0
    Ah = oracle.mxp_gen(5, n)
    LUo, info_o = oracle.lu_mxp(Ah, nb, fmt)
    assert info_o == 0
    G = LU.cpu().numpy().astype(np.float64)
    O = LUo.astype(np.float64)
    # the same method in the same formats: differences only from FP32 rounding
    # order (FMA, the panel's blocking, the MFMA's accumulation), each of which
    # may move an operand across a rounding boundary of the format
    Lg, Ug = np.tril(G, -1) + np.eye(n), np.triu(G)
    scale = np.abs(np.tril(O, -1) + np.eye(n)) @ np.abs(np.triu(O))
    d = np.abs(Lg @ Ug - (np.tril(O, -1) + np.eye(n)) @ np.triu(O))
    ratio = float(np.max(d / (UNIT[fmt] * scale)))
    print(f"n={n} nb={nb} fmt={fmt}: |LU_gpu - LU_oracle| <= {ratio:.3g} u |L||U|")
    assert ratio <= 4.0
    # and the GPU factors satisfy the backward-error bound of the format
    E = np.abs(Ah - Lg @ Ug)
    bound = 2.0 * n * UNIT[fmt] * (np.abs(Lg) @ np.abs(Ug)) + 4.0 * 2.0 ** -24 * np.abs(Ah)
    assert np.all(E <= bound)


@pytest.mark.parametrize("n,nb", [(512, 128), (2048, 256), (3000, 512)])
@pytest.mark.parametrize("fmt", [0, 1])
def test_mxp_refinement_reaches_fp64(n, nb, fmt):
    h = hpl()
    A, b = gpu_mxp_system(n, 9)
    LU, info = h.hpl_mxp_factor(A, nb=nb, fmt=fmt)
    assert info == 0
    x, out = h.hpl_mxp_solve(A, LU, b, max_iter=50)
    print(f"n={n} fmt={fmt}: {int(out[0])} corrections, scaled residual {out[1]:.3g}")
    assert out[1] < 16.0
    Ah = oracle.mxp_gen(9, n)
    bh = oracle.gen(9, 1, n, 1)[:, 0].copy()
    xh = x.cpu().numpy()
    res = oracle.residual(Ah, xh, bh)
    assert res[0] < 16.0
    LU64 = Ah.copy(order="F")
    ipiv, _ = oracle.lu(LU64)
    xo = bh.copy()
    oracle.solve(LU64, ipiv, xo)
    # refinement stops once the residual test passes (scaled residual < 16),
    # which bounds the error at about scaled * n * eps relative (times the
    # condition number); x is held to the 1e-10 relative tolerance of the FP64 path
    err = np.max(np.abs(xh - xo)) / np.max(np.abs(xo))
    print(f"   |x - x_oracle| / |x_oracle| = {err:.2e}")
    assert err <= 1e-10


def test_mxp_solve_sizes_up_and_down():
    """The refinement keeps its vectors and counters in a workspace that later
    calls reuse: a call on a smaller system after a larger one, and a larger
    one again, must each reach the residual test."""
    h = hpl()
    for n, fmt in ((1500, 0), (300, 1), (700, 0), (1500, 1)):
        A, b = gpu_mxp_system(n, 21)
        LU, info = h.hpl_mxp_factor(A, nb=128, fmt=fmt)
        assert info == 0
        x, out = h.hpl_mxp_solve(A, LU, b, max_iter=50)
        assert out[1] < 16.0, (n, fmt, out)
        res = oracle.residual(oracle.mxp_gen(21, n), x.cpu().numpy(), oracle.gen(21, 1, n, 1)[:, 0].copy())
        assert res[0] < 16.0


def test_mxp_zero_refinements_allowed():
    h = hpl()
    A, b = gpu_mxp_system(300, 3)
    LU, _ = h.hpl_mxp_factor(A, nb=64, fmt=0)
    x, out = h.hpl_mxp_solve(A, LU, b, max_iter=0)
    assert out[0] == 0.0 and out[1] > 0.0


@pytest.mark.parametrize("n,nb", [(256, 64), (2048, 256)])
@pytest.mark.parametrize("la", [0, 1])
def test_mxp_factor_scaling_exact(n, nb, la):
    """The per-panel power-of-two scaling where it changes bits: the first
    panel's FP16 copies of L21 (odd multiples of 2^-30) and U12 (up to 2047 *
    2^27) are exact only for an exponent in [22, 35] (tests/inputs.py), so the
    GPU factors equal the construction's L and U, and the oracle's, bit for
    bit, only if the device computes the scaling exponent as the oracle does."""
    import inputs
    h = hpl()
    A, L, U = inputs.mxp_scaled_lu(n, nb, seed=n + nb)
    LUo, info_o = oracle.lu_mxp(A, nb, 0)
    assert info_o == 0
    old = h.hpl_get_option(h.HPL_OPT_LOOKAHEAD)
    try:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, la)
        LU, info = h.hpl_mxp_factor(to_gpu(A), nb=nb, fmt=0)
    finally:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, old)
    assert info == 0
    G = LU.cpu().numpy()
    assert np.array_equal(G.view(np.int32), np.asfortranarray(LUo).view(np.int32))
    G = G.astype(np.float64)
    assert np.array_equal(np.tril(G, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(G), U)

