"""Pins of the oracle's mixed-precision pieces (CPU only).

round_fp16 / round_bf16 are checked against independent implementations
(numpy's float16 conversion, torch's CPU bfloat16 conversion).  mxp_gen is
checked for strict diagonal dominance and against the uniform generator.
lu_mxp is pinned by exact dyadic factorizations (every intermediate value is
representable in the formats, so L and U come back exactly), by the
elementwise backward-error bound |A - LU| <= c n u |L||U| with the format's
unit roundoff u, and by agreement with the partial-pivoting oracle (which
makes no interchange on these inputs) in the unrounded format.
"""
import os

import numpy as np
import pytest

import inputs
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_round_fp16_matches_numpy():
    rng = np.random.default_rng(1)
    xs = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-9, 6, 20000),
        np.array([0.0, -0.0, 1.0, 65504.0, 65519.0, 65520.0, 70000.0, -65520.0, 2.0 ** -24, 2.0 ** -25,
                  3 * 2.0 ** -25, 2.0 ** -14, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 6.1e-5, 5.96e-8], dtype=np.float32),
    ]).astype(np.float32)
    ref = xs.astype(np.float16).astype(np.float32)
    got = np.array([oracle.round_fp16(x) for x in xs], dtype=np.float32)
    same = (got == ref) | (np.isinf(got) & np.isinf(ref) & (np.sign(got) == np.sign(ref)))
    assert np.all(same), xs[~same][:5]


def test_round_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(2)
    xs = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 20000),
        np.array([0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, -3.0e38], dtype=np.float32),
    ]).astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.round_bf16(x) for x in xs], dtype=np.float32)
    same = (got == ref) | (np.isinf(got) & np.isinf(ref))
    assert np.all(same), xs[~same][:5]


def test_mxp_gen_dominant():
    n = 300
    A = oracle.mxp_gen(7, n)
    U = oracle.gen(7, 0, n, n)
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(A[off], U[off])
    offsum = np.sum(np.abs(A) * off, axis=1)
    assert np.all(np.diag(A) > offsum)
    assert np.allclose(np.diag(A), offsum + np.abs(np.diag(U)), rtol=1e-13, atol=0)


def dyadic_lu(n, seed):
    """A = L U with every value exact in FP16, BF16 and FP32 and every product
    and partial sum exact in FP32: L unit lower with entries in {-1/2..1/2} step
    1/8, U upper with integer entries |u| <= 7 and power-of-two diagonal."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-4, 5, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-7, 8, (n, n)).astype(float), 1) + np.diag(2.0 ** rng.integers(0, 3, n))
    return np.asfortranarray(L @ U), L, U


@pytest.mark.parametrize("n,nb", [(5, 2), (24, 8), (40, 16), (64, 64)])
@pytest.mark.parametrize("fmt", [oracle.FMT_FP16, oracle.FMT_BF16, oracle.FMT_NONE])
def test_lu_mxp_dyadic_exact(n, nb, fmt):
    A, L, U = dyadic_lu(n, n + nb)
    LU, info = oracle.lu_mxp(A, nb, fmt)
    assert info == 0
    LU = LU.astype(np.float64)
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(LU), U)


@pytest.mark.parametrize("fmt,u", [(oracle.FMT_FP16, 2.0 ** -11), (oracle.FMT_BF16, 2.0 ** -8),
                                   (oracle.FMT_NONE, 2.0 ** -24)])
@pytest.mark.parametrize("n,nb", [(96, 32), (200, 64)])
def test_lu_mxp_backward_error(fmt, u, n, nb):
    A = oracle.mxp_gen(3, n)
    LU, info = oracle.lu_mxp(A, nb, fmt)
    assert info == 0
    LU = LU.astype(np.float64)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    E = np.abs(A - L @ U)
    bound = 2.0 * n * u * (np.abs(L) @ np.abs(U)) + 4.0 * 2.0 ** -24 * np.abs(A)
    assert np.all(E <= bound)
    # and it is not trivially loose: the worst element uses a fair share of it
    if fmt != oracle.FMT_NONE:
        assert np.max(E / bound) > 1e-4


def test_lu_mxp_unrounded_agrees_with_pivoting_oracle():
    n = 150
    A = oracle.mxp_gen(5, n)
    LU64 = A.copy(order="F")
    ipiv, info = oracle.lu(LU64)
    assert info == 0 and np.array_equal(ipiv, np.arange(n))  # diagonal dominance: no interchange
    LU32, info32 = oracle.lu_mxp(A, 32, oracle.FMT_NONE)
    assert info32 == 0
    assert np.max(np.abs(LU32 - LU64)) <= 1e-5 * np.max(np.abs(LU64))


@pytest.mark.parametrize("n,nb", [(96, 32), (256, 64)])
def test_lu_mxp_scaling_exchanges_exponents(n, nb):
    """The per-panel power-of-two scaling, where it changes bits: the first
    panel's multipliers lie below FP16's normal range (odd multiples of 2^-30)
    and its U block row above FP16's largest value (odd multiples of 2^27, up
    to 2047 * 2^27).  Only an exponent s in [22, 35] makes both FP16 copies
    exact (the construction's docstring); the oracle must reproduce L and U bit
    for bit in FP16, which an unscaled, sign-flipped or doubled s cannot."""
    A, L, U = inputs.mxp_scaled_lu(n, nb, seed=n + nb)
    L21, U12 = L[nb:, :nb], U[:nb, nb:]
    # the construction is sensitive to the exponent: exact only inside the window
    for s in range(-60, 61):
        exact = inputs.fp16_exact(L21 * 2.0 ** s) and inputs.fp16_exact(U12 * 2.0 ** -s)
        assert exact == (22 <= s <= 35), s
    # the scaling rule's exponent (half the difference of the maxima's binary
    # exponents, rounded away from zero) falls in the window: frexp gives
    # e_L = -19 and e_U = 38, so s = 29, while -29, 0, 58 and 14 do not
    LU, info = oracle.lu_mxp(A, nb, oracle.FMT_FP16)
    assert info == 0
    LU = LU.astype(np.float64)
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(LU), U)
    # unrounded (FP32 only) the same factors come back: the construction itself is exact in FP32
    LU32, _ = oracle.lu_mxp(A, nb, oracle.FMT_NONE)
    assert np.array_equal(LU32.astype(np.float64), LU)


@pytest.mark.parametrize("mutation", ["-mxp_scale_exponent(lmax, umax)", "0", "2 * mxp_scale_exponent(lmax, umax)",
                                      "mxp_scale_exponent(lmax, umax) / 2"])
def test_scaling_pin_catches_planted_mistakes(mutation, tmp_path):
    """The scaling pin above is not blind: copies of the oracle with the
    exponent's sign flipped, the scaling dropped, doubled or halved (built from
    the oracle's source with that one line changed, here on the CPU) no longer
    reproduce the exact factors of the construction."""
    import ctypes
    import subprocess
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    line = "const int s = mxp_scale_exponent(lmax, umax);"
    assert src.count(line) == 1
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(line, f"const int s = {mutation};"))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                           "-o", str(lib), str(mutated), "-lm"])
    L_ = ctypes.CDLL(str(lib))
    L_.oracle_lu_mxp.restype = ctypes.c_int64
    L_.oracle_lu_mxp.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_int64]
    n, nb = 96, 32
    A, L, U = inputs.mxp_scaled_lu(n, nb, seed=n + nb)
    A = np.asfortranarray(A)
    LU = np.zeros((n, n), dtype=np.float32, order="F")
    L_.oracle_lu_mxp(A.ctypes.data_as(ctypes.c_void_p), n, n, nb, oracle.FMT_FP16,
                     LU.ctypes.data_as(ctypes.c_void_p), n)
    LU = LU.astype(np.float64)
    exact = np.array_equal(np.tril(LU, -1) + np.eye(n), L) and np.array_equal(np.triu(LU), U)
    assert not exact, mutation
