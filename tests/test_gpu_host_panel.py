"""GPU tests of the FACT variants: hpl_panel_factor (the GPU panel alone) against
the oracle, and hpl_factor with the panel factored on the host
(HPL_OPT_HOST_PANEL, the paper's CPU FACT) against the oracle, with and
without the look-ahead."""
import numpy as np
import pytest

import oracle
from gpu_util import hpl, to_gpu, to_host
from test_host_panel import reference

pytestmark = pytest.mark.gpu

SEED = 2304


@pytest.fixture(autouse=True)
def _restore_options():
    h = hpl()
    saved = {k: h.hpl_get_option(k) for k in (h.HPL_OPT_HOST_PANEL, h.HPL_OPT_LOOKAHEAD)}
    yield
    for k, v in saved.items():
        h.hpl_set_option(k, v)


@pytest.mark.parametrize("m,nb", [(64, 32), (1000, 64), (3000, 256), (2048, 512), (1031, 1024)])
def test_gpu_panel_vs_oracle(m, nb):
    h = hpl()
    rng = np.random.default_rng(m + nb)
    P0 = np.asfortranarray(rng.uniform(-0.5, 0.5, (m, nb)))
    A = to_gpu(P0)
    ipiv, info = h.hpl_panel_factor(A)
    R, ipo, _ = reference(P0)
    assert info == 0
    assert np.array_equal(ipiv.cpu().numpy(), ipo)
    assert np.max(np.abs(to_host(A) - R)) <= 1e-12 * max(1.0, np.max(np.abs(R)))


@pytest.mark.parametrize("n,nb", [(1000, 64), (2048, 256), (3001, 512)])
@pytest.mark.parametrize("lookahead", [0, 1])
def test_factor_with_host_panel_vs_oracle(n, nb, lookahead):
    h = hpl()
    A0 = oracle.gen(SEED, 0, n, n).copy(order="F")
    b0 = oracle.gen(SEED, 1, n, 1)[:, 0].copy()
    LU_o = A0.copy(order="F")
    ipiv_o, info_o = oracle.lu(LU_o)
    x_o = b0.copy()
    oracle.solve(LU_o, ipiv_o, x_o)
    h.hpl_set_option(h.HPL_OPT_HOST_PANEL, 4)
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, lookahead)
    A = h.colmajor(n, n)
    h.hpl_generate(SEED, 0, A)
    b = h.colmajor(n, 1)
    h.hpl_generate(SEED, 1, b)
    ipiv, info = h.hpl_factor(A, nb)
    assert info == info_o == 0
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_o)
    LU = to_host(A)
    assert np.max(np.abs(LU - LU_o)) <= 1e-11 * max(1.0, np.max(np.abs(LU_o)))
    h.hpl_solve(A, ipiv, b)
    x = b.cpu().numpy()[:, 0]
    assert np.max(np.abs(x - x_o)) <= 1e-10 * np.max(np.abs(x_o))
    res = h.hpl_residual(to_gpu(A0), b, to_gpu(b0))
    assert res[0] < 16.0


def test_host_panel_thread_count_and_lookahead_bitwise():
    """The host panel's arithmetic does not depend on T, and the look-ahead
    only reorders independent work: identical bits."""
    h = hpl()
    n, nb = 1500, 128
    outs = []
    for T, la in ((1, 1), (8, 1), (3, 0)):
        h.hpl_set_option(h.HPL_OPT_HOST_PANEL, T)
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, la)
        A = h.colmajor(n, n)
        h.hpl_generate(SEED, 0, A)
        ipiv, info = h.hpl_factor(A, nb)
        outs.append((to_host(A).view(np.int64), ipiv.cpu().numpy()))
    for LU, piv in outs[1:]:
        assert np.array_equal(LU, outs[0][0]) and np.array_equal(piv, outs[0][1])


def test_host_panel_singular_info():
    h = hpl()
    n, nb = 300, 64
    A0 = oracle.gen(SEED, 0, n, n).copy(order="F")
    A0[:, 100] = 0.0
    LU_o = A0.copy(order="F")
    _, info_o = oracle.lu(LU_o)
    h.hpl_set_option(h.HPL_OPT_HOST_PANEL, 2)
    A = to_gpu(A0)
    _, info = h.hpl_factor(A, nb)
    assert info == info_o == 101
