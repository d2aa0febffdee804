"""The paper's CPU FACT (hpl_host_panel: T threads over nb-row tiles, recursive
right-looking) against the oracle, on the CPU: the first nb columns of the
oracle's LU with partial pivoting of a square matrix whose leading columns are
the panel (column k's pivot never depends on later columns)."""
import numpy as np
import pytest

import oracle

h = pytest.importorskip("paper_2304_10397_amd.hpl", reason="libhplx.so not built")


def reference(P):
    m, nb = P.shape
    rng = np.random.default_rng(m * 7 + nb)
    S = np.asfortranarray(np.hstack([P, rng.uniform(-0.5, 0.5, (m, m - nb))]))
    ipiv, info = oracle.lu(S)
    R = S[:, :nb].copy(order="F")
    # the square factorization's later interchanges (steps nb..m-1) also moved
    # the rows of these columns (LAPACK form); undo them, last first
    for k in range(m - 1, nb - 1, -1):
        p = int(ipiv[k])
        if p != k:
            R[[k, p], :] = R[[p, k], :]
    return R, ipiv[:nb], info


@pytest.mark.parametrize("m,nb", [(1, 1), (5, 2), (16, 16), (17, 16), (64, 33), (300, 64), (1000, 128), (700, 256)])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_host_panel_vs_oracle(m, nb, threads):
    rng = np.random.default_rng(m + nb)
    P0 = np.asfortranarray(rng.uniform(-0.5, 0.5, (m, nb)))
    P = P0.copy(order="F")
    ipiv, info = h.hpl_host_panel(P, threads)
    R, ipo, info_o = reference(P0)
    assert info == 0 and np.array_equal(ipiv, ipo)
    assert np.max(np.abs(P - R)) <= 1e-12 * max(1.0, np.max(np.abs(R)))


def test_host_panel_dyadic_exact_and_thread_independent():
    rng = np.random.default_rng(9)
    m, nb = 480, 96
    L = np.tril(rng.integers(-4, 5, (m, nb)) / 8.0, -1)
    L[np.arange(nb), np.arange(nb)] = 1.0
    U = np.triu(rng.integers(-7, 8, (nb, nb)).astype(float), 1) + np.diag(2.0 ** rng.integers(2, 4, nb))
    P0 = np.asfortranarray(L @ U)
    outs = []
    for T in (1, 2, 5, 16):
        P = P0.copy(order="F")
        ipiv, info = h.hpl_host_panel(P, T)
        outs.append((P, ipiv))
        R, ipo, _ = reference(P0)
        assert np.array_equal(ipiv, ipo) and np.array_equal(P, R)
    for P, ipiv in outs[1:]:
        assert np.array_equal(P, outs[0][0]) and np.array_equal(ipiv, outs[0][1])


def test_host_panel_zero_column_info():
    rng = np.random.default_rng(3)
    P = np.asfortranarray(rng.uniform(-0.5, 0.5, (50, 20)))
    P[:, 6] = 0.0
    R, ipo, info_o = reference(P.copy(order="F"))
    ipiv, info = h.hpl_host_panel(P, 4)
    assert info == info_o == 7
    assert np.array_equal(ipiv, ipo)


def test_host_panel_argument_errors():
    import ctypes
    L = h.lib()
    info = ctypes.c_int64(0)
    buf = np.zeros(64)
    piv = np.zeros(8, dtype=np.int32)
    pb, pp = buf.ctypes.data_as(ctypes.c_void_p), piv.ctypes.data_as(ctypes.c_void_p)
    assert L.hpl_host_panel(None, 4, 2, 4, pp, 1, ctypes.byref(info)) == -1
    assert L.hpl_host_panel(pb, -1, 2, 4, pp, 1, ctypes.byref(info)) == -2
    assert L.hpl_host_panel(pb, 4, 5, 4, pp, 1, ctypes.byref(info)) == -3
    assert L.hpl_host_panel(pb, 4, 2, 3, pp, 1, ctypes.byref(info)) == -4
    assert L.hpl_host_panel(pb, 4, 2, 4, None, 1, ctypes.byref(info)) == -5
    assert L.hpl_host_panel(pb, 4, 2, 4, pp, 0, ctypes.byref(info)) == -6
    assert L.hpl_host_panel(pb, 4, 2, 4, pp, 1, None) == -7
    assert L.hpl_set_option(8, -1) == -2 and L.hpl_set_option(8, 257) == -2
    assert L.hpl_set_option(8, 0) == 0
