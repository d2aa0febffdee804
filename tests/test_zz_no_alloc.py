"""hpl_solve_noalloc (the solve with the library's fixed scratch array, for
callers that cannot allocate) against hpl_solve through the C ABI: the same
kernels in the same order, so the results must be identical bit for bit.
Two calls in a row share the scratch array; the second is smaller, so a plan
or counter left over from the first would show."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import hpl, torch

pytestmark = pytest.mark.gpu


def factored(n, seed):
    h = hpl()
    A = h.colmajor(n, n)
    h.hpl_generate(seed, 0, A)
    ipiv, info = h.hpl_factor(A, 64)
    assert info == 0
    return A, ipiv


def rhs(n, nrhs, seed):
    h = hpl()
    B = h.colmajor(n, nrhs)
    h.hpl_generate(seed, 1, B)
    return B


@pytest.mark.parametrize("first,second", [((1031, 3, 0), (300, 1, 0)),
                                          ((4096, 70, 1), (1000, 5, 1)),
                                          ((2048, 16, 0), (65, 2, 1))])
def test_noalloc_matches_solve_twice(first, second):
    t = torch()
    h = hpl()
    for n, nrhs, trans in (first, second):
        A, ipiv = factored(n, 7 + n)
        B = rhs(n, nrhs, 7 + n)
        X_ref = h.hpl_solve(A, ipiv, B.clone(), trans=trans)
        X_na = h.hpl_solve_noalloc(A, ipiv, B.clone(), trans=trans)
        t.cuda.synchronize()
        assert t.equal(X_na.view(t.int64), X_ref.view(t.int64)), (n, nrhs, trans)
        if n <= 1100 and trans == 0:
            Ao = oracle.gen(7 + n, 0, n, n).copy(order="F")
            Bo = oracle.gen(7 + n, 1, n, nrhs).copy(order="F")
            piv, _ = oracle.lu(Ao)
            oracle.solve(Ao, piv, Bo)
            got = X_na.cpu().numpy()
            assert np.max(np.abs(got - Bo)) <= 1e-10 * np.max(np.abs(Bo))


def test_noalloc_rejects_beyond_max():
    h = hpl()
    L = h.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the size check comes first
    n = h.HPL_SOLVE_NOALLOC_MAX_N + 1
    assert L.hpl_solve_noalloc(fake, fake, fake, 1, n, n, n, 0, None) == -5
    assert b"HPL_SOLVE_NOALLOC_MAX_N" in L.hpl_last_error_detail()


def test_noalloc_no_rhs_and_empty():
    h = hpl()
    A, ipiv = factored(100, 3)
    B = h.colmajor(100, 0)
    h.hpl_solve_noalloc(A, ipiv, B)
    E = h.colmajor(0, 0)
    h.hpl_solve_noalloc(E, torch().empty(0, dtype=torch().int32, device="cuda"), h.colmajor(0, 1))
