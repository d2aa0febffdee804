"""GPU parity past 2^31 matrix elements (n * lda > 2^31): the 64-bit offset
paths of the panel, the row interchanges, the TRSM, the trailing GEMM and the
solve at N = 47104, NB = 512 (the full-size run's panel width), with the
look-ahead mode the full-size run uses (1).

* Random system (the HPL input): the HPL scaled residual < 16, and look-ahead
  modes 1 and 0 bit-identical (pivots and factors).
* Exact construction A = P^T L U (L multiples of 1/8 with |l| < 1, U integers,
  built on the device by a library FP64 product, exact in any summation order
  because every partial sum is a multiple of 1/8 far below 2^50): the factors,
  pivots and an integer solution come back bit for bit.
"""
import numpy as np
import pytest

from gpu_util import hpl, torch

pytestmark = pytest.mark.gpu

N, NB, SEED = 47104, 512, 2304


@pytest.fixture(scope="module", autouse=True)
def _lookahead_one():
    h = hpl()
    old = h.hpl_get_option(h.HPL_OPT_LOOKAHEAD)
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 1)
    yield
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, old)
    torch().cuda.empty_cache()


def test_offsets_past_2_31():
    assert N * N > 2 ** 31


def test_random_system_residual_and_lookahead_bitwise():
    h = hpl()
    t = torch()
    A1 = h.colmajor(N, N)
    h.hpl_generate(SEED, 0, A1)
    b = h.colmajor(N, 1)
    h.hpl_generate(SEED, 1, b)
    x = b.clone()
    ipiv1, info1 = h.hpl_factor(A1, NB)
    h.hpl_solve(A1, ipiv1, x)
    res = h.hpl_residual_gen(SEED, N, x, b)
    print(f"N={N} NB={NB} look-ahead 1: scaled residual {res[0]:.4g}")
    assert info1 == 0 and res[0] < 16.0
    A0 = h.colmajor(N, N)
    h.hpl_generate(SEED, 0, A0)
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 0)
    try:
        ipiv0, info0 = h.hpl_factor(A0, NB)
    finally:
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 1)
    assert info0 == 0
    assert t.equal(ipiv0, ipiv1)
    assert t.equal(A0.view(t.int64), A1.view(t.int64))
    del A0, A1
    t.cuda.empty_cache()


def test_exact_construction_bitwise():
    h = hpl()
    t = torch()
    g = t.Generator(device="cuda")
    g.manual_seed(47)
    # L unit lower, entries k/8 with |k| <= 7; U upper integers in [-8, 8], nonzero diagonal
    L = t.randint(-7, 8, (N, N), generator=g, device="cuda", dtype=t.int8).to(t.float64).mul_(0.125)
    L.tril_(-1).diagonal().fill_(1.0)
    U = t.randint(-8, 9, (N, N), generator=g, device="cuda", dtype=t.int8).to(t.float64)
    U.triu_(1)
    d = t.randint(1, 9, (N,), generator=g, device="cuda").to(t.float64)
    d *= t.where(t.rand(N, generator=g, device="cuda") < 0.5, -1.0, 1.0)
    U.diagonal().copy_(d)
    perm = t.randperm(N, generator=g, device="cuda")
    LU = t.matmul(L, U)                                  # exact: multiples of 1/8 below 2^19
    A = h.colmajor(N, N)
    A[perm] = LU                                         # row i of L U at row perm[i]
    del LU
    t.cuda.empty_cache()
    xi = t.randint(-9, 10, (N, 3), generator=g, device="cuda").to(t.float64)
    B = h.colmajor(N, 3)
    B.copy_(t.matmul(A, xi))                             # exact integers
    ipiv, info = h.hpl_factor(A, NB)
    assert info == 0
    # pivots: the interchanges reproduce the permutation
    order = np.arange(N)
    for k, p in enumerate(ipiv.cpu().numpy()):
        order[[k, p]] = order[[p, k]]
    assert np.array_equal(order, perm.cpu().numpy())
    # factors, column chunks compared on the device
    rows = t.arange(N, device="cuda")[:, None]
    for j0 in range(0, N, 4096):
        j1 = min(N, j0 + 4096)
        cols = t.arange(j0, j1, device="cuda")[None, :]
        want = t.where(rows > cols, L[:, j0:j1], U[:, j0:j1])
        assert t.equal(A[:, j0:j1], want), f"columns {j0}..{j1}"
    del L, U, want
    h.hpl_solve(A, ipiv, B)
    assert t.equal(B, xi)
    del A, B
    t.cuda.empty_cache()
