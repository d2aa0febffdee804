"""GPU parity tests of the batched solve (C ABI hpl_batched_solve, one
persistent launch) against the oracle (oracle.batched_solve: per system the
pinned LU with partial pivoting, solve and adjoint)."""
import numpy as np
import pytest

import oracle
from gpu_util import hpl, torch

pytestmark = pytest.mark.gpu

SEED = 2304


def gpu_batch(sizes, nrhs, seed=SEED, adjoint=False):
    """Packed A (stream 0), B (stream 1) and W (normal, stream 2) on the GPU."""
    h, t = hpl(), torch()
    _, _, na, nb = h.batch_layout(sizes, nrhs)
    A = t.empty(max(na, 1), dtype=t.float64, device="cuda")
    B = t.empty(max(nb, 1), dtype=t.float64, device="cuda")
    h.hpl_generate(seed, 0, A)
    h.hpl_generate(seed, 1, B)
    W = GB = GA = None
    if adjoint:
        W = t.empty(max(nb, 1), dtype=t.float64, device="cuda")
        h.hpl_generate_normal(seed, 2, W)
        GB = t.full((max(nb, 1),), float("nan"), dtype=t.float64, device="cuda")
        GA = t.full((max(na, 1),), float("nan"), dtype=t.float64, device="cuda")
    ipiv = t.full((max(int(np.sum(sizes)), 1),), -7, dtype=t.int32, device="cuda")
    return A, B, W, GB, GA, ipiv


def host_batch(sizes, nrhs, seed=SEED, adjoint=False):
    _, _, na, nb = hpl().batch_layout(sizes, nrhs)
    A = oracle.gen(seed, 0, max(na, 1), 1)[:na, 0].copy()
    B = oracle.gen(seed, 1, max(nb, 1), 1)[:nb, 0].copy()
    W = oracle.gen_normal(seed, 2, max(nb, 1), 1)[:nb, 0].copy() if adjoint else None
    return A, B, W


def rel(got, ref):
    return np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)


def check_against_oracle(sizes, nrhs, out_gpu, ref, systems=None):
    aoff, voff = oracle.batch_offsets(sizes, nrhs)
    LU, ipiv, X, GB, GA = out_gpu
    for i in (range(len(sizes)) if systems is None else systems):
        n = int(sizes[i])
        a0, a1 = aoff[i], aoff[i] + n * n
        v0, v1 = nrhs * voff[i], nrhs * voff[i] + n * nrhs
        assert np.array_equal(ipiv[voff[i]:voff[i] + n], ref["ipiv"][voff[i]:voff[i] + n]), (i, n)
        assert rel(LU[a0:a1], ref["LU"][a0:a1]) <= 1e-11, (i, n)
        assert rel(X[v0:v1], ref["X"][v0:v1]) <= 1e-10, (i, n)
        if GB is not None:
            assert rel(GB[v0:v1], ref["GB"][v0:v1]) <= 1e-10, (i, n)
            assert rel(GA[a0:a1], ref["GA"][a0:a1]) <= 1e-10, (i, n)


def test_generated_batch_matches_oracle_inputs():
    sizes = hpl().hpl_batched_sizes(11, 20, 1, 40)
    A, B, W, _, _, _ = gpu_batch(sizes, 3, seed=11, adjoint=True)
    Ah, Bh, Wh = host_batch(sizes, 3, seed=11, adjoint=True)
    assert np.array_equal(A.cpu().numpy()[:Ah.size], Ah)
    assert np.array_equal(B.cpu().numpy()[:Bh.size], Bh)
    assert np.max(np.abs(W.cpu().numpy()[:Wh.size] - Wh)) <= 1e-14 * np.max(np.abs(Wh))


@pytest.mark.parametrize("nrhs", [1, 4, 16])
def test_forward_vs_oracle(nrhs):
    h = hpl()
    sizes = np.concatenate([np.array([1, 2, 31, 32, 33, 63, 64, 65, 97], dtype=np.int32),
                            h.hpl_batched_sizes(5, 30, 1, 130)])
    A, B, _, _, _, ipiv = gpu_batch(sizes, nrhs)
    info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, mode=h.BATCH_FORWARD)
    assert np.all(info == 0)
    Ah, Bh, _ = host_batch(sizes, nrhs)
    ref = oracle.batched_solve(sizes, Ah, Bh, nrhs)
    check_against_oracle(sizes, nrhs, (A.cpu().numpy(), ipiv.cpu().numpy(), B.cpu().numpy(), None, None), ref)


@pytest.mark.parametrize("nrhs", [1, 4])
def test_forward_and_adjoint_vs_oracle(nrhs):
    h = hpl()
    sizes = np.concatenate([np.array([1, 3, 32, 33, 100], dtype=np.int32), h.hpl_batched_sizes(6, 24, 1, 160)])
    A, B, W, GB, GA, ipiv = gpu_batch(sizes, nrhs, adjoint=True)
    info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, W=W, GB=GB, GA=GA, mode=h.BATCH_BOTH)
    assert np.all(info == 0)
    Ah, Bh, Wh = host_batch(sizes, nrhs, adjoint=True)
    # the device's normal values differ from libm's in the last bits: the oracle
    # takes the GPU's W, which agrees with its own to 1e-14
    Wg = W.cpu().numpy()[:Wh.size]
    assert np.max(np.abs(Wg - Wh)) <= 1e-14 * np.max(np.abs(Wh))
    ref = oracle.batched_solve(sizes, Ah, Bh, nrhs, W=Wg)
    check_against_oracle(sizes, nrhs, (A.cpu().numpy(), ipiv.cpu().numpy(), B.cpu().numpy(), GB.cpu().numpy(),
                                       GA.cpu().numpy()), ref)


def test_adjoint_only_matches_fused():
    """mode 1 then mode 2 (from the stored factors and X) gives the bits of mode 3."""
    h = hpl()
    sizes = h.hpl_batched_sizes(8, 40, 1, 200)
    nrhs = 4
    A, B, W, GB, GA, ipiv = gpu_batch(sizes, nrhs, adjoint=True)
    A2, B2, ipiv2 = A.clone(), B.clone(), ipiv.clone()
    GB2, GA2 = GB.clone(), GA.clone()
    h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, W=W, GB=GB, GA=GA, mode=h.BATCH_BOTH)
    h.hpl_batched_solve(sizes, A2, ipiv2, B2, nrhs, mode=h.BATCH_FORWARD)
    h.hpl_batched_solve(sizes, A2, ipiv2, B2, nrhs, W=W, GB=GB2, GA=GA2, mode=h.BATCH_ADJOINT)
    for x, y in ((A, A2), (B, B2), (GB, GB2), (GA, GA2)):
        assert np.array_equal(x.cpu().numpy().view(np.int64), y.cpu().numpy().view(np.int64))
    assert np.array_equal(ipiv.cpu().numpy(), ipiv2.cpu().numpy())


def test_max_size_and_singular_systems():
    h, t = hpl(), torch()
    sizes = np.array([512, 40, 7, 512, 33], dtype=np.int32)
    nrhs = 2
    A, B, W, GB, GA, ipiv = gpu_batch(sizes, nrhs, adjoint=True)
    aoff, voff = oracle.batch_offsets(sizes, nrhs)
    # system 1: column 5 zero; system 2: column 0 zero
    Ah, Bh, _ = host_batch(sizes, nrhs)
    for i, c in ((1, 5), (2, 0)):
        n = int(sizes[i])
        Ah[aoff[i] + c * n:aoff[i] + (c + 1) * n] = 0.0
    A.copy_(t.from_numpy(np.concatenate([Ah, np.zeros(A.numel() - Ah.size)])).cuda())
    info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, mode=h.BATCH_FORWARD)
    ref = oracle.batched_solve(sizes, Ah, Bh, nrhs)
    assert list(info) == list(ref["info"]) == [0, 6, 1, 0, 0]
    check_against_oracle(sizes, nrhs, (A.cpu().numpy(), ipiv.cpu().numpy(), B.cpu().numpy(), None, None), ref,
                         systems=[0, 3, 4])
    # the singular systems' factors (no solve comparison: X is inf/nan there)
    LUg = A.cpu().numpy()
    for i in (1, 2):
        a0, a1 = aoff[i], aoff[i] + int(sizes[i]) ** 2
        assert np.array_equal(ipiv.cpu().numpy()[voff[i]:voff[i] + sizes[i]], ref["ipiv"][voff[i]:voff[i] + sizes[i]])
        assert rel(LUg[a0:a1], ref["LU"][a0:a1]) <= 1e-11


def test_empty_batch():
    h, t = hpl(), torch()
    z = t.zeros(1, dtype=t.float64, device="cuda")
    info = h.hpl_batched_solve(np.zeros(0, np.int32), z, t.zeros(1, dtype=t.int32, device="cuda"), z, 1)
    assert info.size == 0


def test_full_size_batch_residuals_and_sampled_oracle():
    """4096 systems, n ~ U{32..512}, 4 right-hand sides, factor + solve + adjoint in one
    launch: every system's scaled residual, and 6 systems against the oracle."""
    h = hpl()
    sizes = h.hpl_batched_sizes(SEED, 4096, 32, 512)
    nrhs = 4
    A, B, W, GB, GA, ipiv = gpu_batch(sizes, nrhs, adjoint=True)
    info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, W=W, GB=GB, GA=GA, mode=h.BATCH_BOTH)
    assert np.all(info == 0)
    Ah, Bh, _ = host_batch(sizes, nrhs)
    X = B.cpu().numpy()
    aoff, voff = oracle.batch_offsets(sizes, nrhs)
    eps = 2.0 ** -53
    worst = 0.0
    for i, n in enumerate(sizes):
        Ai = Ah[aoff[i]:aoff[i] + n * n].reshape((n, n), order="F")
        Xi = X[nrhs * voff[i]:nrhs * voff[i] + n * nrhs].reshape((n, nrhs), order="F")
        Bi = Bh[nrhs * voff[i]:nrhs * voff[i] + n * nrhs].reshape((n, nrhs), order="F")
        r = np.max(np.abs(Ai @ Xi - Bi)) / (eps * (np.max(np.abs(Ai).sum(1)) * np.max(np.abs(Xi)) + np.max(np.abs(Bi))) * n)
        worst = max(worst, r)
    print(f"worst scaled residual over 4096 systems: {worst:.3g}")
    assert worst < 16.0
    order = np.argsort(sizes)
    sample = [int(order[0]), int(order[1]), int(order[2048]), int(order[-1]), 17, 4000]
    Wg = W.cpu().numpy()
    for i in sample:
        n = int(sizes[i])
        sub = np.array([n], dtype=np.int32)
        ref = oracle.batched_solve(sub, Ah[aoff[i]:aoff[i] + n * n], Bh[nrhs * voff[i]:nrhs * voff[i] + n * nrhs],
                                   nrhs, W=Wg[nrhs * voff[i]:nrhs * voff[i] + n * nrhs])
        LUg = A.cpu().numpy()[aoff[i]:aoff[i] + n * n]
        assert np.array_equal(ipiv.cpu().numpy()[voff[i]:voff[i] + n], ref["ipiv"]), (i, n)
        assert rel(LUg, ref["LU"]) <= 1e-11, (i, n)
        assert rel(X[nrhs * voff[i]:nrhs * voff[i] + n * nrhs], ref["X"]) <= 1e-10, (i, n)
        assert rel(GB.cpu().numpy()[nrhs * voff[i]:nrhs * voff[i] + n * nrhs], ref["GB"]) <= 1e-10, (i, n)
        assert rel(GA.cpu().numpy()[aoff[i]:aoff[i] + n * n], ref["GA"]) <= 1e-10, (i, n)


CONFIGS = [(occ, v) for occ in (1, 2) for v in range(4)]


@pytest.mark.parametrize("occ,v", CONFIGS)
def test_every_schedule_vs_oracle(occ, v):
    """Every schedule the tuner can choose (systems per CU occ, variant v: panel
    width and U12 stage width), forced for the whole batch: factor + solve +
    adjoint in one launch against the oracle, on sizes that straddle the panel
    widths (16, 32), the solves' row blocks and the update's stage widths."""
    h = hpl()
    sizes = np.concatenate([np.array([1, 2, 15, 16, 17, 31, 32, 33, 48, 64, 65, 100, 130, 200, 257, 512],
                                     dtype=np.int32), h.hpl_batched_sizes(9, 20, 1, 300)])
    nrhs = 4
    A, B, W, GB, GA, ipiv = gpu_batch(sizes, nrhs, adjoint=True)
    h.hpl_set_option(h.HPL_OPT_BATCH_CONFIG, 1 + (occ - 1) * h.HPL_BATCH_VARIANTS + v)
    try:
        info = h.hpl_batched_solve(sizes, A, ipiv, B, nrhs, W=W, GB=GB, GA=GA, mode=h.BATCH_BOTH)
    finally:
        h.hpl_set_option(h.HPL_OPT_BATCH_CONFIG, 0)
    assert np.all(info == 0)
    Ah, Bh, Wh = host_batch(sizes, nrhs, adjoint=True)
    Wg = W.cpu().numpy()[:Wh.size]
    ref = oracle.batched_solve(sizes, Ah, Bh, nrhs, W=Wg)
    check_against_oracle(sizes, nrhs, (A.cpu().numpy(), ipiv.cpu().numpy(), B.cpu().numpy(), GB.cpu().numpy(),
                                       GA.cpu().numpy()), ref)
