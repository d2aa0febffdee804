"""GPU parity tests of the differentiable solve: X = A^{-1} B with the adjoint
grad_B = A^{-T} W, grad_A = -grad_B X^T, through the C ABI (hpl_factor,
hpl_solve with trans = 0/1, hpl_solve_grad_a) and the torch.autograd.Function
of the binding, against the CPU oracle (oracle.solve_grad) and against central
finite differences of the GPU forward at the full workload size."""
import numpy as np
import pytest

import oracle
from golden.load import diffsolve_reference
from gpu_util import hpl, to_gpu, to_host, torch

pytestmark = pytest.mark.gpu

SEED = 2304


def diff_inputs(n, nrhs, seed=SEED, shift=8.0):
    """The workload's inputs: A = U[-0.5, 0.5) + shift*I (stream 0), B (stream 1),
    W standard normal (stream 2), made on the GPU."""
    h = hpl()
    A = h.colmajor(n, n)
    h.hpl_generate(seed, 0, A)
    h.hpl_add_diagonal(A, shift)
    B = h.colmajor(n, nrhs)
    h.hpl_generate(seed, 1, B)
    W = h.colmajor(n, nrhs)
    h.hpl_generate_normal(seed, 2, W)
    return A, B, W


def oracle_inputs(n, nrhs, seed=SEED, shift=8.0):
    A = oracle.gen(seed, 0, n, n).copy(order="F")
    A[np.arange(n), np.arange(n)] += shift
    B = oracle.gen(seed, 1, n, nrhs).copy(order="F")
    W = oracle.gen_normal(seed, 2, n, nrhs).copy(order="F")
    return A, B, W


@pytest.mark.parametrize("rows,cols,ld", [(1, 1, 1), (1000, 17, 1000), (777, 5, 800)])
def test_generate_normal_vs_oracle(rows, cols, ld):
    h = hpl()
    M = h.colmajor(rows, cols, ld=ld)
    h.hpl_generate_normal(99, 2, M)
    ref = oracle.gen_normal(99, 2, rows, cols)
    # device log/cos against the C library's: a few units in the last place
    assert np.max(np.abs(to_host(M) - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_add_diagonal_exact():
    h = hpl()
    n = 300
    M = h.colmajor(n, n, ld=307)
    h.hpl_generate(5, 0, M)
    before = to_host(M)
    h.hpl_add_diagonal(M, 8.0)
    after = to_host(M)
    expect = before.copy()
    expect[np.arange(n), np.arange(n)] += 8.0
    assert np.array_equal(after, expect)


@pytest.mark.parametrize("n,k,ld", [(1, 1, 1), (300, 1, 300), (301, 16, 310), (1000, 17, 1000), (257, 40, 260),
                                    (64, 0, 64)])
def test_grad_a_kernel(n, k, ld):
    h = hpl()
    rng = np.random.default_rng(n + k)
    G = rng.standard_normal((n, k))
    X = rng.standard_normal((n, k))
    Gg, Xg = to_gpu(G, ld=ld), to_gpu(X, ld=ld)
    D = h.colmajor(n, n, ld=ld + 3, fill=float("nan"))
    h.hpl_solve_grad_a(Gg, Xg, D)
    ref = -(G @ X.T) if k else np.zeros((n, n))
    got = to_host(D)
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(got - ref)) <= 1e-14 * k * scale + 0.0
    if k == 0:
        assert not np.any(np.signbit(got))


@pytest.mark.parametrize("n,nrhs,nb", [(64, 1, 32), (300, 4, 64), (1000, 16, 256), (2048, 16, 256)])
def test_diff_solve_vs_oracle(n, nrhs, nb):
    h = hpl()
    A, B, W = diff_inputs(n, nrhs)
    A.requires_grad_(True)
    B.requires_grad_(True)
    X = h.hpl_solve_diff(A, B, nb=nb)
    loss = (X * W).sum()
    loss.backward()
    Ao, Bo, Wo = oracle_inputs(n, nrhs)
    Wg = to_host(W)
    # the device's normal values differ from libm's in the last bits: the oracle
    # takes the GPU's W as its loss weights only if they agree to that level
    assert np.max(np.abs(Wg - Wo)) <= 1e-14 * np.max(np.abs(Wo))
    Xo, GBo, GAo, info = oracle.solve_grad(Ao, Bo, Wo)
    assert info == 0
    for got, ref, name in ((to_host(X.detach()), Xo, "X"), (to_host(B.grad), GBo, "grad_B"),
                           (to_host(A.grad), GAo, "grad_A")):
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"n={n} nrhs={nrhs} {name}: relative max error {err:.2e}")
        assert err <= 1e-10, name


def test_diff_solve_vector_rhs():
    h = hpl()
    n = 200
    A, B, W = diff_inputs(n, 1)
    b = B[:, 0].contiguous().clone().requires_grad_(True)
    w = W[:, 0].contiguous()
    A.requires_grad_(True)
    x = h.hpl_solve_diff(A, b, nb=64)
    assert x.shape == (n,)
    (x * w).sum().backward()
    Ao, Bo, Wo = oracle_inputs(n, 1)
    Xo, GBo, GAo, _ = oracle.solve_grad(Ao, Bo, Wo)
    assert np.max(np.abs(b.grad.cpu().numpy() - GBo[:, 0])) <= 1e-10 * np.max(np.abs(GBo))
    assert np.max(np.abs(to_host(A.grad) - GAo)) <= 1e-10 * np.max(np.abs(GAo))


def test_diff_solve_finite_differences_full_size():
    """N = 8192, NB = 256, 16 right-hand sides: central differences (h = 1e-6) of
    the GPU forward on 64 entries of A and 64 of B against the backward."""
    hp = hpl()
    n, nrhs, nb, hstep = 8192, 16, 256, 1e-6
    A, B, W = diff_inputs(n, nrhs)
    A.requires_grad_(True)
    B.requires_grad_(True)
    X = hp.hpl_solve_diff(A, B, nb=nb)
    (X * W).sum().backward()
    GA, GB = A.grad, B.grad
    l1 = float((X.detach() * W).abs().sum())
    eps = 2.0 ** -53
    rng = np.random.default_rng(8192)
    t = torch()

    def loss_of(Ap, Bp):
        with t.no_grad():
            Xp = hp.hpl_solve_diff(Ap, Bp, nb=nb)
            return float((Xp * W).sum())

    worst = 0.0
    with t.no_grad():
        A0, B0 = A.detach(), B.detach()
        for trial in range(64):
            i, j = int(rng.integers(n)), int(rng.integers(n))
            Ap, Am = A0.clone(), A0.clone()
            Ap[i, j] += hstep
            Am[i, j] -= hstep
            fd = (loss_of(Ap, B0) - loss_of(Am, B0)) / (2 * hstep)
            g = float(GA[i, j])
            worst = max(worst, abs(fd - g) / (eps * l1 / hstep))
            # rounding floor of a central difference: the loss is evaluated to
            # about kappa * eps * sum|W * X|; kappa of A + 8I at this size is
            # O(1e3), so allow 1e4 times eps * sum|W * X| / h
            assert abs(fd - g) <= 1e-6 * abs(g) + 1e4 * eps * l1 / hstep, (i, j, fd, g)
        for trial in range(64):
            i, r = int(rng.integers(n)), int(rng.integers(nrhs))
            Bp, Bm = B0.clone(), B0.clone()
            Bp[i, r] += hstep
            Bm[i, r] -= hstep
            fd = (loss_of(A0, Bp) - loss_of(A0, Bm)) / (2 * hstep)
            g = float(GB[i, r])
            worst = max(worst, abs(fd - g) / (eps * l1 / hstep))
            assert abs(fd - g) <= 1e-6 * abs(g) + 1e4 * eps * l1 / hstep, (i, r, fd, g)
    print(f"finite differences: worst |fd - grad| = {worst:.3g} x eps*sum|W*X|/h (sum|W*X| = {l1:.4g})")


def test_diff_solve_vs_oracle_full_size():
    """N = 8192, NB = 256, 16 right-hand sides (the workload's size) against the
    oracle's X, grad_B and grad_A, precomputed by tests/golden/make_diffsolve_n8192.py
    (oracle only): sampled entries of all three within 1e-10 of the oracle's largest
    entry, every column sum of X and grad_B within 1e-10 of its absolute sum, and
    the largest magnitudes within 1e-10."""
    h = hpl()
    n, nrhs, nb = 8192, 16, 256
    maxabs, colsums, entries = diffsolve_reference("diffsolve_n8192_oracle.txt")
    A, B, W = diff_inputs(n, nrhs)
    A.requires_grad_(True)
    B.requires_grad_(True)
    X = h.hpl_solve_diff(A, B, nb=nb)
    (X * W).sum().backward()
    got = {"X": to_host(X.detach()), "GB": to_host(B.grad)}
    GA = A.grad.detach()
    for name in ("X", "GB"):
        M = got[name]
        assert abs(np.max(np.abs(M)) - maxabs[name]) <= 1e-10 * maxabs[name], name
        for r in range(nrhs):
            s, sa = colsums[(name, r)]
            assert abs(float(np.sum(M[:, r])) - s) <= 1e-10 * sa, (name, r)
        worst = max(abs(M[i, j] - v) for i, j, v in entries[name]) / maxabs[name]
        print(f"N={n} {name}: sampled relative error {worst:.2e}")
        assert worst <= 1e-10, name
    ga_max = float(GA.abs().max())
    assert abs(ga_max - maxabs["GA"]) <= 1e-10 * maxabs["GA"]
    idx = torch().tensor([[i, j] for i, j, _ in entries["GA"]], device="cuda")
    vals = GA[idx[:, 0], idx[:, 1]].cpu().numpy()
    ref = np.array([v for _, _, v in entries["GA"]])
    worst = float(np.max(np.abs(vals - ref))) / maxabs["GA"]
    print(f"N={n} GA: sampled relative error {worst:.2e}")
    assert worst <= 1e-10
