"""CPU oracle for the HPL hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  The GPU library never imports, links or calls it, and this package
never imports the GPU library.

Thin ctypes wrappers over oracle/liboracle.so (plain C, fp64, see oracle.c for
the passages of the paper each function follows).  Matrices are numpy float64
arrays in Fortran (column-major) order; lda is taken from the array's strides.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i64, u64, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        P = ctypes.c_void_p
        L.oracle_splitmix64_at.restype = u64
        L.oracle_splitmix64_at.argtypes = [u64, u64]
        L.oracle_stream_key.restype = u64
        L.oracle_stream_key.argtypes = [u64, u64]
        L.oracle_uniform.restype = dbl
        L.oracle_uniform.argtypes = [u64, u64]
        L.oracle_gen.restype = None
        L.oracle_gen.argtypes = [u64, u64, P, i64, i64, i64]
        L.oracle_lu.restype = None
        L.oracle_lu.argtypes = [P, i64, i64, P, P]
        L.oracle_lu_par.restype = ctypes.c_int
        L.oracle_lu_par.argtypes = [P, i64, i64, P, P, ctypes.c_int]
        L.oracle_solve.restype = None
        L.oracle_solve.argtypes = [P, P, P, i64, i64, i64, i64, ctypes.c_int]
        L.oracle_residual.restype = None
        L.oracle_residual.argtypes = [P, i64, i64, P, i64, P, i64, i64, P]
        L.oracle_residual_gen.restype = None
        L.oracle_residual_gen.argtypes = [u64, i64, P, i64, P, i64, i64, P]
        L.oracle_normal.restype = dbl
        L.oracle_normal.argtypes = [u64, u64]
        L.oracle_gen_normal.restype = None
        L.oracle_gen_normal.argtypes = [u64, u64, P, i64, i64, i64]
        L.oracle_solve_grad.restype = i64
        L.oracle_solve_grad.argtypes = [P, i64, i64, P, i64, i64, P, i64, P, i64, P, i64, P, i64]
        L.oracle_solve_grad_par.restype = i64
        L.oracle_solve_grad_par.argtypes = [P, i64, i64, P, i64, i64, P, i64, P, i64, P, i64, P, i64,
                                            ctypes.c_int]
        L.oracle_mxp_gen.restype = None
        L.oracle_mxp_gen.argtypes = [u64, P, i64, i64]
        L.oracle_round_fp16.restype = ctypes.c_float
        L.oracle_round_fp16.argtypes = [ctypes.c_float]
        L.oracle_round_bf16.restype = ctypes.c_float
        L.oracle_round_bf16.argtypes = [ctypes.c_float]
        L.oracle_lu_mxp.restype = i64
        L.oracle_lu_mxp.argtypes = [P, i64, i64, i64, ctypes.c_int, P, i64]
        L.oracle_det.restype = None
        L.oracle_det.argtypes = [P, P, i64, i64, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ld(a):
    """Leading dimension of a Fortran-ordered 2-D float64 array (or 1-D vector)."""
    if a.ndim == 1 or a.size == 0 or a.shape[0] == 1:
        return max(1, a.shape[0])   # one row: the row stride is never used
    assert a.strides[0] == a.itemsize, "matrix must be column-major (Fortran order)"
    return max(1, a.strides[1] // a.itemsize, a.shape[0])


def _check(a, dtype=np.float64):
    assert isinstance(a, np.ndarray) and a.dtype == dtype
    if a.ndim == 2 and a.size > 0 and a.shape[0] > 1:
        assert a.strides[0] == a.itemsize, "matrix must be column-major (Fortran order)"
    return a


def splitmix64_at(s0: int, idx: int) -> int:
    return int(lib().oracle_splitmix64_at(s0 & (2**64 - 1), idx & (2**64 - 1)))


def stream_key(seed: int, stream: int) -> int:
    return int(lib().oracle_stream_key(seed & (2**64 - 1), stream & (2**64 - 1)))


def gen(seed: int, stream: int, rows: int, cols: int, ld: int = None) -> np.ndarray:
    """rows x cols Fortran-ordered matrix (leading dimension ld >= rows) of the stream."""
    ld = rows if ld is None else ld
    buf = np.zeros((ld, cols), dtype=np.float64, order="F")
    lib().oracle_gen(seed, stream, _ptr(buf), rows, cols, max(ld, 1))
    return buf[:rows, :]


def lu(A: np.ndarray):
    """In-place LU with partial pivoting of a square column-major A; returns (ipiv, info)."""
    _check(A)
    n = A.shape[0]
    assert A.shape[1] == n
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    info = ctypes.c_int64(0)
    lib().oracle_lu(_ptr(A), n, _ld(A), _ptr(ipiv), ctypes.byref(info))
    return ipiv[:n], int(info.value)


def lu_par(A: np.ndarray, threads: int):
    """lu() on `threads` host threads (the rank-1 update's columns split among
    them); bitwise the same result.  Returns (ipiv, info, threads that took part)."""
    _check(A)
    n = A.shape[0]
    assert A.shape[1] == n
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    info = ctypes.c_int64(0)
    used = lib().oracle_lu_par(_ptr(A), n, _ld(A), _ptr(ipiv), ctypes.byref(info), int(threads))
    if used < 1:
        raise RuntimeError("oracle_lu_par could not start its threads")
    return ipiv[:n], int(info.value), int(used)


def solve(LU: np.ndarray, ipiv: np.ndarray, B: np.ndarray, trans: int = 0):
    """In-place solve A X = B (trans=0) or A^T X = B (trans=1) with the factors of A."""
    _check(LU)
    n = LU.shape[0]
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    if B.ndim == 1:
        assert B.flags.c_contiguous and B.dtype == np.float64
        nrhs, ldb = 1, max(n, 1)
    else:
        _check(B)
        nrhs, ldb = B.shape[1], _ld(B)
    lib().oracle_solve(_ptr(LU), _ptr(ipiv), _ptr(B), n, _ld(LU), nrhs, ldb, int(trans))
    return B


def residual(A, X, B):
    """[scaled, ||r||inf, ||A||inf, ||x||inf, ||b||inf] for A X = B (A given)."""
    _check(A)
    n = A.shape[0]
    X2 = X.reshape(n, -1, order="F") if X.ndim == 1 else X
    B2 = B.reshape(n, -1, order="F") if B.ndim == 1 else B
    out = np.zeros(5)
    lib().oracle_residual(_ptr(A), n, _ld(A), _ptr(X2), _ld(X2), _ptr(B2), _ld(B2),
                          X2.shape[1], _ptr(out))
    return out


def residual_gen(seed, n, X, B):
    """Same as residual() with A regenerated from (seed, stream 0)."""
    X2 = X.reshape(n, -1, order="F") if X.ndim == 1 else X
    B2 = B.reshape(n, -1, order="F") if B.ndim == 1 else B
    out = np.zeros(5)
    lib().oracle_residual_gen(seed, n, _ptr(X2), _ld(X2), _ptr(B2), _ld(B2), X2.shape[1],
                              _ptr(out))
    return out


def det(LU, ipiv):
    """(sign, log2|det|, plain product) from the factors."""
    n = LU.shape[0]
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    s, l2, ex = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().oracle_det(_ptr(LU), _ptr(ipiv), n, _ld(LU), ctypes.byref(s), ctypes.byref(l2),
                     ctypes.byref(ex))
    return s.value, l2.value, ex.value


def uniform(s0: int, idx: int) -> float:
    """Value of linear index idx of the stream whose SplitMix64 state is s0."""
    return float(lib().oracle_uniform(s0 & (2**64 - 1), idx & (2**64 - 1)))


def normal(s0: int, idx: int) -> float:
    """Box-Muller standard normal value of linear index idx of the stream with state s0."""
    return float(lib().oracle_normal(s0 & (2**64 - 1), idx & (2**64 - 1)))


def gen_normal(seed: int, stream: int, rows: int, cols: int, ld: int = None) -> np.ndarray:
    """rows x cols Fortran-ordered matrix of standard normal values of the stream."""
    ld = rows if ld is None else ld
    buf = np.zeros((ld, cols), dtype=np.float64, order="F")
    lib().oracle_gen_normal(seed, stream, _ptr(buf), rows, cols, max(ld, 1))
    return buf[:rows, :]


def solve_grad(A, B, W, threads: int = 1):
    """(X, grad_B, grad_A, info) for X = A^{-1} B and the loss sum(W * X).  With
    threads > 1 the factorization runs on that many host threads (bitwise the
    same factors, hence the same results)."""
    _check(A)
    n = A.shape[0]
    B = np.asfortranarray(B.reshape(n, -1), dtype=np.float64)
    W = np.asfortranarray(W.reshape(n, -1), dtype=np.float64)
    nrhs = B.shape[1]
    X = np.zeros((n, nrhs), order="F")
    GB = np.zeros((n, nrhs), order="F")
    GA = np.zeros((n, n), order="F")
    args = (_ptr(A), n, _ld(A), _ptr(B), _ld(B), nrhs, _ptr(W), _ld(W),
            _ptr(X), max(n, 1), _ptr(GB), max(n, 1), _ptr(GA), max(n, 1))
    if threads > 1:
        info = lib().oracle_solve_grad_par(*args, int(threads))
    else:
        info = lib().oracle_solve_grad(*args)
    return X, GB, GA, int(info)


def mxp_gen(seed: int, n: int, ld: int = None) -> np.ndarray:
    """The diagonally dominant mixed-precision input: U[-0.5, 0.5) (stream 0), then
    a_ii = sum_j |a_ij| of the generated row."""
    ld = n if ld is None else ld
    buf = np.zeros((max(ld, 1), n), dtype=np.float64, order="F")
    lib().oracle_mxp_gen(seed, _ptr(buf), n, max(ld, 1))
    return buf[:n, :]


def round_fp16(x: float) -> float:
    return float(lib().oracle_round_fp16(float(x)))


def round_bf16(x: float) -> float:
    return float(lib().oracle_round_bf16(float(x)))


FMT_FP16, FMT_BF16, FMT_NONE = 0, 1, 2


def lu_mxp(A: np.ndarray, nb: int, fmt: int):
    """(LU float32 Fortran n x n, info): no-pivot LU in the mixed precision of the method."""
    _check(A)
    n = A.shape[0]
    LU = np.zeros((max(n, 1), n), dtype=np.float32, order="F")
    info = lib().oracle_lu_mxp(_ptr(A), n, _ld(A), int(nb), int(fmt), _ptr(LU), max(n, 1))
    return LU[:n, :], int(info)


# ---------------------------------------------------------------------------
# Batches of independent small systems (packed column-major, leading dimension
# n_i): A_i at sum_{j<i} n_j^2, B_i / W_i / X_i / grad_B_i at nrhs sum_{j<i} n_j.
# ---------------------------------------------------------------------------
BATCH_SIZE_STREAM = 3


def batched_sizes(seed: int, count: int, nmin: int, nmax: int) -> np.ndarray:
    """n_i = nmin + min(floor(u_i (nmax - nmin + 1)), nmax - nmin), u_i = value(seed, stream 3, i) + 1/2."""
    v = gen(seed, BATCH_SIZE_STREAM, count, 1)[:, 0]
    u = v + 0.5
    rng = nmax - nmin + 1
    k = np.minimum(np.floor(u * float(rng)), rng - 1).astype(np.int64)
    return (nmin + k).astype(np.int32)


def batch_offsets(sizes, nrhs):
    sizes = np.asarray(sizes, dtype=np.int64)
    aoff = np.concatenate([[0], np.cumsum(sizes * sizes)]).astype(np.int64)
    voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return aoff, voff


def batch_system(sizes, packed, aoff, i):
    """View of system i of a packed A-layout array as an n x n Fortran matrix."""
    n = int(sizes[i])
    return packed[aoff[i]:aoff[i] + n * n].reshape((n, n), order="F")


def batch_rhs(sizes, packed, voff, nrhs, i):
    n = int(sizes[i])
    return packed[nrhs * voff[i]:nrhs * voff[i] + n * nrhs].reshape((n, nrhs), order="F")


def batched_solve(sizes, A, B, nrhs, W=None):
    """Per system: LU with partial pivoting, X = A^{-1} B and, with W, the adjoint
    grad_B = A^{-T} W, grad_A = -grad_B X^T.  Inputs and outputs packed; returns
    dict(LU, ipiv, X, GB, GA, info) (GB, GA None without W)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    aoff, voff = batch_offsets(sizes, nrhs)
    LU = np.array(A, dtype=np.float64, copy=True)
    X = np.array(B, dtype=np.float64, copy=True)
    ipiv = np.zeros(int(voff[-1]), dtype=np.int32)
    GB = np.zeros_like(X) if W is not None else None
    GA = np.zeros_like(LU) if W is not None else None
    info = np.zeros(sizes.size, dtype=np.int64)
    for i in range(sizes.size):
        n = int(sizes[i])
        Ai = np.asfortranarray(batch_system(sizes, np.asarray(A, dtype=np.float64), aoff, i))
        F = Ai.copy(order="F")
        piv, inf = lu(F)
        info[i] = inf
        LU[aoff[i]:aoff[i] + n * n] = F.reshape(-1, order="F")
        ipiv[voff[i]:voff[i] + n] = piv
        Bi = np.asfortranarray(batch_rhs(sizes, np.asarray(B, dtype=np.float64), voff, nrhs, i))
        Xi = Bi.copy(order="F")
        solve(F, piv, Xi)
        X[nrhs * voff[i]:nrhs * voff[i] + n * nrhs] = Xi.reshape(-1, order="F")
        if W is not None:
            Wi = np.asfortranarray(batch_rhs(sizes, np.asarray(W, dtype=np.float64), voff, nrhs, i))
            _, gb, ga, _ = solve_grad(Ai, Bi, Wi)
            GB[nrhs * voff[i]:nrhs * voff[i] + n * nrhs] = gb.reshape(-1, order="F")
            GA[aoff[i]:aoff[i] + n * n] = ga.reshape(-1, order="F")
    return {"LU": LU, "ipiv": ipiv, "X": X, "GB": GB, "GA": GA, "info": info}
