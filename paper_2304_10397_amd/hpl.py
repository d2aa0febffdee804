"""Python binding of libhplx (include/hpl.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Device memory and
streams come from PyTorch (HIP build): matrices are float64 CUDA tensors in
column-major layout, i.e. ``A.stride(0) == 1`` and ``A.stride(1) == lda``
(``colmajor(n, m)`` makes one).  All arithmetic runs in the HIP kernels of
libhplx.so; there is no fallback: if the library is missing the import of this
module raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhplx.so")

HPL_OK = 0
HPL_ERR_HIP = 1
HPL_ERR_NOMEM = 2
HPL_ERR_DEVICE = 3
HPL_ERR_INTERNAL = 4

HPL_OPT_LOOKAHEAD = 1
HPL_OPT_PANEL_BASE = 2
HPL_OPT_PANEL_WGS = 3
HPL_OPT_TIMING = 4
HPL_OPT_PROGRESS = 5
HPL_OPT_SERIALIZE = 6
HPL_OPT_GEMM_TILE = 7
HPL_OPT_HOST_PANEL = 8
HPL_OPT_LASWP_WGS = 9
HPL_OPT_BATCH_CONFIG = 10
HPL_BATCH_VARIANTS = 4
HPL_BATCH_BUCKETS = 16

STAT_CLASSES = ("gemm", "panel", "laswp", "trsm", "solve", "plan", "mxp_gemm", "mxp_fact", "grad_a", "batched")


class HplError(RuntimeError):
    def __init__(self, fn, code, detail=""):
        self.code = code
        msg = f"{fn}: {strerror(code)} (code {code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


def _load():
    # PyTorch (ROCm build) ships its own HIP runtime.  Load it first so that
    # libhplx's dependency on libamdhip64.so.7 resolves to that same, already
    # loaded runtime: two runtimes in one process would not share devices,
    # streams or allocations.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libhplx.so not found at {LIB_PATH}; build it with "
            "`python -m paper_2304_10397_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    i64, u64, i32, dbl, P = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sig = {
        "hpl_factor": (i32, [P, i64, i64, i64, P, P, P]),
        "hpl_solve": (i32, [P, P, P, i64, i64, i64, i64, i32, P]),
        "hpl_solve_noalloc": (i32, [P, P, P, i64, i64, i64, i64, i32, P]),
        "hpl_solve_augmented": (i32, [P, i64, i64, i64, i64, P, P, P]),
        "hpl_residual": (i32, [P, i64, i64, P, i64, P, i64, i64, P, P]),
        "hpl_residual_gen": (i32, [u64, i64, P, i64, P, i64, i64, P, P]),
        "hpl_generate": (i32, [u64, u64, P, i64, i64, i64, P]),
        "hpl_set_option": (i32, [i32, i64]),
        "hpl_get_option": (i64, [i32]),
        "hpl_get_stats": (i32, [P, P, P, P, i32]),
        "hpl_reset_stats": (None, []),
        "hpl_mfma_peak": (i32, [i64, P, P]),
        "hpl_solve_grad_a": (i32, [P, i64, P, i64, i64, i64, P, i64, P]),
        "hpl_generate_normal": (i32, [u64, u64, P, i64, i64, i64, P]),
        "hpl_add_diagonal": (i32, [P, i64, i64, dbl, P]),
        "hpl_mxp_generate": (i32, [u64, P, i64, i64, P]),
        "hpl_mxp_factor": (i32, [P, i64, i64, i64, i32, P, i64, P, P]),
        "hpl_mxp_solve": (i32, [P, i64, P, i64, i64, P, P, i64, P, P]),
        "hpl_batched_sizes": (i32, [u64, i64, ctypes.c_int32, ctypes.c_int32, P]),
        "hpl_host_panel": (i32, [P, i64, i64, i64, P, i32, P]),
        "hpl_panel_factor": (i32, [P, i64, i64, i64, P, P, P]),
        "hpl_batched_solve": (i32, [i64, P, i64, P, P, P, P, P, P, i32, P, P]),
        "hpl_batched_config": (i32, [i64, P, P, P, P]),
        "hpl_batched_table": (i32, [P, P]),
        "hpl_release": (i32, []),
        "hpl_strerror": (ctypes.c_char_p, [i32]),
        "hpl_last_error_detail": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()
EXPORTED = ("hpl_factor", "hpl_solve", "hpl_solve_noalloc", "hpl_residual", "hpl_residual_gen", "hpl_generate",
            "hpl_set_option", "hpl_get_option", "hpl_get_stats", "hpl_reset_stats",
            "hpl_mfma_peak", "hpl_solve_grad_a", "hpl_generate_normal", "hpl_add_diagonal",
            "hpl_mxp_generate", "hpl_mxp_factor", "hpl_mxp_solve", "hpl_batched_sizes", "hpl_batched_solve",
            "hpl_batched_config", "hpl_batched_table",
            "hpl_host_panel", "hpl_panel_factor",
            "hpl_release", "hpl_strerror", "hpl_last_error_detail")


def lib():
    return _lib


def strerror(code: int) -> str:
    return _lib.hpl_strerror(int(code)).decode()


def _check(fn, rc):
    if rc != 0:
        detail = _lib.hpl_last_error_detail().decode() if rc > 0 else ""
        if rc < 0:
            raise ValueError(f"{fn}: {strerror(rc)}")
        raise HplError(fn, rc, detail)


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _matrix(name, M, rows=None):
    """(pointer, rows, cols, ld) of a column-major float64 CUDA tensor (1-D = one column)."""
    torch = _torch()
    if not isinstance(M, torch.Tensor) or M.dtype != torch.float64 or not M.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if M.dim() == 1:
        if M.stride(0) != 1 and M.numel() > 1:
            raise ValueError(f"{name} must be contiguous")
        r = M.shape[0]
        return ctypes.c_void_p(M.data_ptr()), r, 1, max(1, r)
    if M.dim() != 2:
        raise ValueError(f"{name} must be 1-D or 2-D")
    r, c = M.shape
    if r > 1 and M.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    ld = M.stride(1) if c > 1 else max(1, r)
    return ctypes.c_void_p(M.data_ptr()), r, c, max(ld, 1)


def colmajor(rows, cols, ld=None, device="cuda", fill=None):
    """Empty (or filled) column-major float64 tensor of shape (rows, cols), leading dimension ld."""
    torch = _torch()
    ld = rows if ld is None else ld
    buf = torch.empty((max(cols, 1), max(ld, 1)), dtype=torch.float64, device=device)
    if fill is not None:
        buf.fill_(fill)
    return buf.t()[:rows, :cols]


def hpl_factor(A, nb, ipiv=None, stream=None):
    """LU with partial pivoting in place; returns (ipiv int32 CUDA tensor, info)."""
    torch = _torch()
    pA, n, m, lda = _matrix("A", A)
    if n != m:
        raise ValueError("A must be square")
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    if ipiv.dtype != torch.int32 or not ipiv.is_cuda or ipiv.numel() < n:
        raise TypeError("ipiv must be an int32 CUDA tensor with n entries")
    info = ctypes.c_int64(0)
    rc = _lib.hpl_factor(pA, n, lda, int(nb), ctypes.c_void_p(ipiv.data_ptr()), ctypes.byref(info),
                         _stream(stream))
    _check("hpl_factor", rc)
    return ipiv[:n], int(info.value)


def hpl_solve(LU, ipiv, B, trans=0, stream=None):
    """Overwrite B (n or n x nrhs, column-major) with the solution of A X = B (or A^T X = B)."""
    pLU, n, m, lda = _matrix("LU", LU)
    pB, nb_, nrhs, ldb = _matrix("B", B)
    if nb_ != n:
        raise ValueError("B must have n rows")
    rc = _lib.hpl_solve(pLU, ctypes.c_void_p(ipiv.data_ptr()), pB, nrhs, n, lda, ldb, int(trans),
                        _stream(stream))
    _check("hpl_solve", rc)
    return B


def hpl_solve_augmented(AB, n, nb, ipiv=None, stream=None):
    """Solve of the augmented system AB = [A | B] (n x (n + nrhs), column-major
    CUDA tensor) in place: returns (ipiv, info); AB[:, n:] then holds X."""
    torch = _torch()
    pA, rows, cols, lda = _matrix("AB", AB)
    if rows != n or cols < n:
        raise ValueError(f"AB must be {n} x (n + nrhs), got {rows} x {cols}")
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=AB.device)
    if ipiv.dtype != torch.int32 or not ipiv.is_cuda or ipiv.numel() < n:
        raise TypeError("ipiv must be an int32 CUDA tensor with n entries")
    info = ctypes.c_int64(0)
    _check("hpl_solve_augmented", _lib.hpl_solve_augmented(pA, n, lda, int(nb), cols - n,
                                                            ctypes.c_void_p(ipiv.data_ptr()), ctypes.byref(info),
                                                            _stream(stream)))
    return ipiv[:n], int(info.value)


def hpl_solve_noalloc(LU, ipiv, B, trans=0, stream=None):
    """hpl_solve with the library's fixed scratch array instead of allocated
    workspace (n <= HPL_SOLVE_NOALLOC_MAX_N); same results."""
    pLU, n, m, lda = _matrix("LU", LU)
    pB, nb_, nrhs, ldb = _matrix("B", B)
    if nb_ != n:
        raise ValueError("B must have n rows")
    rc = _lib.hpl_solve_noalloc(pLU, ctypes.c_void_p(ipiv.data_ptr()), pB, nrhs, n, lda, ldb, int(trans),
                                _stream(stream))
    _check("hpl_solve_noalloc", rc)
    return B


HPL_SOLVE_NOALLOC_MAX_N = 262144


def hpl_residual(A0, X, B, stream=None):
    """numpy [scaled, ||r||inf, ||A||inf, ||x||inf, ||b||inf] (HPL passes when scaled < 16)."""
    pA, n, m, lda = _matrix("A0", A0)
    pX, _, nrhs, ldx = _matrix("X", X)
    pB, _, _, ldb = _matrix("B", B)
    out = np.zeros(5)
    rc = _lib.hpl_residual(pA, n, lda, pX, ldx, pB, ldb, nrhs, out.ctypes.data_as(ctypes.c_void_p),
                           _stream(stream))
    _check("hpl_residual", rc)
    return out


def hpl_residual_gen(seed, n, X, B, stream=None):
    """As hpl_residual with A regenerated from (seed, stream 0)."""
    pX, _, nrhs, ldx = _matrix("X", X)
    pB, _, _, ldb = _matrix("B", B)
    out = np.zeros(5)
    rc = _lib.hpl_residual_gen(int(seed) % 2**64, int(n), pX, ldx, pB, ldb, nrhs,
                               out.ctypes.data_as(ctypes.c_void_p), _stream(stream))
    _check("hpl_residual_gen", rc)
    return out


def hpl_generate(seed, stream_id, M, stream=None):
    """Fill the column-major tensor M with the random stream (seed, stream_id); returns M."""
    pM, r, c, ld = _matrix("M", M)
    rc = _lib.hpl_generate(int(seed) % 2**64, int(stream_id) % 2**64, pM, r, c, ld, _stream(stream))
    _check("hpl_generate", rc)
    return M


def hpl_generate_normal(seed, stream_id, M, stream=None):
    """Fill the column-major tensor M with Box-Muller normal values of (seed, stream_id); returns M."""
    pM, r, c, ld = _matrix("M", M)
    rc = _lib.hpl_generate_normal(int(seed) % 2**64, int(stream_id) % 2**64, pM, r, c, ld, _stream(stream))
    _check("hpl_generate_normal", rc)
    return M


def hpl_add_diagonal(M, alpha, stream=None):
    """M(i,i) += alpha in place (square column-major M); returns M."""
    pM, r, c, ld = _matrix("M", M)
    if r != c:
        raise ValueError("M must be square")
    _check("hpl_add_diagonal", _lib.hpl_add_diagonal(pM, r, ld, float(alpha), _stream(stream)))
    return M


def hpl_solve_grad_a(GB, X, dA=None, stream=None):
    """dA = -GB X^T (n x n, column-major), written once; returns dA."""
    pG, n, k, ldg = _matrix("GB", GB)
    pX, n2, k2, ldx = _matrix("X", X)
    if n2 != n or k2 != k:
        raise ValueError("GB and X must have the same shape")
    if dA is None:
        dA = colmajor(n, n, device=GB.device)
    pD, n3, m3, ldd = _matrix("dA", dA)
    if n3 != n or m3 != n:
        raise ValueError("dA must be n x n")
    _check("hpl_solve_grad_a", _lib.hpl_solve_grad_a(pG, ldg, pX, ldx, n, k, pD, ldd, _stream(stream)))
    return dA


MXP_FP16, MXP_BF16 = 0, 1


def colmajor32(rows, cols, ld=None, device="cuda"):
    """Empty column-major float32 tensor of shape (rows, cols), leading dimension ld."""
    torch = _torch()
    ld = rows if ld is None else ld
    return torch.empty((max(cols, 1), max(ld, 1)), dtype=torch.float32, device=device).t()[:rows, :cols]


def hpl_mxp_generate(seed, A, stream=None):
    """Fill the square column-major float64 tensor A with the diagonally dominant MxP input."""
    pA, n, m, lda = _matrix("A", A)
    if n != m:
        raise ValueError("A must be square")
    _check("hpl_mxp_generate", _lib.hpl_mxp_generate(int(seed) % 2**64, pA, n, lda, _stream(stream)))
    return A


def hpl_mxp_factor(A, nb=512, fmt=MXP_FP16, LU=None, stream=None):
    """No-pivot LU of A (float64) in mixed precision; returns (LU float32 column-major, info)."""
    torch = _torch()
    pA, n, m, lda = _matrix("A", A)
    if n != m:
        raise ValueError("A must be square")
    if LU is None:
        LU = colmajor32(n, n, device=A.device)
    if LU.dtype != torch.float32 or not LU.is_cuda or LU.shape != (n, n) or (n > 1 and LU.stride(0) != 1):
        raise TypeError("LU must be a column-major float32 CUDA tensor of A's shape")
    ldlu = LU.stride(1) if n > 1 else max(1, n)
    info = ctypes.c_int64(0)
    _check("hpl_mxp_factor", _lib.hpl_mxp_factor(pA, n, lda, int(nb), int(fmt), ctypes.c_void_p(LU.data_ptr()),
                                                  ldlu, ctypes.byref(info), _stream(stream)))
    return LU, int(info.value)


def hpl_mxp_solve(A, LU, b, x=None, max_iter=50, stream=None):
    """x refined in FP64 from the FP32 factors; returns (x, out[5] numpy)."""
    pA, n, m, lda = _matrix("A", A)
    ldlu = LU.stride(1) if n > 1 else max(1, n)
    if x is None:
        x = _torch().empty(n, dtype=_torch().float64, device=A.device)
    pb, nb_, _, _ = _matrix("b", b)
    px, nx, _, _ = _matrix("x", x)
    if nb_ != n or nx != n:
        raise ValueError("b and x must have n entries")
    out = np.zeros(5)
    _check("hpl_mxp_solve", _lib.hpl_mxp_solve(pA, lda, ctypes.c_void_p(LU.data_ptr()), ldlu, n, pb, px,
                                                int(max_iter), out.ctypes.data_as(ctypes.c_void_p),
                                                _stream(stream)))
    return x, out


def hpl_host_panel(P, threads, ipiv=None):
    """The paper's CPU FACT of the m x nb panel P (numpy float64, Fortran order, in place)
    with T threads; returns (ipiv int32[nb] 0-based, info)."""
    if not (isinstance(P, np.ndarray) and P.dtype == np.float64 and P.ndim == 2):
        raise TypeError("P must be a 2-D float64 numpy array")
    if P.shape[0] > 1 and P.strides[0] != 8:
        raise TypeError("P must be column-major (Fortran order)")
    m, nb = P.shape
    ldp = max(1, P.strides[1] // 8 if nb > 1 else m, m)
    ipiv = np.zeros(max(nb, 1), dtype=np.int32) if ipiv is None else ipiv
    info = ctypes.c_int64(0)
    _check("hpl_host_panel", _lib.hpl_host_panel(P.ctypes.data_as(ctypes.c_void_p), m, nb, ldp,
                                                  ipiv.ctypes.data_as(ctypes.c_void_p), int(threads),
                                                  ctypes.byref(info)))
    return ipiv[:nb], int(info.value)


def hpl_panel_factor(A, ipiv=None, stream=None):
    """GPU FACT of the m x nb column-major CUDA panel A (in place); returns (ipiv, info)."""
    torch = _torch()
    pA, m, nb, lda = _matrix("A", A)
    if ipiv is None:
        ipiv = torch.empty(max(nb, 1), dtype=torch.int32, device=A.device)
    info = ctypes.c_int64(0)
    _check("hpl_panel_factor", _lib.hpl_panel_factor(pA, m, nb, lda, ctypes.c_void_p(ipiv.data_ptr()),
                                                      ctypes.byref(info), _stream(stream)))
    return ipiv[:nb], int(info.value)


BATCH_FORWARD, BATCH_ADJOINT, BATCH_BOTH = 1, 2, 3


def hpl_batched_sizes(seed, count, nmin=32, nmax=512):
    """Seeded system sizes of a batch (host computation); numpy int32 array."""
    sizes = np.zeros(max(int(count), 1), dtype=np.int32)
    _check("hpl_batched_sizes", _lib.hpl_batched_sizes(int(seed), int(count), int(nmin), int(nmax),
                                                        sizes.ctypes.data_as(ctypes.c_void_p)))
    return sizes[:int(count)]


def batch_layout(sizes, nrhs):
    """Packed offsets: (aoff, voff, total A elements, total B elements), numpy int64."""
    sizes = np.asarray(sizes, dtype=np.int64)
    aoff = np.concatenate([[0], np.cumsum(sizes * sizes)[:-1]]) if sizes.size else np.zeros(0, np.int64)
    voff = np.concatenate([[0], np.cumsum(sizes)[:-1]]) if sizes.size else np.zeros(0, np.int64)
    return aoff, voff, int(np.sum(sizes * sizes)), int(np.sum(sizes)) * int(nrhs)


def hpl_batched_config(sizes):
    """The schedule hpl_batched_solve picks for these sizes by default:
    (occ, variant per size bucket (numpy int8[16]), predicted ms)."""
    sizes = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    occ = ctypes.c_int(0)
    vtab = np.zeros(HPL_BATCH_BUCKETS, dtype=np.int8)
    pred = ctypes.c_double(0.0)
    _check("hpl_batched_config", _lib.hpl_batched_config(int(sizes.size), sizes.ctypes.data_as(ctypes.c_void_p),
                                                         ctypes.byref(occ), vtab.ctypes.data_as(ctypes.c_void_p),
                                                         ctypes.byref(pred)))
    return int(occ.value), vtab, float(pred.value)


def hpl_batched_table():
    """(cost[occ-1, variant, bucket] in microseconds per system, tuned flag) of the library's table."""
    cost = np.zeros((2, HPL_BATCH_VARIANTS, HPL_BATCH_BUCKETS))
    tuned = ctypes.c_int(0)
    _check("hpl_batched_table", _lib.hpl_batched_table(cost.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tuned)))
    return cost, bool(tuned.value)


def hpl_batched_solve(sizes, A, ipiv, B, nrhs, W=None, GB=None, GA=None, mode=BATCH_FORWARD, stream=None):
    """One launch over the packed batch (see hpl.h); returns the info array (numpy int64)."""
    torch = _torch()
    sizes = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    count = sizes.size
    _, _, na, nb_ = batch_layout(sizes, nrhs)

    def dev(name, T, n, dtype, need):
        if T is None:
            if need:
                raise ValueError(f"{name} is required for mode {mode}")
            return None
        if not T.is_cuda or T.dtype != dtype or not T.is_contiguous() or T.numel() < n:
            raise TypeError(f"{name} must be a contiguous CUDA {dtype} tensor of at least {n} elements")
        return ctypes.c_void_p(T.data_ptr())

    adj = bool(mode & 2)
    pA = dev("A", A, na, torch.float64, True)
    pI = dev("ipiv", ipiv, int(np.sum(sizes)), torch.int32, True)
    pB = dev("B", B, nb_, torch.float64, True)
    pW = dev("W", W, nb_, torch.float64, adj)
    pGB = dev("GB", GB, nb_, torch.float64, adj)
    pGA = dev("GA", GA, na, torch.float64, adj)
    info = np.zeros(max(count, 1), dtype=np.int64)
    _check("hpl_batched_solve", _lib.hpl_batched_solve(count, sizes.ctypes.data_as(ctypes.c_void_p), int(nrhs), pA,
                                                        pI, pB, pW, pGB, pGA, int(mode),
                                                        info.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return info[:count]


def _colmajor_copy(T):
    """Column-major float64 copy of a 1-D or 2-D CUDA tensor (a device copy)."""
    if T.dim() == 1:
        return T.detach().to(dtype=_torch().float64).clone()
    out = colmajor(T.shape[0], T.shape[1], device=T.device)
    out.copy_(T.detach())
    return out


def _autograd():
    torch = _torch()

    class HplSolve(torch.autograd.Function):
        """X = A^{-1} B through hpl_factor + hpl_solve; backward reuses the factors:
        grad_B = A^{-T} G (hpl_solve, trans = 1) and grad_A = -grad_B X^T
        (hpl_solve_grad_a)."""

        @staticmethod
        def forward(ctx, A, B, nb):
            LU = _colmajor_copy(A)
            ipiv, info = hpl_factor(LU, nb)
            if info != 0:
                raise ZeroDivisionError(f"hpl_factor: U({info - 1},{info - 1}) is exactly zero")
            X = _colmajor_copy(B)
            hpl_solve(LU, ipiv, X)
            ctx.save_for_backward(LU, ipiv, X)
            ctx.vec = B.dim() == 1
            return X

        @staticmethod
        def backward(ctx, G):
            LU, ipiv, X = ctx.saved_tensors
            GB = _colmajor_copy(G)
            hpl_solve(LU, ipiv, GB, trans=1)
            n = LU.shape[0]
            GB2 = GB.reshape(n, 1) if ctx.vec else GB
            X2 = X.reshape(n, 1) if ctx.vec else X
            GA = hpl_solve_grad_a(GB2, X2) if ctx.needs_input_grad[0] else None
            return GA, (GB if ctx.needs_input_grad[1] else None), None

    return HplSolve


_HPL_SOLVE = None


def hpl_solve_diff(A, B, nb=256):
    """Differentiable X = A^{-1} B (float64 CUDA tensors; B n or n x nrhs)."""
    global _HPL_SOLVE
    if _HPL_SOLVE is None:
        _HPL_SOLVE = _autograd()
    return _HPL_SOLVE.apply(A, B, int(nb))


def hpl_set_option(key, value):
    rc = _lib.hpl_set_option(int(key), int(value))
    if rc != 0:
        raise ValueError(f"hpl_set_option({key}, {value}) -> {rc}")


def hpl_get_option(key):
    return int(_lib.hpl_get_option(int(key)))


def hpl_get_stats():
    """{class: {"launches", "ms", "flops", "bytes"}} accumulated while HPL_OPT_TIMING is 1."""
    cap = 16
    la = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    fl = (ctypes.c_double * cap)()
    by = (ctypes.c_double * cap)()
    k = _lib.hpl_get_stats(la, ms, fl, by, cap)
    return {STAT_CLASSES[i] if i < len(STAT_CLASSES) else str(i):
            {"launches": int(la[i]), "ms": ms[i], "flops": fl[i], "bytes": by[i]} for i in range(k)}


def hpl_reset_stats():
    _lib.hpl_reset_stats()


def hpl_mfma_peak(iters=200000, stream=None):
    """(TFLOP/s, ms) of a pure FP64 16x16x4 MFMA loop on the current device."""
    out = np.zeros(2)
    _check("hpl_mfma_peak", _lib.hpl_mfma_peak(int(iters), out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return float(out[0]), float(out[1])


def hpl_release():
    _check("hpl_release", _lib.hpl_release())


def hpl_strerror(code):
    return strerror(code)


def hpl_last_error_detail():
    return _lib.hpl_last_error_detail().decode()
