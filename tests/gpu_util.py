"""Helpers for the GPU tests: host <-> device copies of column-major matrices."""
import numpy as np


def torch():
    import torch as _t
    return _t


def hpl():
    import paper_2304_10397_amd.hpl as _h
    return _h


def to_gpu(a, ld=None, pad_value=np.nan):
    """Copy a float64 numpy matrix to a column-major CUDA tensor (leading dimension ld).

    Rows between a.shape[0] and ld are filled with pad_value so that writes outside
    the matrix are detectable."""
    t = torch()
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return t.from_numpy(a.copy()).to("cuda")
    n, m = a.shape
    ld = n if ld is None else ld
    M = hpl().colmajor(n, m, ld=ld, fill=float(pad_value))
    M.copy_(t.from_numpy(np.ascontiguousarray(a)))
    return M


def padding_of(M, ld):
    """The rows between M.shape[0] and the leading dimension ld (None when there are none)."""
    n, m = M.shape
    if ld == n or m == 0:
        return None
    base = M.as_strided((ld, m), (1, ld))
    return base[n:, :].cpu().numpy()


def to_host(M):
    return np.asfortranarray(M.cpu().numpy())
