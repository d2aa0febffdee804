"""MI355X (gfx950) HPL hot path: FP64 blocked LU with partial pivoting, look-ahead, solves.

The compute lives in libhplx.so (HIP kernels behind the C ABI of include/hpl.h);
this package holds the build script and the ctypes binding (paper_2304_10397_amd.hpl).
Importing the binding raises if the library has not been built.
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "libhplx.so")


def hpl():
    """The binding module (imported lazily so that `import paper_2304_10397_amd` never fails)."""
    from . import hpl as _hpl
    return _hpl
