"""C-ABI checks that need no GPU: the library loads, exports every function that
include/hpl.h declares, and rejects invalid arguments on the host (-k) before
any HIP call."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpl.h")

h = pytest.importorskip("paper_2304_10397_amd.hpl", reason="libhplx.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpl_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", h.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hpl_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(h.lib(), n)


P = ctypes.c_void_p
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def test_factor_argument_errors():
    L = h.lib()
    info = ctypes.c_int64(7)
    assert L.hpl_factor(None, 10, 10, 64, FAKE, ctypes.byref(info), None) == -1
    assert L.hpl_factor(FAKE, -1, 10, 64, FAKE, ctypes.byref(info), None) == -2
    assert L.hpl_factor(FAKE, 2**31, 2**31, 64, FAKE, ctypes.byref(info), None) == -2
    assert L.hpl_factor(FAKE, 10, 9, 64, FAKE, ctypes.byref(info), None) == -3
    assert L.hpl_factor(FAKE, 10, 10, 0, FAKE, ctypes.byref(info), None) == -4
    assert L.hpl_factor(FAKE, 10, 10, 1025, FAKE, ctypes.byref(info), None) == -4
    assert L.hpl_factor(FAKE, 10, 10, 64, None, ctypes.byref(info), None) == -5
    assert L.hpl_factor(FAKE, 10, 10, 64, FAKE, None, None) == -6
    assert info.value == 7  # untouched on argument errors
    assert L.hpl_factor(None, 0, 1, 64, None, ctypes.byref(info), None) == 0 and info.value == 0


def test_solve_augmented_argument_errors():
    L = h.lib()
    info = ctypes.c_int64(7)
    assert L.hpl_solve_augmented(None, 10, 10, 64, 1, FAKE, ctypes.byref(info), None) == -1
    assert L.hpl_solve_augmented(FAKE, -1, 10, 64, 1, FAKE, ctypes.byref(info), None) == -2
    assert L.hpl_solve_augmented(FAKE, 10, 9, 64, 1, FAKE, ctypes.byref(info), None) == -3
    assert L.hpl_solve_augmented(FAKE, 10, 10, 0, 1, FAKE, ctypes.byref(info), None) == -4
    assert L.hpl_solve_augmented(FAKE, 10, 10, 1025, 1, FAKE, ctypes.byref(info), None) == -4
    assert L.hpl_solve_augmented(FAKE, 10, 10, 64, -1, FAKE, ctypes.byref(info), None) == -5
    assert L.hpl_solve_augmented(FAKE, 10, 10, 64, 1, None, ctypes.byref(info), None) == -6
    assert L.hpl_solve_augmented(FAKE, 10, 10, 64, 1, FAKE, None, None) == -7
    assert info.value == 7  # untouched on argument errors
    assert L.hpl_solve_augmented(None, 0, 1, 64, 1, None, ctypes.byref(info), None) == 0 and info.value == 0


def test_solve_argument_errors():
    L = h.lib()
    assert L.hpl_solve(None, FAKE, FAKE, 1, 10, 10, 10, 0, None) == -1
    assert L.hpl_solve(FAKE, None, FAKE, 1, 10, 10, 10, 0, None) == -2
    assert L.hpl_solve(FAKE, FAKE, None, 1, 10, 10, 10, 0, None) == -3
    assert L.hpl_solve(FAKE, FAKE, FAKE, -1, 10, 10, 10, 0, None) == -4
    assert L.hpl_solve(FAKE, FAKE, FAKE, 1, -1, 10, 10, 0, None) == -5
    assert L.hpl_solve(FAKE, FAKE, FAKE, 1, 10, 9, 10, 0, None) == -6
    assert L.hpl_solve(FAKE, FAKE, FAKE, 1, 10, 10, 9, 0, None) == -7
    assert L.hpl_solve(FAKE, FAKE, FAKE, 1, 10, 10, 10, 2, None) == -8
    assert L.hpl_solve(FAKE, FAKE, FAKE, 0, 10, 10, 10, 0, None) == 0  # nothing to do


def test_residual_generate_argument_errors():
    L = h.lib()
    out = (ctypes.c_double * 5)()
    assert L.hpl_residual(None, 4, 4, FAKE, 4, FAKE, 4, 1, out, None) == -1
    assert L.hpl_residual(FAKE, 4, 3, FAKE, 4, FAKE, 4, 1, out, None) == -3
    assert L.hpl_residual(FAKE, 4, 4, FAKE, 4, FAKE, 4, 0, out, None) == -8
    assert L.hpl_residual(FAKE, 4, 4, FAKE, 4, FAKE, 4, 1, None, None) == -9
    assert L.hpl_residual_gen(1, -1, FAKE, 4, FAKE, 4, 1, out, None) == -2
    assert L.hpl_residual_gen(1, 4, None, 4, FAKE, 4, 1, out, None) == -3
    assert L.hpl_residual_gen(1, 4, FAKE, 4, FAKE, 4, 1, None, None) == -8
    assert L.hpl_generate(1, 0, None, 4, 4, 4, None) == -3
    assert L.hpl_generate(1, 0, FAKE, -1, 4, 4, None) == -4
    assert L.hpl_generate(1, 0, FAKE, 4, -1, 4, None) == -5
    assert L.hpl_generate(1, 0, FAKE, 4, 4, 3, None) == -6
    assert L.hpl_generate(1, 0, FAKE, 0, 4, 1, None) == 0


def test_mfma_peak_argument_errors():
    L = h.lib()
    out = (ctypes.c_double * 2)()
    assert L.hpl_mfma_peak(0, out, None) == -1
    assert L.hpl_mfma_peak(-5, out, None) == -1
    assert L.hpl_mfma_peak(10, None, None) == -2


def test_mxp_argument_errors():
    L = h.lib()
    info = ctypes.c_int64(0)
    out = (ctypes.c_double * 5)()
    assert L.hpl_mxp_factor(None, 4, 4, 64, 0, FAKE, 4, ctypes.byref(info), None) == -1
    assert L.hpl_mxp_factor(FAKE, -1, 4, 64, 0, FAKE, 4, ctypes.byref(info), None) == -2
    assert L.hpl_mxp_factor(FAKE, 4, 3, 64, 0, FAKE, 4, ctypes.byref(info), None) == -3
    assert L.hpl_mxp_factor(FAKE, 4, 4, 96, 0, FAKE, 4, ctypes.byref(info), None) == -4
    assert L.hpl_mxp_factor(FAKE, 4, 4, 4160, 0, FAKE, 4, ctypes.byref(info), None) == -4
    assert L.hpl_mxp_factor(FAKE, 4, 4, 0, 0, FAKE, 4, ctypes.byref(info), None) == -4
    assert L.hpl_mxp_factor(FAKE, 4, 4, 64, 2, FAKE, 4, ctypes.byref(info), None) == -5
    assert L.hpl_mxp_factor(FAKE, 4, 4, 64, 1, None, 4, ctypes.byref(info), None) == -6
    assert L.hpl_mxp_factor(FAKE, 4, 4, 64, 1, FAKE, 2, ctypes.byref(info), None) == -7
    assert L.hpl_mxp_factor(FAKE, 4, 4, 64, 1, FAKE, 4, None, None) == -8
    assert L.hpl_mxp_solve(FAKE, 4, FAKE, 4, 4, FAKE, FAKE, -1, out, None) == -8
    assert L.hpl_mxp_solve(FAKE, 4, FAKE, 4, 4, FAKE, FAKE, 5, None, None) == -9
    assert L.hpl_mxp_solve(FAKE, 3, FAKE, 4, 4, FAKE, FAKE, 5, out, None) == -2
    assert L.hpl_mxp_generate(1, None, 4, 4, None) == -2
    assert L.hpl_mxp_generate(1, FAKE, 4, 2, None) == -4


def test_options_roundtrip_and_rejects():
    old = h.hpl_get_option(h.HPL_OPT_LOOKAHEAD)
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 0)
    assert h.hpl_get_option(h.HPL_OPT_LOOKAHEAD) == 0
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 2)
    assert h.hpl_get_option(h.HPL_OPT_LOOKAHEAD) == 2
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 3)
    assert h.hpl_get_option(h.HPL_OPT_LOOKAHEAD) == 3
    with pytest.raises(ValueError):
        h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, 4)
    assert h.hpl_get_option(h.HPL_OPT_LOOKAHEAD) == 3
    h.hpl_set_option(h.HPL_OPT_LOOKAHEAD, old)
    with pytest.raises(ValueError):
        h.hpl_set_option(h.HPL_OPT_PANEL_BASE, 12)
    with pytest.raises(ValueError):
        h.hpl_set_option(999, 1)
    assert h.hpl_get_option(999) == -(2**63)
    assert h.hpl_get_option(h.HPL_OPT_LASWP_WGS) == 96
    h.hpl_set_option(h.HPL_OPT_LASWP_WGS, 0)
    assert h.hpl_get_option(h.HPL_OPT_LASWP_WGS) == 0
    with pytest.raises(ValueError):
        h.hpl_set_option(h.HPL_OPT_LASWP_WGS, -1)
    assert h.hpl_get_option(h.HPL_OPT_LASWP_WGS) == 0
    h.hpl_set_option(h.HPL_OPT_LASWP_WGS, 96)


def test_strerror():
    assert h.hpl_strerror(0) == "success"
    assert h.hpl_strerror(-4) == "invalid argument 4"
    assert "HIP" in h.hpl_strerror(1)
    assert h.hpl_strerror(12345) == "unknown error code"


def test_stats_interface():
    h.hpl_reset_stats()
    st = h.hpl_get_stats()
    assert set(st) >= {"gemm", "panel", "laswp", "trsm", "solve"}
    assert all(v["launches"] == 0 for v in st.values())


def test_batched_argument_errors_and_sizes():
    import numpy as np
    import oracle
    L = h.lib()
    info = (ctypes.c_int64 * 4)()
    sz = (ctypes.c_int32 * 2)(4, 513)
    ok = (ctypes.c_int32 * 2)(4, 5)
    assert L.hpl_batched_solve(-1, ok, 1, FAKE, FAKE, FAKE, None, None, None, 1, info, None) == -1
    assert L.hpl_batched_solve(2, None, 1, FAKE, FAKE, FAKE, None, None, None, 1, info, None) == -2
    assert L.hpl_batched_solve(2, sz, 1, FAKE, FAKE, FAKE, None, None, None, 1, info, None) == -2
    assert L.hpl_batched_solve(2, ok, 0, FAKE, FAKE, FAKE, None, None, None, 1, info, None) == -3
    assert L.hpl_batched_solve(2, ok, 17, FAKE, FAKE, FAKE, None, None, None, 1, info, None) == -3
    assert L.hpl_batched_solve(2, ok, 1, None, FAKE, FAKE, None, None, None, 1, info, None) == -4
    assert L.hpl_batched_solve(2, ok, 1, FAKE, None, FAKE, None, None, None, 1, info, None) == -5
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, None, None, None, None, 1, info, None) == -6
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, FAKE, None, FAKE, FAKE, 3, info, None) == -7
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, FAKE, FAKE, None, FAKE, 2, info, None) == -8
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None, 2, info, None) == -9
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, FAKE, None, None, None, 0, info, None) == -10
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, FAKE, None, None, None, 4, info, None) == -10
    assert L.hpl_batched_solve(2, ok, 1, FAKE, FAKE, FAKE, None, None, None, 1, None, None) == -11
    assert L.hpl_batched_solve(0, None, 1, None, None, None, None, None, None, 1, None, None) == 0
    assert L.hpl_batched_sizes(1, -1, 1, 2, info) == -2
    assert L.hpl_batched_sizes(1, 2, 0, 2, info) == -3
    assert L.hpl_batched_sizes(1, 2, 5, 4, info) == -4
    assert L.hpl_batched_sizes(1, 2, 1, 4, None) == -5
    # the library's host-side sizes equal the oracle's, bit for bit
    for seed, cnt, lo, hi in ((2304, 4096, 32, 512), (7, 1000, 1, 100), (1, 10, 5, 5)):
        got = h.hpl_batched_sizes(seed, cnt, lo, hi)
        assert np.array_equal(got, oracle.batched_sizes(seed, cnt, lo, hi))


def test_solve_noalloc_argument_errors():
    """The no-allocation solve rejects sizes beyond its fixed scratch array (and
    the other invalid arguments, as hpl_solve) on the host, before any HIP call."""
    L = h.lib()
    big = h.HPL_SOLVE_NOALLOC_MAX_N + 1
    assert L.hpl_solve_noalloc(FAKE, FAKE, FAKE, 1, big, big, big, 0, None) == -5
    assert b"HPL_SOLVE_NOALLOC_MAX_N" in L.hpl_last_error_detail()
    assert L.hpl_solve_noalloc(None, FAKE, FAKE, 1, 10, 10, 10, 0, None) == -1
    assert L.hpl_solve_noalloc(FAKE, None, FAKE, 1, 10, 10, 10, 0, None) == -2
    assert L.hpl_solve_noalloc(FAKE, FAKE, None, 1, 10, 10, 10, 0, None) == -3
    assert L.hpl_solve_noalloc(FAKE, FAKE, FAKE, -1, 10, 10, 10, 0, None) == -4
    assert L.hpl_solve_noalloc(FAKE, FAKE, FAKE, 1, -1, 10, 10, 0, None) == -5
    assert L.hpl_solve_noalloc(FAKE, FAKE, FAKE, 1, 10, 9, 10, 0, None) == -6
    assert L.hpl_solve_noalloc(FAKE, FAKE, FAKE, 1, 10, 10, 9, 0, None) == -7
    assert L.hpl_solve_noalloc(FAKE, FAKE, FAKE, 1, 10, 10, 10, 2, None) == -8
    assert L.hpl_solve_noalloc(None, None, None, 1, 0, 1, 1, 0, None) == 0
    hdr = open(HEADER).read()
    assert f"#define HPL_SOLVE_NOALLOC_MAX_N {h.HPL_SOLVE_NOALLOC_MAX_N}" in hdr


def test_batched_schedule_choice():
    """hpl_batched_config (host only) against a plain re-derivation from the
    library's own table: per systems-per-CU, each size bucket's cheapest variant;
    the smaller predicted total wins."""
    import numpy as np
    cost, tuned = h.hpl_batched_table()
    assert cost.shape == (2, h.HPL_BATCH_VARIANTS, h.HPL_BATCH_BUCKETS) and np.all(cost > 0)
    for seed, lo, hi in ((2304, 32, 512), (1, 1, 64), (7, 400, 512)):
        sizes = h.hpl_batched_sizes(seed, 1000, lo, hi)
        occ, vtab, pred = h.hpl_batched_config(sizes)
        hist = np.bincount((sizes - 1) // 32, minlength=h.HPL_BATCH_BUCKETS)
        best = [(float(np.sum(hist * cost[o].min(axis=0))), o + 1, cost[o].argmin(axis=0)) for o in (0, 1)]
        tot, o_ref, v_ref = min(best, key=lambda b: b[0])
        assert occ == o_ref
        assert np.array_equal(vtab, v_ref.astype(np.int8))
        assert abs(pred - tot * 1e-3) <= 1e-9 * max(1.0, tot)
    assert h.lib().hpl_set_option(h.HPL_OPT_BATCH_CONFIG, 2 * h.HPL_BATCH_VARIANTS + 1) == -2
    assert h.lib().hpl_get_option(h.HPL_OPT_BATCH_CONFIG) == 0
