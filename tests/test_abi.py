"""The C-ABI library loads and exports every function that include/fzw.h
declares; argument validation that happens before any GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_03969_amd", "libfzw.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "fzw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fzw_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfzw.so not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fzw_plan_create", "fzw_forward", "fzw_value_and_grad", "fzw_leapfrog", "fzw_set_counts"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_plan_create_rejects_bad_arguments_without_gpu(lib):
    from paper_2506_03969_amd.fzw import CCosmo, CWeb, load_library
    lib = load_library(LIB)
    h = ctypes.c_void_p()
    n = (ctypes.c_int * 1)(100)
    box = (ctypes.c_double * 1)(100.0)
    cc = CCosmo(0.31, 0.68, 0.81, 0.96, 1.0, 0.5, 4.0, -1, 0.0, 1e-6)
    cw = CWeb()
    cw.n_webs = 1
    cw.steepness, cw.lambda_th = 20.0, 0.1
    assert lib.fzw_plan_create(ctypes.byref(h), 1, n, box, ctypes.byref(cc), ctypes.byref(cw), None) == -2
    assert b"unsupported mesh size" in lib.fzw_last_error()
    cw.n_webs = 3
    n[0] = 32
    assert lib.fzw_plan_create(ctypes.byref(h), 1, n, box, ctypes.byref(cc), ctypes.byref(cw), None) == -1
    assert lib.fzw_plan_create(None, 1, n, box, ctypes.byref(cc), ctypes.byref(cw), None) == -1
    assert lib.fzw_forward(None, None, None, None, None) == -1


def test_fft_schedule_query_and_validation_without_gpu(lib):
    from paper_2506_03969_amd.fzw import load_library
    lib = load_library(LIB)
    z, xy, pure = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    us = (ctypes.c_double * 6)()
    # unsupported size; bad family codes
    assert lib.fzw_fft_schedule(100, ctypes.byref(z), ctypes.byref(xy), ctypes.byref(pure), us) == -1
    assert lib.fzw_set_fft_schedule(64, 2, 0, 0) == -1
    assert lib.fzw_set_fft_schedule(100, 0, 0, 0) == -1
    # a size no plan has used yet: defaults (four-step), reported as not tuned
    assert lib.fzw_fft_schedule(16, ctypes.byref(z), ctypes.byref(xy), ctypes.byref(pure), us) == -5
    assert (z.value, xy.value, pure.value) == (0, 0, 0)
    # setting by hand marks it as chosen
    assert lib.fzw_set_fft_schedule(16, 1, 1, 0) == 0
    assert lib.fzw_fft_schedule(16, ctypes.byref(z), ctypes.byref(xy), ctypes.byref(pure), None) == 0
    assert (z.value, xy.value, pure.value) == (1, 1, 0)


def test_dual_averaging_host_functions_match_the_oracle():
    """The library's host-side step-size adaptation follows the same
    recursion as the oracle's, to rounding."""
    import math
    from oracle import nuts
    from paper_2506_03969_amd import DualAveraging
    ours, ref = DualAveraging(0.3, 0.8), nuts.DualAveraging(0.3, 0.8)
    rng = np.random.default_rng(4)
    for a in rng.uniform(0.2, 1.0, size=200):
        assert ours.update(a) == pytest.approx(ref.update(a), rel=1e-12)
    assert ours.final() == pytest.approx(ref.final(), rel=1e-12)
    assert math.isfinite(ours.final())
