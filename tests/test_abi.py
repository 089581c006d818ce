"""The C-ABI library loads and exports every function include/hyb.h declares;
argument validation that returns before any device work.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hyb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hyb_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2305_07253_amd as hyb
    if not os.path.exists(hyb.LIB_PATH):
        from paper_2305_07253_amd import build
        build.build()
    return hyb.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code, name in enumerate(["HYB_OK", "HYB_ERR_INVALID_ARG", "HYB_ERR_OOM", "HYB_ERR_HIP", "HYB_ERR_UNSUPPORTED"]):
        assert lib.hyb_status_str(code).decode() == name


def test_invalid_arguments_rejected_before_device_work(lib):
    P = ctypes.c_void_p
    out = P()
    # NULL output pointer / NULL handles
    assert lib.hyb_build_bvh(None, 0, None, 0, None, None) == 1
    assert lib.hyb_trace(None, None, None, 1, 1.0, 1.0, None, None) == 1
    assert lib.hyb_trace_bvh(None, None, 1, 1.0, None, None) == 1
    assert lib.hyb_trace_df(None, None, 1, 1.0, None, None) == 1
    assert lib.hyb_build_sdf(None, 32, None, 0, 0, None, ctypes.byref(out)) == 1
    assert lib.hyb_sdf_info(None, None, None, None) == 1
    assert lib.hyb_bvh_destroy(None) == 1 and lib.hyb_sdf_destroy(None) == 1
    # non-finite vertex, out-of-range index, negative counts
    v = np.array([[0, 0, 0], [1, 0, 0], [0, np.nan, 0]], np.float32)
    t = np.array([[0, 1, 2]], np.int32)
    vp, tp = v.ctypes.data_as(P), t.ctypes.data_as(P)
    assert lib.hyb_build_bvh(vp, 3, tp, 1, None, ctypes.byref(out)) == 1
    v[2, 1] = 1.0
    t[0, 2] = 7
    assert lib.hyb_build_bvh(vp, 3, tp, 1, None, ctypes.byref(out)) == 1
    assert lib.hyb_build_bvh(vp, -1, tp, 1, None, ctypes.byref(out)) == 1
    # bad grids for hyb_sdf_from_grid
    g = np.array([0, 0, 0, -1], np.float32)
    assert lib.hyb_sdf_from_grid(P(1), 8, g.ctypes.data_as(P), 0, 0, None, ctypes.byref(out)) == 1
    g[3] = 0.1
    assert lib.hyb_sdf_from_grid(P(1), 8, g.ctypes.data_as(P), 8, 0, None, ctypes.byref(out)) == 1  # unknown flag
    g[3] = np.inf
    assert lib.hyb_sdf_from_grid(P(1), 8, g.ctypes.data_as(P), 0, 0, None, ctypes.byref(out)) == 1


def test_python_binding_validates(lib):
    import paper_2305_07253_amd as hyb
    with pytest.raises(ValueError):
        hyb._query_args(float("nan"), 1.0)
    with pytest.raises(ValueError):
        hyb._query_args(1.0, -1.0)
    with pytest.raises(hyb.HybError):
        hyb.build_bvh(np.array([[0, 0, 0]], np.float32), np.array([[0, 0, 5]], np.int32))
