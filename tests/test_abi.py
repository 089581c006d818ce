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
    h = ctypes.c_float()
    assert lib.hyb_sdf_voxel_size(None, ctypes.byref(h)) == 1
    assert lib.hyb_sdf_check(None, None) == 1
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


def test_batch_arguments_rejected_before_device_work(lib):
    import paper_2305_07253_amd as hyb
    P = ctypes.c_void_p
    out = P()
    items = (hyb._BatchItem * 2)()
    assert lib.hyb_batch_create(None, 1, None, ctypes.byref(out)) == 1
    assert lib.hyb_batch_create(items, 0, None, ctypes.byref(out)) == 1
    assert lib.hyb_batch_create(items, 1 << 17, None, ctypes.byref(out)) == 1
    assert lib.hyb_batch_create(items, 1, None, None) == 1
    assert lib.hyb_batch_create(items, 2, None, ctypes.byref(out)) == 1  # neither bvh nor sdf
    cfg = hyb._BatchConfig(16, 256, 4)
    assert lib.hyb_batch_set_config(None, ctypes.byref(cfg)) == 1
    assert lib.hyb_batch_get_config(None, ctypes.byref(cfg)) == 1
    assert lib.hyb_batch_set_threshold(None, 0, 1.0) == 1
    assert lib.hyb_batch_get_threshold(None, 0, None) == 1
    assert lib.hyb_batch_launch(None, None) == 1
    assert lib.hyb_batch_launch_eager(None, None) == 1
    opts = hyb._TuneOpts(None, 0, 0.01, 3, 3)
    assert lib.hyb_batch_tune(None, ctypes.byref(opts), None, None, None) == 1
    assert lib.hyb_batch_destroy(None) == 1


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes
    and field offsets."""
    import subprocess
    import paper_2305_07253_amd as hyb
    mirrors = {"hyb_rays": hyb._Rays, "hyb_hits": hyb._Hits, "hyb_batch_item": hyb._BatchItem,
               "hyb_batch_config": hyb._BatchConfig, "hyb_batch_tune_opts": hyb._TuneOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hyb.h"', "int main(void) {"]
    for c, m in mirrors.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (c, c))
        for f, _ in m._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (c, f, c, f))
    lines.append("return 0; }")
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines))
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True,
                                                 check=True).stdout.splitlines())
    for c, m in mirrors.items():
        assert int(got[c]) == ctypes.sizeof(m), c
        for f, _ in m._fields_:
            assert int(got["%s.%s" % (c, f)]) == getattr(m, f).offset, (c, f)
