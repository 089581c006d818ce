"""GPU parity for F16 grids large enough that the library lays the kernels'
copy out in two-cell bricks (the one-cell copy, (n - 1)^3 cells of 16 bytes,
above 128 MiB: n >= 205), and a batch whose F16 scenes use both layouts.

The tiny room at n = 208: the kernels interpolate the F16 samples that
hyb_sdf_read returns (dequantized to FP32), and the oracle gets exactly those.
"""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

N = 208  # 207^3 * 16 B = 142 MB > 128 MiB
TMAX = 2.0


@pytest.fixture(scope="module")
def hyb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2305_07253_amd as hyb
    hyb.lib()
    return hyb


@pytest.fixture(scope="module")
def big(hyb, tiny):
    from paper_2305_07253_amd import workloads as W
    sc = tiny["scene"]
    g4 = W.room_grid(N)
    bvh = hyb.build_bvh(sc.verts, sc.tris)
    sdf = hyb.build_sdf(bvh, N, g4, fmt=hyb.SDF_F16)
    deq = np.ascontiguousarray(hyb.sdf_read(sdf).cpu().numpy())
    return dict(scene=sc, g4=g4, bvh=bvh, sdf=sdf, deq=deq)


def _dev(soa):
    import torch
    return torch.from_numpy(np.ascontiguousarray(soa, dtype=np.float32)).cuda()


@pytest.mark.parametrize("tau", [0.0, 1.0, 4.0])
def test_two_cell_f16_parity(hyb, orc, tiny, big, tau):
    sc = big["scene"]
    for name in ("free", "surf"):
        soa = np.ascontiguousarray(tiny[name].soa()[:, :2048])
        print("n=%d F16 tau %s rays %s" % (N, tau, name), flush=True)
        got = [x.cpu().numpy() for x in hyb.trace(big["bvh"], big["sdf"], _dev(soa), TMAX, tau)]
        ref = orc.query(sc.verts, sc.tris, big["deq"], big["g4"], soa, TMAX, tau)
        m, c = orc.margin(sc.verts, sc.tris, big["deq"], big["g4"], soa, TMAX, tau)
        parity.check(got, ref, m, c, label="n=%d F16 tau %s %s" % (N, tau, name))


def test_two_cell_f16_df_only(hyb, orc, tiny, big):
    sc = big["scene"]
    soa = np.ascontiguousarray(tiny["free"].soa()[:, :2048])
    got = [x.cpu().numpy() for x in hyb.trace_df(big["sdf"], _dev(soa), TMAX)]
    ref = orc.query(sc.verts, sc.tris, big["deq"], big["g4"], soa, TMAX, 0.0, mode=orc.MODE_DF)
    m, c = orc.margin(sc.verts, sc.tris, big["deq"], big["g4"], soa, TMAX, 0.0, mode=orc.MODE_DF)
    parity.check(got, ref, m, c, label="n=%d F16 DF only" % N)


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_batch_mixes_f16_layouts(hyb, tiny, big, graph):
    """A 32^3 F16 grid (one-cell bricks) and the 208^3 one (two-cell bricks)
    in one batch: every item bit for bit equal to its single-scene call."""
    import torch
    small = hyb.sdf_from_grid(_dev(tiny["grid"].reshape(-1)), tiny["grid4"], fmt=hyb.SDF_F16)
    specs = [(small, tiny["free"].soa(), 1.0), (big["sdf"], tiny["surf"].soa(), 0.0),
             (small, tiny["surf"].soa()[:, :3001], 0.0), (big["sdf"], tiny["free"].soa()[:, :999], 4.0)]
    items = [dict(bvh=big["bvh"], sdf=s, rays=_dev(r), tmax=TMAX, threshold=thr) for s, r, thr in specs]
    refs = [[x.cpu().numpy() for x in hyb.trace(it["bvh"], it["sdf"], it["rays"], TMAX, it["threshold"])]
            for it in items]
    b = hyb.Batch(items)
    b.launch(graph=graph)
    torch.cuda.synchronize()
    for k, (out, ref) in enumerate(zip(b.outs, refs)):
        got = [x.cpu().numpy() for x in out]
        for name, g, r in zip(("t", "prim", "u", "v"), got, ref):
            assert np.array_equal(g, r), (k, name)
