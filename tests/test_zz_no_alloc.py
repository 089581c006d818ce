"""GPU: hyb_batch_launch_static, the batch launch that allocates nothing
(its work counter and descriptor table in the library's fixed device array),
against hyb_batch_launch_eager, the launch of the same kernels by a batch that
allocated them: every output bit for bit, on two calls in a row, the second
with fewer items and fewer rays (the array keeps the first call's contents),
in two launch shapes; and the size limit rejected before any work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TMAX = 2.0


@pytest.fixture(scope="module")
def hyb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2305_07253_amd as hyb
    hyb.lib()
    return hyb


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def scenes(hyb, orc, tiny):
    from paper_2305_07253_amd import workloads as W
    a = dict(scene=tiny["scene"], g4=tiny["grid4"], grid=tiny["grid"])
    sb = W.make_scene(5, 40, 0.03, 0.1, box_subdiv=1, ico_splits=1)
    g4b = W.room_grid(48)
    b = dict(scene=sb, g4=g4b, grid=orc.sdf_grid(sb, g4b, 48))
    for s in (a, b):
        s["bvh"] = hyb.build_bvh(s["scene"].verts, s["scene"].tris)
        s["sdf"] = hyb.sdf_from_grid(to_dev(s["grid"].reshape(-1)), s["g4"], lipschitz_samples=True)
    rng = np.random.default_rng(8)
    free_b = W.uniform_rays(sb, 9000, 24).soa()
    tmin = to_dev((0.05 * rng.random(9000)).astype(np.float32))
    tmax_ray = to_dev((0.3 + 1.7 * rng.random(9000)).astype(np.float32))
    surf_b = W.offset_rays(W.surface_points(sb, 3000, 25), 1e-5, 26).soa()
    return dict(a=a, b=b, specs=[
        (a, tiny["free"].soa(), 1.0, "both", None, None),
        (b, surf_b, 0.0, "both", None, None),
        (a, np.zeros((6, 0), np.float32), 2.0, "both", None, None),
        (b, free_b[:, :777], np.inf, "bvh", None, None),
        (a, tiny["surf"].soa()[:, :4001], 0.0, "df", None, None),
        (b, free_b, 4.0, "both", tmin, tmax_ray),
        (a, tiny["free"].soa()[:, 5:6], 0.5, "both", None, None),
    ])


def items_of(specs):
    return [dict(bvh=None if kind == "df" else s["bvh"], sdf=None if kind == "bvh" else s["sdf"], rays=to_dev(soa),
                 tmax=TMAX, threshold=tau, tmin=tmin, tmax_ray=tmax_ray)
            for s, soa, tau, kind, tmin, tmax_ray in specs]


def results(outs):
    return [[x.cpu().numpy() for x in out] for out in outs]


@pytest.mark.parametrize("config", [None, dict(lds_depth=8, rays_per_item=64, blocks_per_cu=2)])
def test_static_launch_equals_batch_launch(hyb, scenes, config):
    import torch
    specs = scenes["specs"]
    # a smaller second call: fewer items, fewer rays per item
    small = [(s, soa[:, :max(0, soa.shape[1] // 3)], tau, kind,
              None if t0 is None else t0[:max(0, soa.shape[1] // 3)],
              None if t1 is None else t1[:max(0, soa.shape[1] // 3)])
             for s, soa, tau, kind, t0, t1 in specs[1:5]]
    for case in (specs, small):
        ref_items = items_of(case)
        batch = hyb.Batch(ref_items)
        if config is not None:
            batch.config = config
        ref = results(batch.launch(graph=False))
        got_items = items_of(case)
        for it in got_items:
            it["out"] = tuple(torch.full((it["rays"].shape[1],), 7, dtype=d, device="cuda")
                              for d in (torch.float32, torch.int32, torch.float32, torch.float32))
        got = results(hyb.batch_launch_static(got_items, config=config))
        assert len(got) == len(ref)
        for k, (g, r) in enumerate(zip(got, ref)):
            for j, (x, y) in enumerate(zip(g, r)):
                assert np.array_equal(x, y), (len(case), k, j)
        # the rays were traced: not every item left its buffers untouched
        assert any((r[1] != -1).any() for r in ref if len(r[1]))


def test_static_launch_limits(hyb, scenes):
    L = hyb.lib()
    import paper_2305_07253_amd as H
    arr, keep, outs = H._batch_items(items_of(scenes["specs"][:1]))
    assert L.hyb_batch_launch_static(None, 1, None, None) == 1
    assert L.hyb_batch_launch_static(arr, 0, None, None) == 1
    big = (H._BatchItem * (H.STATIC_BATCH_MAX_ITEMS + 1))()
    for k in range(len(big)):
        big[k] = arr[0]
    assert L.hyb_batch_launch_static(big, H.STATIC_BATCH_MAX_ITEMS + 1, None, None) == 1
    bad = H._BatchConfig(12, 256, 4)
    assert L.hyb_batch_launch_static(arr, 1, ctypes.byref(bad), None) == 1
    # the maximum itself is accepted (the same item 256 times)
    assert L.hyb_batch_launch_static(big, H.STATIC_BATCH_MAX_ITEMS, None, None) == 0
    import torch
    torch.cuda.synchronize()
    del keep
