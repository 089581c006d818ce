"""GPU parity at the full sizes of the precision, batch and differentiation
workloads, in the launch configurations the benchmark times, checked on
sampled outputs (the GI-shaped workload is in test_gpu_parity.py).

  precision  1,880,236 triangles, 256^3 grid, 8,294,400 rays, F32, F16 and
             I8 at thresholds 0 and 1: an 8,192-ray fixed-stride sample
             against the oracle, which computes its own exact samples at every
             node those rays reach before their first root
  batch      64 scenes, 6.5M triangles, 14.7M rays, one tuned graph launch:
             every item bit for bit equal to its single-scene call, and every
             scene against the oracle on 1,024 rays at its tuned threshold
  refit      128^3 learnable grid, 1,048,576 rays: the backward against the
             oracle's FP64 implicit derivatives and central differences on 64
             voxels
"""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

TMAX = 0.5


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


# ---------------------------------------------------------------------------
# precision workload
# ---------------------------------------------------------------------------

N_PREC = 8192


def coarse_fill(orc, scene, g4, n, step=4):
    """An oracle field for every node of an n^3 grid: exact signed distances
    on a grid `step` times coarser (node (i, j, k) step of it at the fine node
    of the same index times step), interpolated trilinearly to the fine
    nodes, in FP64."""
    m = (n - 1) // step + 2
    cg4 = np.array([g4[0], g4[1], g4[2], np.float32(g4[3]) * step], np.float32)
    coarse = orc.sdf_nodes(scene, cg4, m).reshape(m, m, m)  # [k, j, i]
    # the coarse spacing is fl32(h step) = h step exactly for step 4: fine
    # node i lies at coarse coordinate i / step
    assert np.float64(cg4[3]) == np.float64(g4[3]) * step
    x = np.arange(n) / step
    i0 = np.minimum(np.floor(x).astype(np.int64), m - 2)
    w = x - i0
    f = coarse[i0] * (1 - w)[:, None, None] + coarse[i0 + 1] * w[:, None, None]
    f = f[:, i0] * (1 - w)[None, :, None] + f[:, i0 + 1] * w[None, :, None]
    return f[:, :, i0] * (1 - w)[None, None, :] + f[:, :, i0 + 1] * w[None, None, :]


@pytest.fixture(scope="module")
def precision(hyb, orc):
    """The precision workload in the benchmark's launch configuration; the
    oracle's exact samples at every node of the cells that 8,192 sample rays
    cross up to their first root at thresholds 0 and 1; and, for the compact
    formats, a complete grid of those samples with the other nodes filled from
    a coarse exact grid (the same array goes to the library and the oracle, so
    an int8 block's scale sees the same nodes on both sides)."""
    from paper_2305_07253_amd import workloads as W
    scene = W.precision_scene(3)
    g4 = W.room_grid(256)
    rays = W.gbuffer_rays(W.gbuffer(scene, 1920, 1080), 31, spp=4)
    bvh = hyb.build_bvh(scene.verts, scene.tris)
    sdf = hyb.build_sdf(bvh, 256, g4)
    idx = np.linspace(0, rays.n - 1, N_PREC).astype(np.int64)
    sub = rays.subset(idx)
    t1 = parity.split_t1(1.0, g4[3], TMAX)
    both = np.concatenate([sub.soa(), sub.soa()], axis=1)
    og, _ = orc.sdf_grid_on_paths(scene, g4, 256, both, np.concatenate([np.zeros(sub.n), np.full(sub.n, t1)]), TMAX)
    filled = np.where(np.isnan(og), coarse_fill(orc, scene, g4, 256).astype(np.float32), og)
    return dict(scene=scene, g4=g4, R=to_dev(rays.soa()), n=rays.n, bvh=bvh, sdf=sdf, idx=idx, sub=sub, og=og,
                filled=filled, refs={})


def precision_refs(orc, P, tau):
    """Oracle results of the sample rays at one threshold for the exact grid
    (F32) and the compact formats' dequantized filled grid (the triangle
    sub-query computed once for all three)."""
    if tau not in P["refs"]:
        sc = P["scene"]
        grids = [P["og"], orc.quantize(P["filled"], 1)[0], orc.quantize(P["filled"], 2)[0]]
        P["refs"][tau] = parity.combined_oracle(orc, sc.verts, sc.tris, grids, P["g4"], P["sub"].soa(), TMAX, tau)
    return P["refs"][tau]


@pytest.mark.parametrize("fmt,tau", [(0, 0.0), (1, 0.0), (2, 0.0), (0, 1.0), (1, 1.0), (2, 1.0)])
def test_precision_full_launch_parity(hyb, orc, precision, fmt, tau):
    """All 8,294,400 rays (1,880,236 triangles, 256^3 grid) in one launch, in
    each storage format at thresholds 0 and 1, against the oracle on 8,192
    sample rays: FP32 through the GPU-built grid against the exact samples;
    F16 and I8 through the library's conversion of the filled grid against
    the oracle's conversion of the same grid."""
    P = precision
    assert P["n"] == 8294400 and P["scene"].n_tris == 1880236
    if fmt == 0:
        sdf = P["sdf"]
    else:
        sdf = hyb.sdf_from_grid(to_dev(P["filled"].reshape(-1)), P["g4"], fmt=fmt)
    out = hyb.trace(P["bvh"], sdf, P["R"], TMAX, tau)
    got = [x.cpu().numpy()[P["idx"]] for x in out]
    ref, m, c = precision_refs(orc, P, tau)[fmt]
    if fmt == 0:
        assert np.all(np.isfinite(ref[0]) | (ref[1] == -1)), "the oracle read a node it did not sample"
    st = parity.check(got, ref, m, c, label="precision fmt %d tau %s" % (fmt, tau))
    print("precision", fmt, tau, st)


# ---------------------------------------------------------------------------
# batch workload
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def batch64(hyb):
    from paper_2305_07253_amd import workloads as W
    items, meta = [], []
    for sp in W.batch_specs(4, 64):
        scene = W.batch_scene(sp)
        bvh = hyb.build_bvh(scene.verts, scene.tris)
        g4 = W.room_grid(sp.n_grid)
        sdf = hyb.build_sdf(bvh, sp.n_grid, g4)
        rays = W.gbuffer_rays(W.gbuffer(scene, sp.width, sp.height), sp.seed)
        items.append(dict(bvh=bvh, sdf=sdf, rays=to_dev(rays.soa()), tmax=TMAX, threshold=1.0))
        meta.append(dict(scene=scene, g4=g4, n_grid=sp.n_grid, rays=rays))
    return items, meta


def test_batch_full_workload(hyb, orc, batch64):
    import torch
    items, meta = batch64
    assert sum(m["rays"].n for m in meta) == 14658048
    b = hyb.Batch(items)
    err, ms = b.tune(max_error_rate=0.03, reps=2)
    assert np.all(err <= 0.03) and ms > 0
    for k in range(len(items)):
        b.outs[k][1].fill_(-99)
    torch.cuda.synchronize()
    b.launch()
    torch.cuda.synchronize()
    taus = [b.threshold(k) for k in range(len(items))]
    for k, it in enumerate(items):
        ref = hyb.trace(it["bvh"], it["sdf"], it["rays"], TMAX, taus[k])
        for g, r in zip(b.outs[k], ref):
            assert torch.equal(g, r), "item %d differs from its single-scene call" % k
    # every scene against the oracle on 1,024 rays at its tuned threshold,
    # with the oracle's exact samples on the cells those rays cross
    excluded = []
    for k in range(len(items)):
        m = meta[k]
        sc = m["scene"]
        idx = np.linspace(0, m["rays"].n - 1, 1024).astype(np.int64)
        s = m["rays"].subset(idx).soa()
        t1 = parity.split_t1(taus[k], m["g4"][3], TMAX)
        if t1 < TMAX or taus[k] == 0.0:
            grid, _ = orc.sdf_grid_on_paths(sc, m["g4"], m["n_grid"], s, np.full(1024, t1), TMAX)
        else:
            grid = None  # triangles only
        got = [x.cpu().numpy()[idx] for x in b.outs[k]]
        (ref, mg, c), = parity.combined_oracle(orc, sc.verts, sc.tris, [grid], m["g4"], s, TMAX, taus[k])
        st = parity.check(got, ref, mg, c, label="batch scene %d (%d triangles, tau %s)" % (k, sc.n_tris, taus[k]))
        excluded.append(st["excluded"])
        print("batch scene", k, sc.n_tris, m["n_grid"], taus[k], st, flush=True)
    assert np.mean(excluded) < 0.02


# ---------------------------------------------------------------------------
# differentiation workload
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def refit(hyb, orc, gi_exact):
    from paper_2305_07253_amd import workloads as W
    scene, g4, grid = gi_exact["scene"], gi_exact["g4"], gi_exact["grid"]
    h = float(g4[3])
    gb = W.gbuffer(scene, 1024, 1024)
    rays = W.rebias(W.gbuffer_rays(gb, 41), gb, h)
    s = rays.soa()
    t_ref = orc.df_hit(grid, g4, s, 0.0, TMAX)
    m, c = orc.margin(None, np.zeros((0, 3)), grid, g4, s, TMAX, 0.0, mode=orc.MODE_DF)
    p = rays.o.astype(np.float64) + np.where(np.isfinite(t_ref), t_ref, 0)[:, None] * rays.d.astype(np.float64)
    x = (p - np.float64(g4[0])) / np.float64(g4[3])
    face = np.abs(x - np.round(x)).min(axis=1)
    return dict(g4=g4, h=h, rays=rays, grid=grid, t_ref=t_ref, m=m, c=c, face=face, R=to_dev(s))


def test_refit_backward_vs_oracle_gradient(hyb, orc, refit):
    import torch
    F = refit
    assert F["rays"].n == 1048576
    sel = np.isfinite(F["t_ref"]) & (F["t_ref"] > 0) & (F["m"] > 1e-5) & (F["c"] > 1e-2) & (F["face"] > 1e-4)
    theta = to_dev(F["grid"].reshape(-1))
    sdf = hyb.sdf_from_grid(theta, F["g4"])
    t, _, _, _ = hyb.trace_df(sdf, F["R"], TMAX)
    grad = torch.zeros_like(theta)
    hyb.df_backward(sdf, F["R"], TMAX, t, to_dev(sel.astype(np.float32)), grad)
    got = grad.cpu().numpy().astype(np.float64)
    nodes, dt = orc.df_grad(F["grid"], F["g4"], F["rays"].soa(), F["t_ref"], 0.0, TMAX)
    ref = np.zeros(128 ** 3)
    keep = sel[:, None] & (nodes >= 0)
    np.add.at(ref, nodes[keep], dt[keep])
    scale = np.abs(ref).max()
    assert (ref != 0).sum() > 100000
    assert np.abs(got - ref).max() <= 1e-4 * scale, np.abs(got - ref).max() / scale


def test_refit_finite_differences(hyb, refit):
    import torch
    F = refit
    g4, h = F["g4"], F["h"]
    sel = np.isfinite(F["t_ref"]) & (F["t_ref"] > 0) & (F["m"] > 1e-5) & (F["c"] > 0.1) & (F["face"] > 2e-2)
    sub = F["rays"].subset(np.nonzero(sel)[0])
    R = to_dev(sub.soa())
    theta = to_dev(F["grid"].reshape(-1))
    sdf = hyb.sdf_from_grid(theta, g4)
    t, _, _, _ = hyb.trace_df(sdf, R, TMAX)
    grad = torch.zeros_like(theta)
    hyb.df_backward(sdf, R, TMAX, t, torch.ones_like(t), grad)
    g = grad.cpu().numpy()
    # corner nodes of each ray's hit cell: the rays whose t depends on a node
    th = t.cpu().numpy().astype(np.float64)
    p = sub.o.astype(np.float64) + th[:, None] * sub.d.astype(np.float64)
    cell = np.clip(np.floor((p - g4[:3].astype(np.float64)) / np.float64(h)).astype(np.int64), 0, 126)
    corner = np.stack([(cell[:, 0] + dx) + 128 * ((cell[:, 1] + dy) + 128 * (cell[:, 2] + dz))
                       for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], axis=1)
    cand = np.nonzero(np.abs(g) > 1e-2 * np.abs(g).max())[0]
    pick = np.random.default_rng(6).choice(cand, size=64, replace=False)
    delta = 2e-4 * h
    for j in pick:
        rays_j = torch.from_numpy(np.nonzero((corner == j).any(axis=1))[0]).cuda()
        tp_theta = theta.clone()
        tp_theta[j] += delta
        tm_theta = theta.clone()
        tm_theta[j] -= delta
        tp = hyb.trace_df(hyb.sdf_from_grid(tp_theta, g4), R, TMAX)[0][rays_j].double().sum().item()
        tm = hyb.trace_df(hyb.sdf_from_grid(tm_theta, g4), R, TMAX)[0][rays_j].double().sum().item()
        fd = (tp - tm) / (2 * delta)
        assert abs(fd - g[j]) <= 2e-2 * abs(g[j]) + 2e-3, (j, fd, g[j])
