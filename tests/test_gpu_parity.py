"""GPU parity: the HIP kernels through the C ABI against the FP64 oracle.

Tiny room (1,052 triangles, 32^3 grid) at every threshold, the pure baselines,
the distance-field build, ragged and degenerate inputs, and the GI-shaped
workload (188k triangles, 128^3 grid, 2.07M G-buffer rays) traced in full in
the launch configuration the benchmark times and compared on a sampled
subset."""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

TAUS = (0.0, 0.5, 1.0, 2.0, 4.0, np.inf)


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


def host(out):
    return [x.cpu().numpy() for x in out]


@pytest.fixture(scope="module")
def tiny_dev(hyb, tiny):
    sc = tiny["scene"]
    bvh = hyb.build_bvh(sc.verts, sc.tris)
    sdf = hyb.sdf_from_grid(to_dev(tiny["grid"].reshape(-1)), tiny["grid4"])
    # the oracle's grid is exact, so it may be certified (longer safe steps)
    sdf_c = hyb.sdf_from_grid(to_dev(tiny["grid"].reshape(-1)), tiny["grid4"], lipschitz_samples=True)
    return dict(bvh=bvh, sdf=sdf, sdf_c=sdf_c, free=to_dev(tiny["free"].soa()), surf=to_dev(tiny["surf"].soa()))


@pytest.mark.parametrize("grid_kind", ["sdf", "sdf_c"])
@pytest.mark.parametrize("which", ["free", "surf"])
@pytest.mark.parametrize("tau", TAUS)
def test_tiny_combined(hyb, orc, tiny, tiny_dev, which, tau, grid_kind):
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    s = tiny[which].soa()
    got = host(hyb.trace(tiny_dev["bvh"], tiny_dev[grid_kind], tiny_dev[which], 2.0, tau))
    ref = orc.query(sc.verts, sc.tris, grid, g4, s, 2.0, tau)
    m, c = orc.margin(sc.verts, sc.tris, grid, g4, s, 2.0, tau)
    st = parity.check(got, ref, m, c, label="gpu tiny %s tau=%s %s" % (which, tau, grid_kind))
    print("tiny", which, tau, grid_kind, st)


@pytest.mark.parametrize("which", ["free", "surf"])
def test_tiny_pure_and_limits(hyb, orc, tiny, tiny_dev, which):
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    s = tiny[which].soa()
    bvh = host(hyb.trace_bvh(tiny_dev["bvh"], tiny_dev[which], 2.0))
    df = host(hyb.trace_df(tiny_dev["sdf"], tiny_dev[which], 2.0))
    for got, mode in ((bvh, 1), (df, 2)):
        ref = orc.query(sc.verts, sc.tris, grid, g4, s, 2.0, 0.0, mode=mode)
        m, c = orc.margin(sc.verts, sc.tris, grid, g4, s, 2.0, 0.0, mode=mode)
        parity.check(got, ref, m, c, label="gpu pure mode %d" % mode)
    # threshold 0 / +inf equal the pure kernels bit for bit
    c0 = host(hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], tiny_dev[which], 2.0, 0.0))
    ci = host(hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], tiny_dev[which], 2.0, np.inf))
    for a, b in zip(c0, df):
        assert np.array_equal(a, b)
    for a, b in zip(ci, bvh):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_tiny_inflated_bound(hyb, orc, tiny, tiny_dev, fmt):
    """One extreme sample far outside the room (1000 at node (0, 0, 0)) makes
    the grid's bounds huge (L about 4.7e4): every sphere step would be a tiny
    fraction of a cell, so the march takes cell steps and still ends at the
    oracle's first root on every decided ray, within one fetch per crossed
    cell and without NaN; the voxel size reported is the grid's h."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    grid = tiny["grid"].copy()
    grid.reshape(-1)[0] = 1000.0
    sdf = hyb.sdf_from_grid(to_dev(grid.reshape(-1)), g4, fmt=fmt)
    assert sdf.lipschitz > 1e4 and sdf.h == g4[3]
    deq = orc.quantize(grid, fmt)[0] if fmt else grid
    N = grid.shape[0]
    for which in ("free", "surf"):
        s = tiny[which].soa()
        for tau in (0.0, 1.0):
            got = host(hyb.trace(tiny_dev["bvh"], sdf, tiny_dev[which], 2.0, tau))
            ref = orc.query(sc.verts, sc.tris, deq, g4, s, 2.0, tau)
            m, c = orc.margin(sc.verts, sc.tris, deq, g4, s, 2.0, tau)
            st = parity.check(got, ref, m, c, label="gpu outlier fmt %d %s tau=%s" % (fmt, which, tau))
            assert not np.isnan(got[0]).any()
            print("outlier", fmt, which, tau, st)
        (_, prim, _, _), cnt = hyb.trace_counters(tiny_dev["bvh"], sdf, tiny_dev[which], 2.0, 0.0, hyb.MODE_DF)
        assert cnt.cpu().numpy()[:, 2].max() <= 3 * N


def test_tiny_counters_early_exit(hyb, tiny_dev):
    (t, prim, u, v), cnt = hyb.trace_counters(tiny_dev["bvh"], tiny_dev["sdf"], tiny_dev["surf"], 2.0, 2.0)
    prim, cnt = prim.cpu().numpy(), cnt.cpu().numpy()
    assert (prim >= 0).sum() > 100
    assert np.all(cnt[prim >= 0, 2] == 0)  # first hit in order: no DF work after a triangle hit
    assert np.all(cnt[prim == -2, 2] > 0)
    plain = host(hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], tiny_dev["surf"], 2.0, 2.0))
    assert np.array_equal(plain[1], prim)


def test_tiny_sdf_build(hyb, tiny):
    """hyb_build_sdf (FP64 on the GPU) against the oracle's exact grid."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    bvh = hyb.build_bvh(sc.verts, sc.tris)
    sdf = hyb.build_sdf(bvh, 32, g4, exterior_solid=True)
    got = hyb.sdf_read(sdf).cpu().numpy()
    ref = tiny["grid"]
    ulp = np.maximum(np.spacing(np.abs(ref).astype(np.float32)), 1e-15)
    assert np.all(np.abs(got.astype(np.float64) - ref) <= ulp)
    far = np.abs(ref) > 1e-6
    assert np.array_equal(np.sign(got[far]), np.sign(ref[far]))
    assert abs(sdf.lipschitz - orc_lipschitz(tiny)) <= 1e-5


def orc_lipschitz(tiny):
    import oracle
    return oracle.lipschitz(tiny["grid"], np.float64(tiny["grid4"][3]))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 257, 1000])
def test_ragged_sizes(hyb, orc, tiny, tiny_dev, n):
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    r = tiny["surf"].subset(slice(0, n))
    got = host(hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], to_dev(r.soa()), 2.0, 1.0))
    ref = orc.query(sc.verts, sc.tris, grid, g4, r.soa(), 2.0, 1.0)
    m, c = orc.margin(sc.verts, sc.tris, grid, g4, r.soa(), 2.0, 1.0)
    parity.check(got, ref, m, c, label="ragged %d" % n, max_excluded=1.0)


def test_edge_arguments(hyb, orc, tiny, tiny_dev):
    import torch
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    empty = torch.zeros((6, 0), dtype=torch.float32, device="cuda")
    out = hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], empty, 1.0, 1.0)  # n = 0: no-op
    assert out[0].numel() == 0
    with pytest.raises(ValueError):
        hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], tiny_dev["free"], float("nan"), 1.0)
    with pytest.raises(ValueError):
        hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], tiny_dev["free"], 1.0, -1.0)
    # per-ray tmin, including tmin > tmax (a miss, not an error), and tmax = +inf
    r = tiny["free"].subset(slice(0, 512))
    tmin = np.linspace(0.0, 2.5, 512).astype(np.float32)
    for tmax in (2.0, np.inf):
        got = host(hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], to_dev(r.soa()), tmax, 1.0, tmin=to_dev(tmin)))
        ref = orc.query(sc.verts, sc.tris, grid, g4, r.soa(), tmax, 1.0, tmin=tmin)
        m, c = orc.margin(sc.verts, sc.tris, grid, g4, r.soa(), tmax, 1.0, tmin=tmin)
        parity.check(got, ref, m, c, label="tmin tmax=%s" % tmax, max_excluded=0.1)
    got = host(hyb.trace(tiny_dev["bvh"], tiny_dev["sdf"], to_dev(r.soa()), 2.0, 1.0, tmin=to_dev(tmin)))
    assert np.all(got[1][tmin > 2.0] == -1)
    # more rays than one call takes (HYB_MAX_RAYS = 2^31 - 1): rejected before
    # anything is read, so small buffers stand in
    import ctypes
    R = to_dev(r.soa())
    rs, _ = hyb._rays_struct(R, None)
    out = hyb.alloc_hits(r.n)
    hs = hyb._hits_struct(out, r.n)
    for fn, args in (("hyb_trace", (tiny_dev["bvh"].handle, tiny_dev["sdf"].handle)),
                     ("hyb_trace_bvh", (tiny_dev["bvh"].handle,)), ("hyb_trace_df", (tiny_dev["sdf"].handle,))):
        extra = (ctypes.c_float(1.0),) if fn == "hyb_trace" else ()
        st = getattr(hyb.lib(), fn)(*args, ctypes.byref(rs), ctypes.c_int64(2 ** 31), ctypes.c_float(1.0), *extra,
                                    ctypes.byref(hs), None)
        assert st == 1, (fn, st)  # HYB_ERR_INVALID_ARG


def test_empty_and_degenerate_meshes(hyb, orc):
    rng = np.random.default_rng(3)
    o = rng.uniform(0, 1, (300, 3)).astype(np.float32)
    d = rng.normal(size=(300, 3)).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    s = np.ascontiguousarray(np.concatenate([o.T, d.T]).astype(np.float32))
    bvh = hyb.build_bvh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    got = host(hyb.trace_bvh(bvh, to_dev(s), 10.0))
    assert np.all(got[1] == -1) and np.all(np.isinf(got[0]))
    # a degenerate (zero-area) triangle is never hit; a real one is
    v = np.array([[0.2, 0.2, 0.5], [0.8, 0.3, 0.5], [0.4, 0.9, 0.5], [0.5, 0.5, 0.5]], np.float32)
    tris = np.array([[0, 1, 2], [3, 3, 3], [0, 0, 1]], np.int32)
    bvh = hyb.build_bvh(v, tris)
    got = host(hyb.trace_bvh(bvh, to_dev(s), 10.0))
    ref = orc.query(v, tris, None, None, s, 10.0, np.inf, mode=1)
    m, c = orc.margin(v, tris, None, None, s, 10.0, np.inf, mode=1)
    parity.check(got, ref, m, c, label="degenerate", max_excluded=0.2)
    assert set(np.unique(got[1])) <= {-1, 0}


# ---------------------------------------------------------------------------
# GI-shaped workload: full size on the GPU, sampled rays against the oracle
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def gi(hyb, orc, gi_exact):
    from paper_2305_07253_amd import workloads as W
    sc = gi_exact["scene"]
    g4 = gi_exact["g4"]
    gb = W.gbuffer(sc, 1920, 1080)
    rays = W.gbuffer_rays(gb, 21)
    bvh = hyb.build_bvh(sc.verts, sc.tris)
    sdf = hyb.build_sdf(bvh, 128, g4, exterior_solid=True)
    sample = np.arange(0, rays.n, 32 * 16)  # 4,050 rays, fixed stride in tile order
    oracle_grid = gi_exact["grid"]
    return dict(scene=sc, g4=g4, rays=rays, bvh=bvh, sdf=sdf, dev=to_dev(rays.soa()), sample=sample,
                oracle_grid=oracle_grid)


def test_gi_sdf_build_all_nodes(hyb, orc, gi):
    """Every node of the GPU-built 128^3 grid against the oracle's exact grid."""
    got = hyb.sdf_read(gi["sdf"]).cpu().numpy()
    ref = gi["oracle_grid"]
    ulp = np.maximum(np.spacing(np.abs(ref).astype(np.float32)), 1e-15)
    bad = np.abs(got.astype(np.float64) - ref.astype(np.float64)) > ulp
    assert bad.sum() == 0, (bad.sum(), np.argwhere(bad)[:5])
    far = np.abs(ref) > 1e-6
    assert np.array_equal(np.sign(got[far]), np.sign(ref[far]))


@pytest.mark.parametrize("tau", [0.0, 0.5, 1.0, 2.0, 4.0, np.inf])
def test_gi_full_launch_parity(hyb, orc, gi, tau):
    """All 2,073,600 rays traced in one launch through the GPU-built grid, as
    the benchmark times them, against the oracle on its own exact grid: every
    ray at threshold 0 (the distance-field query the headline measures),
    65,536 rays at a fixed stride in tile order at thresholds 0.5, 1 and 2
    (both techniques on one ray), 4,050 at 4 and +inf (whose triangle
    segments make the brute-force oracle slow)."""
    sc, g4 = gi["scene"], gi["g4"]
    n = gi["rays"].n
    out = hyb.trace(gi["bvh"], gi["sdf"], gi["dev"], 0.5, tau)
    if tau == 0.0:
        sample = np.arange(n)
    elif tau in (0.5, 1.0, 2.0):
        sample = np.arange(65536) * (n // 65536)
    else:
        sample = gi["sample"]
    got = [x.cpu().numpy()[sample] for x in out]
    sub = gi["rays"].subset(sample)
    (ref, m, c), = parity.combined_oracle(orc, sc.verts, sc.tris, [gi["oracle_grid"]], g4, sub.soa(), 0.5, tau)
    st = parity.check(got, ref, m, c, label="gi tau=%s" % tau)
    print("gi", tau, st)


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_gi_kernels_equal_counter_kernels(hyb, gi, fmt):
    """The counters variant of each query (another instantiation of the same
    kernels) gives every one of the 2,073,600 results bit for bit, with and
    without a per-ray tmin and tmax, for all three storage formats."""
    import torch
    sdf = gi["sdf"] if fmt == 0 else hyb.sdf_from_grid(to_dev(gi["oracle_grid"].reshape(-1)), gi["g4"], fmt=fmt)
    n = gi["rays"].n
    rng = np.random.default_rng(17)
    tmin = to_dev(rng.uniform(0.0, 0.02, n).astype(np.float32))
    tmax_ray = to_dev(rng.uniform(0.1, 0.6, n).astype(np.float32))
    cases = [(0.0, hyb.MODE_COMBINED, None, None), (1.0, hyb.MODE_COMBINED, None, None),
             (0.5, hyb.MODE_COMBINED, tmin, tmax_ray), (0.0, hyb.MODE_DF, None, None)]
    for tau, mode, t0, t1 in cases:
        if mode == hyb.MODE_DF:
            got = hyb.trace_df(sdf, gi["dev"], 0.5, tmin=t0, tmax_ray=t1)
        else:
            got = hyb.trace(gi["bvh"], sdf, gi["dev"], 0.5, tau, tmin=t0, tmax_ray=t1)
        ref, cnt = hyb.trace_counters(gi["bvh"], sdf, gi["dev"], 0.5, tau, mode, tmin=t0, tmax_ray=t1)
        for g, r in zip(got, ref):
            assert torch.equal(g, r), (fmt, tau, mode)


# ---------------------------------------------------------------------------
# compact distance-field storage (F16, int8 with block scales)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fmt", [1, 2])
def test_formats_quantize_and_trace(hyb, orc, tiny, tiny_dev, fmt):
    """The library's conversion equals the oracle's definition bit for bit;
    traces interpolate exactly those values."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    sdf = hyb.sdf_from_grid(to_dev(tiny["grid"].reshape(-1)), g4, fmt=fmt)
    deq, _, _ = orc.quantize(tiny["grid"], fmt)
    got_grid = hyb.sdf_read(sdf).cpu().numpy()
    assert np.array_equal(got_grid, deq)
    assert abs(sdf.lipschitz - orc.lipschitz(deq, np.float64(g4[3]))) <= 1e-5
    for which in ("free", "surf"):
        for tau in (0.0, 1.0, np.inf):
            got = host(hyb.trace(tiny_dev["bvh"], sdf, tiny_dev[which], 2.0, tau))
            ref = orc.query(sc.verts, sc.tris, deq, g4, tiny[which].soa(), 2.0, tau)
            m, c = orc.margin(sc.verts, sc.tris, deq, g4, tiny[which].soa(), 2.0, tau)
            parity.check(got, ref, m, c, label="fmt %d %s tau %s" % (fmt, which, tau))


@pytest.mark.parametrize("fmt", [1, 2])
def test_formats_build_sdf(hyb, orc, tiny, fmt):
    """hyb_build_sdf with a compact format: the GPU's FP32 distances (within
    one ulp of the oracle's) converted by the format's rule; at most one
    quantisation step from the oracle's converted grid."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    bvh = hyb.build_bvh(sc.verts, sc.tris)
    got = hyb.sdf_read(hyb.build_sdf(bvh, 32, g4, fmt=fmt)).cpu().numpy().astype(np.float64)
    deq, _, scales = orc.quantize(tiny["grid"], fmt)
    if fmt == 1:
        step = np.maximum(np.spacing(np.abs(deq).astype(np.float16)).astype(np.float64), 2.0 ** -24)
    else:
        # the largest scale of the blocks holding each node (one step: a
        # value near a rounding or clamping boundary may go either way)
        nb = scales.shape[0]
        idx = np.arange(32)
        lo, hi = np.clip((idx - 1) // 8, 0, nb - 1), np.clip(idx // 8, 0, nb - 1)
        step = np.zeros((32, 32, 32))
        for bk in (lo, hi):
            for bj in (lo, hi):
                for bi in (lo, hi):
                    step = np.maximum(step, scales[np.ix_(bk, bj, bi)].astype(np.float64))
    assert np.all(np.abs(got - deq) <= step * (1 + 1e-6))
    assert (got == deq).mean() > 0.999


@pytest.mark.parametrize("fmt", [1, 2])
def test_gi_formats_full_launch(hyb, orc, gi, fmt):
    """All 2,073,600 GI rays through an F16 / I8 copy of the oracle's 128^3
    grid; 4,050 sampled rays against the oracle on the same dequantized grid."""
    sc, g4 = gi["scene"], gi["g4"]
    deq, _, _ = orc.quantize(gi["oracle_grid"], fmt)
    sdf = hyb.sdf_from_grid(to_dev(gi["oracle_grid"].reshape(-1)), g4, fmt=fmt)
    sub = gi["rays"].subset(gi["sample"])
    for tau in (0.0, 1.0):
        out = hyb.trace(gi["bvh"], sdf, gi["dev"], 0.5, tau)
        got = [x.cpu().numpy()[gi["sample"]] for x in out]
        ref = orc.query(sc.verts, sc.tris, deq, g4, sub.soa(), 0.5, tau)
        m, c = orc.margin(sc.verts, sc.tris, deq, g4, sub.soa(), 0.5, tau)
        parity.check(got, ref, m, c, label="gi fmt %d tau %s" % (fmt, tau))


@pytest.mark.parametrize("tau", [0.0, 1.0])
def test_formats_agree_on_a_lossless_grid(hyb, orc, tiny, tiny_dev, gi, tau):
    """Samples every format stores exactly (integer multiples of one power of
    two, at most 127 of them): the F16 and I8 kernels return the FP32
    kernel's hits bit for bit, on the tiny room and on all 2,073,600 GI rays
    with a lossless copy of the 128^3 grid."""
    cases = [(tiny_dev["bvh"], tiny["grid"], tiny["grid4"], tiny_dev["free"], 2.0),
             (tiny_dev["bvh"], tiny["grid"], tiny["grid4"], tiny_dev["surf"], 2.0),
             (gi["bvh"], gi["oracle_grid"], gi["g4"], gi["dev"], 0.5)]
    for bvh, grid, g4, rays, tmax in cases:
        g = parity.lossless_grid(grid)
        for fmt in (1, 2):
            deq, _, _ = orc.quantize(g, fmt)
            assert np.array_equal(deq, g)
        ref = host(hyb.trace(bvh, hyb.sdf_from_grid(to_dev(g.reshape(-1)), g4), rays, tmax, tau))
        assert (ref[1] == -2).sum() > 100
        for fmt in (1, 2):
            sdf = hyb.sdf_from_grid(to_dev(g.reshape(-1)), g4, fmt=fmt)
            got = host(hyb.trace(bvh, sdf, rays, tmax, tau))
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (fmt, tau, len(a))


# ---------------------------------------------------------------------------
# shadow-ray query: triangles at both ends, the distance field in between, any hit
# ---------------------------------------------------------------------------

def shadow_segments(g4, tmax, ts, te):
    h = np.float32(g4[3])
    t1 = np.minimum(np.float32(ts) * h, tmax).astype(np.float64)
    t2 = np.maximum((tmax - np.float32(te) * h).astype(np.float32).astype(np.float64), t1)
    return [(0.0, t1), (t2, tmax.astype(np.float64))]


@pytest.mark.parametrize("taus", [(0.0, 0.0), (1.0, 1.0), (2.0, 4.0), (np.inf, np.inf)])
def test_tiny_shadow(hyb, orc, tiny, tiny_dev, taus):
    from paper_2305_07253_amd import workloads as W
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    pts = W.surface_points(sc, 4096, 14)
    rays, tmax = W.shadow_rays(pts.p, pts.n, 15)
    s = rays.soa()
    ts, te = taus
    got = host(hyb.trace_shadow(tiny_dev["bvh"], tiny_dev["sdf"], to_dev(s), 10.0, ts, te, tmax_ray=to_dev(tmax)))
    ref = orc.query(sc.verts, sc.tris, grid, g4, s, 10.0, ts, mode=3, tmax_ray=tmax, tau_end=te)
    m, _ = orc.margin(sc.verts, sc.tris, grid, g4, s, 10.0, ts, mode=3, tmax_ray=tmax, tau_end=te)
    st = parity.check_shadow(got, ref, m, orc, sc.verts, sc.tris, s, shadow_segments(g4, tmax, ts, te),
                             label="gpu shadow %s" % (taus,))
    assert st["occluded"] > 200


def test_gi_shadow_full_launch(hyb, orc, gi):
    """Shadow rays from every G-buffer point to the area light, all 2,073,600
    in one launch; the fixed-stride sample against the oracle."""
    from paper_2305_07253_amd import workloads as W
    sc, g4 = gi["scene"], gi["g4"]
    gb = W.gbuffer(sc, 1920, 1080)
    rays, tmax = W.shadow_rays(gb.p, gb.n, 22)
    sub = rays.subset(gi["sample"])
    tsub = tmax[gi["sample"]]
    for ts, te in ((1.0, 1.0), (4.0, 2.0)):
        out = hyb.trace_shadow(gi["bvh"], gi["sdf"], to_dev(rays.soa()), 10.0, ts, te, tmax_ray=to_dev(tmax))
        got = [x.cpu().numpy()[gi["sample"]] for x in out]
        ref = orc.query(sc.verts, sc.tris, gi["oracle_grid"], g4, sub.soa(), 10.0, ts, mode=3, tmax_ray=tsub,
                        tau_end=te)
        m, _ = orc.margin(sc.verts, sc.tris, gi["oracle_grid"], g4, sub.soa(), 10.0, ts, mode=3, tmax_ray=tsub,
                          tau_end=te)
        parity.check_shadow(got, ref, m, orc, sc.verts, sc.tris, sub.soa(), shadow_segments(g4, tsub, ts, te),
                            label="gi shadow %s %s" % (ts, te))


# ---------------------------------------------------------------------------
# differentiable distance-field hit
# ---------------------------------------------------------------------------

def _well_posed(orc, tiny, face=1e-4, cond_min=1e-2):
    grid, g4 = tiny["grid"], tiny["grid4"]
    r = tiny["free"]
    s = r.soa()
    t = orc.df_hit(grid, g4, s, 0.0, 2.0)
    m, c = orc.margin(None, np.zeros((0, 3)), grid, g4, s, 2.0, 0.0, mode=orc.MODE_DF)
    p = r.o.astype(np.float64) + np.where(np.isfinite(t), t, 0)[:, None] * r.d.astype(np.float64)
    x = (p - np.float64(g4[0])) / np.float64(g4[3])
    return np.isfinite(t) & (t > 0) & (m > 1e-5) & (c > cond_min) & (np.abs(x - np.round(x)).min(axis=1) > face), t


def test_df_backward_vs_oracle_gradient(hyb, orc, tiny, tiny_dev):
    """d(sum of selected t) / d samples: GPU kernel (FP32, atomics) against the
    oracle's FP64 implicit derivatives accumulated at its own hits."""
    import torch
    grid, g4 = tiny["grid"], tiny["grid4"]
    sel, t_ref = _well_posed(orc, tiny)
    R = tiny_dev["free"]
    t, prim, _, _ = hyb.trace_df(tiny_dev["sdf"], R, 2.0)
    grad = torch.zeros(32 ** 3, dtype=torch.float32, device="cuda")
    hyb.df_backward(tiny_dev["sdf"], R, 2.0, t, to_dev(sel.astype(np.float32)), grad)
    got = grad.cpu().numpy().astype(np.float64)
    nodes, dt = orc.df_grad(grid, g4, tiny["free"].soa(), t_ref, 0.0, 2.0)
    ref = np.zeros(32 ** 3)
    keep = sel[:, None] & (nodes >= 0)
    np.add.at(ref, nodes[keep], dt[keep])
    scale = np.abs(ref).max()
    assert scale > 0.5 and (ref != 0).sum() > 1000
    assert np.abs(got - ref).max() <= 1e-4 * scale, np.abs(got - ref).max()
    # deterministic up to the order of float atomic additions
    grad2 = torch.zeros_like(grad)
    hyb.df_backward(tiny_dev["sdf"], R, 2.0, t, to_dev(sel.astype(np.float32)), grad2)
    assert torch.allclose(grad, grad2, rtol=1e-5, atol=1e-6 * scale)


def test_df_backward_long_runs_of_one_cell(hyb, orc, tiny, tiny_dev):
    """The backward sorts the rays by hit cell and sums each run of one cell
    inside a wavefront before adding: 40 well-posed rays repeated 1 to 150
    times (runs across several wavefronts), shuffled, 1,000 rays in all (a
    ragged last wavefront), each with its own grad_t, against the oracle's
    FP64 derivatives summed per copy."""
    import torch
    grid, g4 = tiny["grid"], tiny["grid4"]
    sel, t_ref = _well_posed(orc, tiny)
    base = np.nonzero(sel)[0][:40]
    rng = np.random.default_rng(11)
    reps = rng.integers(1, 60, size=len(base))
    reps[:3] = [150, 97, 64]
    idx = np.repeat(base, reps)
    idx = idx[rng.permutation(len(idx))][:1000]
    assert len(idx) == 1000
    gt = rng.standard_normal(len(idx)).astype(np.float32)
    R = to_dev(tiny["free"].subset(idx).soa())
    t, _, _, _ = hyb.trace_df(tiny_dev["sdf"], R, 2.0)
    grad = torch.zeros(32 ** 3, dtype=torch.float32, device="cuda")
    hyb.df_backward(tiny_dev["sdf"], R, 2.0, t, to_dev(gt), grad)
    got = grad.cpu().numpy().astype(np.float64)
    nodes, dt = orc.df_grad(grid, g4, tiny["free"].soa(), t_ref, 0.0, 2.0)
    ref = np.zeros(32 ** 3)
    keep = nodes[idx] >= 0
    np.add.at(ref, nodes[idx][keep], (gt.astype(np.float64)[:, None] * dt[idx])[keep])
    scale = np.abs(ref).max()
    assert scale > 0.5 and (ref != 0).sum() >= 8 * 30
    assert np.abs(got - ref).max() <= 1e-4 * scale, np.abs(got - ref).max()


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_df_backward_small_and_degenerate(hyb, orc, tiny, tiny_dev, n):
    """Ragged ray counts below one wavefront up to a few (the sort's
    single-block path), against the oracle; then rays that add nothing (all
    grad_t zero, or every ray a miss) leave the gradient untouched, and a
    second call with more rays than the first grows the handle's buffers."""
    import torch
    grid, g4 = tiny["grid"], tiny["grid4"]
    sel, t_ref = _well_posed(orc, tiny)
    idx = np.nonzero(sel)[0][:n]
    R = to_dev(tiny["free"].subset(idx).soa())
    sdf = hyb.sdf_from_grid(torch.from_numpy(grid.reshape(-1).copy()).cuda(), g4)
    t, _, _, _ = hyb.trace_df(sdf, R, 2.0)
    grad = torch.zeros(32 ** 3, dtype=torch.float32, device="cuda")
    hyb.df_backward(sdf, R, 2.0, t, torch.ones_like(t), grad)
    nodes, dt = orc.df_grad(grid, g4, tiny["free"].soa(), t_ref, 0.0, 2.0)
    ref = np.zeros(32 ** 3)
    keep = nodes[idx] >= 0
    np.add.at(ref, nodes[idx][keep], dt[idx][keep])
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(grad.cpu().numpy().astype(np.float64) - ref).max() <= 1e-4 * scale
    before = grad.clone()
    hyb.df_backward(sdf, R, 2.0, t, torch.zeros_like(t), grad)
    miss = torch.full_like(t, float("inf"))
    hyb.df_backward(sdf, R, 2.0, miss, torch.ones_like(t), grad)
    assert torch.equal(grad, before)
    # more rays than any call before on this handle: the buffers grow
    R2 = to_dev(tiny["free"].subset(np.nonzero(sel)[0][:4 * n + 64]).soa())
    t2, _, _, _ = hyb.trace_df(sdf, R2, 2.0)
    g2 = torch.zeros_like(grad)
    hyb.df_backward(sdf, R2, 2.0, t2, torch.ones_like(t2), g2)
    assert torch.count_nonzero(g2) >= torch.count_nonzero(grad)


def test_df_backward_finite_differences(hyb, orc, tiny):
    """Central differences through the GPU forward on 64 voxels with non-zero
    gradient (rays clear of cell faces and well conditioned)."""
    import torch
    g4 = tiny["grid4"]
    h = float(g4[3])
    sel, _ = _well_posed(orc, tiny, face=2e-2, cond_min=0.1)
    sub = tiny["free"].subset(np.nonzero(sel)[0])
    R = to_dev(sub.soa())
    theta = torch.from_numpy(tiny["grid"].reshape(-1).copy()).cuda()
    sdf = hyb.sdf_from_grid(theta, g4)
    t, _, _, _ = hyb.trace_df(sdf, R, 2.0)
    grad = torch.zeros_like(theta)
    hyb.df_backward(sdf, R, 2.0, t, torch.ones_like(t), grad)
    g = grad.cpu().numpy()
    cand = np.nonzero(np.abs(g) > 1e-2 * np.abs(g).max())[0]
    pick = np.random.default_rng(5).choice(cand, size=64, replace=False)
    delta = 2e-4 * h
    for j in pick:
        tp_theta = theta.clone(); tp_theta[j] += delta
        tm_theta = theta.clone(); tm_theta[j] -= delta
        tp = hyb.trace_df(hyb.sdf_from_grid(tp_theta, g4), R, 2.0)[0].double().sum().item()
        tm = hyb.trace_df(hyb.sdf_from_grid(tm_theta, g4), R, 2.0)[0].double().sum().item()
        fd = (tp - tm) / (2 * delta)
        assert abs(fd - g[j]) <= 2e-2 * abs(g[j]) + 2e-3, (j, fd, g[j])


def test_autograd_df_hit(hyb, tiny):
    import torch
    from paper_2305_07253_amd.autograd import df_hit
    g4 = tiny["grid4"]
    theta = torch.from_numpy(tiny["grid"].copy()).cuda().requires_grad_(True)
    R = to_dev(tiny["free"].soa())
    t = df_hit(theta, g4, R, 2.0)
    w = torch.linspace(0.5, 1.5, t.numel(), device="cuda")
    loss = (torch.where(torch.isfinite(t), t, torch.zeros_like(t)) * w).sum()
    loss.backward()
    sdf = hyb.sdf_from_grid(theta.detach().reshape(-1).contiguous(), g4)
    t2, _, _, _ = hyb.trace_df(sdf, R, 2.0)
    assert torch.equal(t.detach(), t2)
    ref = torch.zeros(32 ** 3, device="cuda")
    hyb.df_backward(sdf, R, 2.0, t2, torch.where(torch.isfinite(t2), w, torch.zeros_like(w)).contiguous(), ref)
    assert torch.allclose(theta.grad.reshape(-1), ref, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("n", [30, 33, 35])
def test_grid_sizes_with_partial_bricks(hyb, orc, tiny, tiny_dev, n):
    """Grid sides that are not a multiple of the 4-node brick or the 8-node
    I8 scale block, every storage format, against the oracle."""
    from paper_2305_07253_amd import workloads as W
    sc = tiny["scene"]
    g4 = W.room_grid(n)
    grid = orc.sdf_grid(sc, g4, n)
    s = tiny["free"].soa()
    for fmt in (0, 1, 2):
        sdf = hyb.sdf_from_grid(to_dev(grid.reshape(-1)), g4, fmt=fmt)
        deq = orc.quantize(grid, fmt)[0] if fmt else grid
        assert np.array_equal(hyb.sdf_read(sdf).cpu().numpy(), np.asarray(deq, np.float32).reshape(n, n, n))
        for tau in (0.0, 1.0):
            got = host(hyb.trace(tiny_dev["bvh"], sdf, tiny_dev["free"], 2.0, tau))
            ref = orc.query(sc.verts, sc.tris, deq, g4, s, 2.0, tau)
            m, c = orc.margin(sc.verts, sc.tris, deq, g4, s, 2.0, tau)
            parity.check(got, ref, m, c, label="gpu n=%d fmt %d tau %s" % (n, fmt, tau))
