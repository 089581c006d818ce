"""The library's kernel bodies, compiled for the host (with AddressSanitizer and
UBSan on), against the FP64 oracle on the tiny room at every threshold.  This
checks the kernel logic and its memory accesses without a GPU; the GPU tests
repeat the comparison on the device."""
import numpy as np
import pytest

from tests.emu import runner
from tests import parity

TAUS = (0.0, 0.5, 1.0, 2.0, 4.0, np.inf)


@pytest.fixture(scope="module")
def emu():
    runner.build()
    return runner


@pytest.mark.parametrize("certified", [False, True])
@pytest.mark.parametrize("which", ["free", "surf"])
@pytest.mark.parametrize("tau", TAUS)
def test_combined_matches_oracle(emu, orc, tiny, which, tau, certified):
    """certified: the grid is exact, so the tracer may also step by g - 2E."""
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    rays = tiny[which]
    got = emu.trace(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, tau, certified=certified)
    ref = orc.query(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, tau)
    m, c = orc.margin(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, tau)
    parity.check(got, ref, m, c, label="emu %s tau=%s certified=%s" % (which, tau, certified))


@pytest.mark.parametrize("fmt", [1, 2, 3])
@pytest.mark.parametrize("tau", [0.0, 1.0, 4.0])
def test_compact_formats_match_oracle(emu, orc, tiny, fmt, tau):
    """F16 and I8 grids: the kernels interpolate the dequantized values, which
    the oracle computes by the same definition (3: F16 in the two-cell bricks
    the library uses for large grids)."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    deq, _, _ = orc.quantize(tiny["grid"], 1 if fmt == 3 else fmt)
    for rays in (tiny["free"], tiny["surf"]):
        got = emu.trace(sc.verts, sc.tris, tiny["grid"], g4, rays.soa(), 2.0, tau, fmt=fmt)
        ref = orc.query(sc.verts, sc.tris, deq, g4, rays.soa(), 2.0, tau)
        m, c = orc.margin(sc.verts, sc.tris, deq, g4, rays.soa(), 2.0, tau)
        parity.check(got, ref, m, c, label="emu fmt %d tau %s" % (fmt, tau))


@pytest.mark.parametrize("tau", [0.0, 1.0])
def test_formats_agree_on_a_lossless_grid(emu, orc, tiny, tau):
    """On samples every format stores exactly, the F16 (one- and two-cell
    bricks) and I8 kernel bodies return the FP32 body's hits bit for bit:
    their decoding, the I8 scale applied after interpolating the codes and
    the brick layouts change no value the march computes."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    g = parity.lossless_grid(tiny["grid"])
    for fmt in (1, 2):
        deq, _, _ = orc.quantize(g, fmt)
        assert np.array_equal(deq, g)
    for rays in (tiny["free"], tiny["surf"]):
        ref = emu.trace(sc.verts, sc.tris, g, g4, rays.soa(), 2.0, tau)
        assert (ref[1] == -2).sum() > 100  # the distance field decides many rays
        for fmt in (1, 2, 3):
            got = emu.trace(sc.verts, sc.tris, g, g4, rays.soa(), 2.0, tau, fmt=fmt)
            for a, b in zip(got[:4], ref[:4]):
                assert np.array_equal(a, b), (fmt, tau)


@pytest.mark.parametrize("mode", [1, 2])
def test_pure_modes_match_oracle(emu, orc, tiny, mode):
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    for rays in (tiny["free"], tiny["surf"]):
        got = emu.trace(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, 0.0, mode=mode)
        ref = orc.query(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, 0.0, mode=mode)
        m, c = orc.margin(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, 0.0, mode=mode)
        parity.check(got, ref, m, c, label="emu mode %d" % mode)


def test_limits_equal_pure_kernels(emu, tiny):
    """threshold 0 is DF-only and +inf is BVH-only, bit for bit."""
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    s = tiny["surf"].soa()
    for tau, mode in ((0.0, 2), (np.inf, 1)):
        a = emu.trace(sc.verts, sc.tris, grid, g4, s, 2.0, tau, mode=0)
        b = emu.trace(sc.verts, sc.tris, grid, g4, s, 2.0, tau, mode=mode)
        for x, y in zip(a[:4], b[:4]):
            assert np.array_equal(x, y)


def test_certified_steps_are_not_more(emu, tiny):
    """The certified bound only ever lengthens steps: no more fetches over all
    rays, and per ray at most a few more (an over-relaxed longer step that
    overshoots costs the ray one return to its verified point)."""
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    s = tiny["free"].soa()
    a = emu.trace(sc.verts, sc.tris, grid, g4, s, 2.0, 0.0, mode=2)
    b = emu.trace(sc.verts, sc.tris, grid, g4, s, 2.0, 0.0, mode=2, certified=True)
    fa, fb = a[4][:, 2], b[4][:, 2]
    assert fb.sum() <= fa.sum()
    assert np.mean(fb <= fa + 1) >= 0.98 and np.all(fb <= fa + 4)


def test_early_exit_takes_no_df_steps(emu, tiny):
    """First-hit in order: a ray caught by the triangle segment never touches
    the distance field."""
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    t, prim, u, v, cnt = emu.trace(sc.verts, sc.tris, grid, g4, tiny["surf"].soa(), 2.0, 2.0)
    assert (prim >= 0).sum() > 100
    assert np.all(cnt[prim >= 0, 2] == 0)
    assert np.all(cnt[prim == -2, 2] > 0)


def test_tmin_and_empty_interval(emu, orc, tiny):
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    r = tiny["free"].subset(slice(0, 512))
    tmin = np.linspace(0.0, 2.5, 512).astype(np.float32)  # tail has tmin > tmax
    for mode, tau in ((0, 1.0), (1, np.inf), (2, 0.0)):
        got = emu.trace(sc.verts, sc.tris, grid, g4, r.soa(), 2.0, tau, mode=mode, tmin=tmin)
        ref = orc.query(sc.verts, sc.tris, grid, g4, r.soa(), 2.0, tau, mode=mode, tmin=tmin)
        m, c = orc.margin(sc.verts, sc.tris, grid, g4, r.soa(), 2.0, tau, mode=mode, tmin=tmin)
        parity.check(got, ref, m, c, label="emu tmin mode %d" % mode)
        assert np.all(got[1][tmin > 2.0] == -1)


def test_empty_mesh_and_single_triangle(emu, orc):
    rng = np.random.default_rng(3)
    o = rng.uniform(0, 1, (64, 3)).astype(np.float32)
    d = rng.normal(size=(64, 3)).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    s = np.ascontiguousarray(np.concatenate([o.T, d.T]).astype(np.float32))
    got = emu.trace(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), None, None, s, 10.0, np.inf, mode=1)
    assert np.all(got[1] == -1)
    v = np.array([[0.2, 0.2, 0.5], [0.8, 0.3, 0.5], [0.4, 0.9, 0.5]], np.float32)
    got = emu.trace(v, [[0, 1, 2]], None, None, s, 10.0, np.inf, mode=1)
    ref = orc.query(v, [[0, 1, 2]], None, None, s, 10.0, np.inf, mode=1)
    m, c = orc.margin(v, np.array([[0, 1, 2]]), None, None, s, 10.0, np.inf, mode=1)
    parity.check(got, ref, m, c, label="single triangle")


def test_sdf_build_matches_oracle(emu, orc, tiny):
    """The build kernel's exact distance (FP64 -> FP32) against the oracle's:
    within one FP32 ulp (nodes lying on a surface: within 1e-15 of zero), same
    sign wherever |f| > 1e-6."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    got = emu.sdf(sc.verts, sc.tris, g4, 32)
    ref = tiny["grid"]
    ulp = np.maximum(np.spacing(np.abs(ref).astype(np.float32)), 1e-15)
    assert np.all(np.abs(got.astype(np.float64) - ref) <= ulp)
    far = np.abs(ref) > 1e-6
    assert np.array_equal(np.sign(got[far]), np.sign(ref[far]))


@pytest.mark.parametrize("taus", [(0.0, 0.0), (1.0, 1.0), (2.0, 4.0), (np.inf, np.inf)])
def test_shadow_query_matches_oracle(emu, orc, tiny, taus):
    from paper_2305_07253_amd import workloads as W
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    pts = W.surface_points(sc, 2048, 14)
    rays, tmax = W.shadow_rays(pts.p, pts.n, 15)
    s = rays.soa()
    ts, te = taus
    got = emu.trace(sc.verts, sc.tris, grid, g4, s, 10.0, ts, mode=3, tmax_ray=tmax, tau_end=te)
    ref = orc.query(sc.verts, sc.tris, grid, g4, s, 10.0, ts, mode=3, tmax_ray=tmax, tau_end=te)
    m, c = orc.margin(sc.verts, sc.tris, grid, g4, s, 10.0, ts, mode=3, tmax_ray=tmax, tau_end=te)
    h = np.float32(g4[3])
    t1 = np.minimum(np.float32(ts) * h, tmax).astype(np.float64)
    t2 = np.maximum((tmax - np.float32(te) * h).astype(np.float32).astype(np.float64), t1)
    st = parity.check_shadow(got, ref, m, orc, sc.verts, sc.tris, s, [(0.0, t1), (t2, tmax.astype(np.float64))],
                             label="emu shadow %s" % (taus,))
    assert st["occluded"] > 100


def test_df_gradient_matches_oracle(emu, orc, tiny):
    """The backward kernel's per-ray implicit derivatives against the oracle's
    FP64 ones (O-6) at the same hits."""
    grid, g4 = tiny["grid"], tiny["grid4"]
    s = tiny["free"].soa()
    t = orc.df_hit(grid, g4, s, 0.0, 2.0)
    m, c = orc.margin(None, np.zeros((0, 3)), grid, g4, s, 2.0, 0.0, mode=orc.MODE_DF)
    nodes, dt = emu.df_grad(grid, g4, s, t.astype(np.float32), 2.0)
    rn, rdt = orc.df_grad(grid, g4, s, t.astype(np.float32).astype(np.float64), 0.0, 2.0)
    ok = (m > 1e-5) & (c > 1e-2)
    # away from cell faces both sides pick the same cell
    p = tiny["free"].o.astype(np.float64) + np.where(np.isfinite(t), t, 0)[:, None] * tiny["free"].d.astype(np.float64)
    x = (p - np.float64(g4[0])) / np.float64(g4[3])
    ok &= np.abs(x - np.round(x)).min(axis=1) > 1e-4  # most free rays end on walls, which lie on node planes
    assert ok.sum() > 300
    assert np.array_equal(nodes[ok], rn[ok])
    assert np.all(np.abs(dt[ok] - rdt[ok]) <= 1e-4 * np.maximum(np.abs(rdt[ok]).max(axis=1, keepdims=True), 1.0))
    # rays whose hit is the start of their segment contribute nothing on either side
    assert np.array_equal(nodes[:, 0] == -1, rn[:, 0] == -1)


@pytest.mark.parametrize("n", [30, 33, 35])
def test_grid_sizes_with_partial_bricks(emu, orc, tiny, n):
    """Grids whose side is not a multiple of the 4-node brick (and, for I8, of
    the 8-node scale block): every format against the oracle."""
    from paper_2305_07253_amd import workloads as W
    sc = tiny["scene"]
    g4 = W.room_grid(n)
    grid = orc.sdf_grid(sc, g4, n)
    rays = tiny["free"].soa()[:, :1024]
    for fmt in (0, 1, 2, 3):
        deq = orc.quantize(grid, 1 if fmt == 3 else fmt)[0] if fmt else grid
        for tau in (0.0, 1.0):
            got = emu.trace(sc.verts, sc.tris, grid, g4, rays, 2.0, tau, fmt=fmt)
            ref = orc.query(sc.verts, sc.tris, deq, g4, rays, 2.0, tau)
            m, c = orc.margin(sc.verts, sc.tris, deq, g4, rays, 2.0, tau)
            parity.check(got, ref, m, c, label="emu n=%d fmt %d tau %s" % (n, fmt, tau))


@pytest.mark.parametrize("run", [1, 16, 64, 100, 128])
def test_block_order_is_a_permutation(emu, run):
    """The trace kernels' workgroup-to-block map: every block of a launch is
    processed exactly once, and within each full group of 8 * run blocks the
    workgroups of one die (b mod 8) take `run` consecutive blocks in turn."""
    for nb in (1, 7, 8, 9, 127, 128, 129, 8100, 24 * run + 5):
        order = runner.block_order(nb, run).astype(np.int64)
        assert np.array_equal(np.sort(order), np.arange(nb)), nb
        full = nb // (8 * run) * (8 * run)
        assert np.array_equal(order[full:], np.arange(full, nb))
        for x in range(8):
            runs = order[x:full:8].reshape(-1, run)
            assert np.all(np.diff(runs, axis=1) == 1) and np.all(runs[:, 0] % run == 0), (nb, x)


def test_block_order_eighths(emu):
    """run = nb / 8 (the backward kernel's choice): each die gets one
    contiguous eighth of the blocks, the remainder keeps its place."""
    for nb in (8, 64, 4099, 8100):
        order = runner.block_order(nb, nb // 8).astype(np.int64)
        for x in range(8):
            mine = order[x:nb // 8 * 8:8]
            assert np.array_equal(mine, np.arange(x * (nb // 8), (x + 1) * (nb // 8)))


def outlier_grid(tiny):
    """The tiny room's exact grid with one far corner sample, outside the room
    and off every ray's path, set to 1000: the grid's Lipschitz bound grows
    from sqrt(3) to about 4.7e4, so every certified sphere step shrinks to a
    tiny fraction of a cell."""
    g = tiny["grid"].copy()
    g.reshape(-1)[0] = 1000.0
    return g


@pytest.mark.parametrize("walk", [False, True])
@pytest.mark.parametrize("tau", [0.0, 1.0])
def test_inflated_bound_still_exact(emu, orc, tiny, tau, walk):
    """A grid whose bound is inflated by one extreme sample is traced exactly:
    the march takes cell steps where sphere steps would be short, so every ray
    ends within about one fetch per crossed cell.  walk: the build whose
    march falls back to the cell-by-cell walk after 4 iterations (the path a
    ray takes when its mixed march runs out of iterations) gives the same
    classes and the oracle's roots."""
    sc, g4 = tiny["scene"], tiny["grid4"]
    grid = outlier_grid(tiny)
    assert orc.lipschitz(grid, np.float64(g4[3])) > 1e4
    N = grid.shape[0]
    for rays in (tiny["free"], tiny["surf"]):
        got = emu.trace(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, tau, walk=walk)
        ref = orc.query(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, tau)
        m, c = orc.margin(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, tau)
        parity.check(got, ref, m, c, label="emu outlier tau=%s walk=%s" % (tau, walk))
        assert not np.isnan(got[0]).any()
        # at most the cells a segment crosses (3 (N - 2) + 1) plus one fetch
        # per sphere step and per return to the verified point
        assert got[4][:, 2].max() <= 3 * N


@pytest.mark.parametrize("certified", [False, True])
def test_walk_fallback_matches_march(emu, tiny, certified):
    """On the exact grid, the walk-only fall-back finds the same first roots
    as the full march (same classes, t within a few FP32 ulps of the root
    refinement), with more fetches."""
    sc, grid, g4 = tiny["scene"], tiny["grid"], tiny["grid4"]
    for rays in (tiny["free"], tiny["surf"]):
        a = emu.trace(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, 0.0, mode=2, certified=certified)
        b = emu.trace(sc.verts, sc.tris, grid, g4, rays.soa(), 2.0, 0.0, mode=2, certified=certified, walk=True)
        assert np.array_equal(a[1], b[1])
        hit = np.isfinite(a[0])
        assert np.array_equal(hit, np.isfinite(b[0]))
        assert np.all(np.abs(a[0][hit] - b[0][hit]) <= 1e-6 * np.maximum(a[0][hit], 0.05))
        assert b[4][:, 2].sum() > a[4][:, 2].sum()
