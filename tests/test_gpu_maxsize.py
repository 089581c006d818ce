"""GPU parity at the largest grid the API accepts (n = 1024), where every
bricked store passes 2^32 bytes and the I8 one 2^32 elements (F16 at this size
is kept in two-cell bricks): every address above that must be formed in 64
bits.

The field is the exact FP32 signed distance to a sphere (centre 0.5, radius
0.3) on the nodes i h, h = 2^-10.  Rays start near the sphere's top (node
k ~ 819, far into the upper half of every store) and are short enough that each
segment stays inside a 160^3-node window aligned to the 8^3 scale blocks; the
oracle gets that window of the same FP32 samples (dequantized by its own rule
for F16 and I8, from a window one scale block larger below and one node
larger above, so every window node sees all the blocks holding it), so its
first root equals the one on the full grid.
"""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

N = 1024
H = 2.0 ** -10
CENTRE, RADIUS = 0.5, 0.3
TMAX = 0.045
WIN = (744, 432, 432)  # window start, nodes (k, j, i); multiples of 8
WSIZE = 160


@pytest.fixture(scope="module")
def hyb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2305_07253_amd as hyb
    hyb.lib()
    return hyb


@pytest.fixture(scope="module")
def sphere_grid():
    print("building the 1024^3 sphere field", flush=True)
    x = np.arange(N, dtype=np.float64) * H - CENTRE
    g = np.empty((N, N, N), dtype=np.float32)
    yy = (x * x)[:, None] + (x * x)[None, :]
    for k in range(N):
        g[k] = (np.sqrt(yy + x[k] * x[k]) - RADIUS).astype(np.float32)
    return g


@pytest.fixture(scope="module")
def rays():
    rng = np.random.default_rng(23)
    n = 4096
    # origins 4-20 voxels above the surface within 4 degrees of the top
    th = np.deg2rad(4.0) * np.sqrt(rng.uniform(0, 1, n))
    ph = rng.uniform(0, 2 * np.pi, n)
    u = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    o = CENTRE + (RADIUS + rng.uniform(4, 20, n)[:, None] * H) * u
    # towards the centre, spread so that some rays graze or miss
    d = -u + rng.normal(0, 1.0, (n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    soa = np.ascontiguousarray(np.concatenate([o.T, d.T]), dtype=np.float32)
    # every segment inside the window, two cells from its faces
    lo = np.array(WIN[::-1], dtype=np.float64) * H + 2 * H
    hi = (np.array(WIN[::-1], dtype=np.float64) + WSIZE - 1) * H - 2 * H
    for t in (0.0, TMAX):
        p = soa[:3].T.astype(np.float64) + t * soa[3:].T.astype(np.float64)
        assert np.all((p >= lo) & (p <= hi))
    return soa


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_max_grid_size_parity(hyb, orc, sphere_grid, rays, fmt):
    import torch
    print("format", fmt, flush=True)
    values = torch.from_numpy(sphere_grid.reshape(-1)).cuda()
    sdf = hyb.sdf_from_grid(values, np.array([0.0, 0.0, 0.0, H], dtype=np.float32), fmt=fmt)
    del values
    got = [x.cpu().numpy() for x in hyb.trace_df(sdf, torch.from_numpy(rays).cuda(), TMAX)]
    del sdf
    torch.cuda.empty_cache()
    k0, j0, i0 = WIN
    if fmt:
        # an I8 node's value depends on the scale blocks holding it: quantize
        # the window grown by one block below and one node above (whole blocks
        # around every window node, aligned as in the full grid), then crop
        big = np.ascontiguousarray(sphere_grid[k0 - 8:k0 + WSIZE + 1, j0 - 8:j0 + WSIZE + 1, i0 - 8:i0 + WSIZE + 1])
        win = np.ascontiguousarray(orc.quantize(big, fmt)[0][8:8 + WSIZE, 8:8 + WSIZE, 8:8 + WSIZE])
    else:
        win = np.ascontiguousarray(sphere_grid[k0:k0 + WSIZE, j0:j0 + WSIZE, i0:i0 + WSIZE])
    g4 = np.array([i0 * H, j0 * H, k0 * H, H], dtype=np.float32)
    ref = orc.query(None, np.zeros((0, 3)), win, g4, rays, TMAX, 0.0, mode=orc.MODE_DF)
    m, c = orc.margin(None, np.zeros((0, 3)), win, g4, rays, TMAX, 0.0, mode=orc.MODE_DF)
    hits = (ref[1] == -2).mean()
    assert 0.5 < hits < 0.9, hits
    st = parity.check(got, ref, m, c, label="n=1024 fmt %d" % fmt)
    print("n=1024 fmt", fmt, "hits %.3f" % hits, st)


def test_max_grid_size_sdf_build(hyb, orc, tiny):
    """hyb_build_sdf at n = 1024 (FP32, 4.3e9 store slots): 4,096 random nodes,
    the first and the last 256 included, within one FP32 ulp of the oracle's
    exact signed distances, signs equal away from the surface."""
    import torch
    from paper_2305_07253_amd import workloads as W
    sc = tiny["scene"]
    g4 = W.room_grid(N)
    print("building the 1024^3 grid of the tiny room", flush=True)
    sdf = hyb.build_sdf(hyb.build_bvh(sc.verts, sc.tris), N, g4)
    rng = np.random.default_rng(29)
    idx = np.concatenate([np.arange(256), N ** 3 - 256 + np.arange(256), rng.integers(0, N ** 3, 3584)])
    got = hyb.sdf_read(sdf).reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    del sdf
    torch.cuda.empty_cache()
    ref = orc.sdf_nodes(sc, g4, N, nodes=idx)
    ulp = np.maximum(np.spacing(np.abs(ref).astype(np.float32)), 1e-15)
    bad = np.abs(got.astype(np.float64) - ref) > ulp
    assert bad.sum() == 0, (bad.sum(), idx[bad][:5], got[bad][:5], ref[bad][:5])
    far = np.abs(ref) > 1e-6
    assert np.array_equal(np.sign(got[far]), np.sign(ref[far]))
