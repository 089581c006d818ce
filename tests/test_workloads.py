"""CPU: the seeded workload generators give the documented sizes, and the
oracle's sparse exact-sample grid agrees with its full grid."""
import numpy as np

from paper_2305_07253_amd import workloads as W


def test_scene_sizes():
    assert W.tiny_scene(1).n_tris == 1052
    assert W.gi_scene(2).n_tris == 188572
    assert W.precision_scene(3).n_tris == 1880236


def test_batch_specs_ranges_and_determinism():
    specs = W.batch_specs(4, 64)
    assert len(specs) == 64 and specs == W.batch_specs(4, 64)
    tris = np.array([s.n_objects * W.TRIS_PER_OBJECT + 12 for s in specs])
    rays = np.array([s.n_rays for s in specs])
    grids = np.array([s.n_grid for s in specs])
    assert tris.min() >= 700 and tris.max() <= 520000
    assert rays.min() >= 900 and rays.max() <= 2.2e6 and rays.sum() == 14658048
    assert np.all((grids >= 32) & (grids <= 128) & (grids % 8 == 0))
    assert all(s.width % 8 == 0 and s.height % 8 == 0 for s in specs)
    # larger scenes never get coarser grids
    order = np.argsort(tris)
    assert np.all(np.diff(grids[order]) >= 0)


def test_sparse_oracle_grid_matches_full(orc, tiny):
    sc, g4, full = tiny["scene"], tiny["grid4"], tiny["grid"]
    rays = tiny["surf"].subset(np.arange(0, 4096, 64))
    sparse, count = orc.sdf_grid_sparse(sc, g4, 32, rays.o, rays.d, 0.5)
    have = np.isfinite(sparse)
    assert count == have.sum() and 0 < count < 32 ** 3
    assert np.array_equal(sparse[have], full[have])
    # every node a query on these rays reads was sampled
    for tau in (0.0, 1.0):
        a = orc.query(sc.verts, sc.tris, sparse, g4, rays.soa(), 0.5, tau)
        b = orc.query(sc.verts, sc.tris, full, g4, rays.soa(), 0.5, tau)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
