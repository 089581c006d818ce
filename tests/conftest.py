"""Shared fixtures.  Tests marked `gpu` need an MI355X; everything else runs on
the CPU (oracle pins, host logic, the C-ABI symbol table)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def tiny(orc):
    """Tiny room: 1,052 triangles, exact 32^3 grid (h = 1/27), 4,096 rays from
    free space with uniform directions, and 4,096 surface-origin diffuse rays."""
    from paper_2305_07253_amd import workloads as W
    scene = W.tiny_scene(1)
    g4 = W.room_grid(32)
    grid = orc.sdf_grid(scene, g4, 32)
    free = W.uniform_rays(scene, 4096, 11)
    surf = W.offset_rays(W.surface_points(scene, 4096, 12), 1e-5, 13)
    return dict(scene=scene, grid4=g4, grid=grid, N=32, free=free, surf=surf, tmax=2.0)


@pytest.fixture(scope="session")
def gi_exact(orc):
    """GI-shaped scene (188,572 triangles) with the oracle's exact 128^3 grid
    (computed once per session; the GPU tests of several modules use it)."""
    from paper_2305_07253_amd import workloads as W
    scene = W.gi_scene(2)
    g4 = W.room_grid(128)
    print("building the oracle's exact 128^3 grid", flush=True)
    return dict(scene=scene, g4=g4, grid=orc.sdf_grid(scene, g4, 128))
