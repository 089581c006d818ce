"""Writes tests/golden/oracle_tiny.txt: the oracle's results on a small seeded
case of the tiny room, so that a change to the oracle's arithmetic shows up as
a difference (tests/test_golden.py).  Calls nothing but `oracle` and the
seeded input generators.  Test infrastructure only.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2305_07253_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_tiny.txt")
TAUS = (0.0, 1.0, float("inf"))
TMAX = 2.0


def case():
    """The tiny room (seed 1), its exact 32^3 grid, 64 free-space and 64
    surface-origin rays, 64 grid nodes at a fixed stride."""
    scene = W.tiny_scene(1)
    g4 = W.room_grid(32)
    free = W.uniform_rays(scene, 64, 11)
    surf = W.offset_rays(W.surface_points(scene, 64, 12), 1e-5, 13)
    rays = np.concatenate([free.soa(), surf.soa()], axis=1)
    nodes = np.arange(0, 32 ** 3, 32 ** 3 // 64, dtype=np.int64)[:64]
    return scene, g4, rays, nodes


def compute():
    scene, g4, rays, nodes = case()
    grid = oracle.sdf_grid(scene, g4, 32)
    hits = {tau: oracle.query(scene.verts, scene.tris, grid, g4, rays, TMAX, tau) for tau in TAUS}
    dist = oracle.sdf_nodes(scene, g4, 32, nodes=nodes)
    return hits, nodes, dist


def main():
    hits, nodes, dist = compute()
    with open(OUT, "w") as f:
        f.write("# oracle results on the tiny room (seed 1), exact 32^3 grid, tmax %s;\n" % TMAX)
        f.write("# rays: 64 uniform free-space (seed 11) then 64 surface-origin (seeds 12, 13);\n")
        f.write("# written by tests/golden/make_golden.py from oracle/ only\n")
        for tau in TAUS:
            t, prim, u, v = hits[tau]
            for i in range(len(t)):
                f.write("hit %r %d %r %d %r %r\n" % (tau, i, float(t[i]), int(prim[i]), float(u[i]), float(v[i])))
        for k, d in zip(nodes, dist):
            f.write("node %d %r\n" % (int(k), float(d)))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
