"""FP64 CPU oracle for the combined ray query (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke check
and the CPU-baseline leg of the benchmark, never by the GPU library.  It shares
no code with the GPU path.

Every function takes the exact FP32 inputs the GPU sees and computes in FP64:
  closest_hit   O-1  closest triangle on [a,b] (Section 2, Eq. (1) on a sub-interval)
  sdf_nodes     O-5  exact signed distance to the mesh at grid nodes
  df_hit        O-3  first root of the trilinear interpolant on [a,b]
  sphere_trace  cross-check of df_hit by plain sphere tracing
  query         O-4  combined / triangles-only / DF-only query (Section 2, Eq. (2))
  margin        per-ray distance from a decision boundary, for parity filtering
  df_grad       O-6  d t_hit / d grid sample by implicit differentiation
  sdf_grid_on_paths  O-5 samples only on the cells each ray's walk reaches
                before its first root (for full-size parity tests)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_COMBINED, MODE_BVH, MODE_DF, MODE_SHADOW = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, FP64, no hand SIMD)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_double
        L.oracle_closest_hit.argtypes = [P, P, i64, P, i64, P, P, P, P, P, P]
        L.oracle_sdf_nodes.argtypes = [P, P, i64, P, P, P, i32, P, i32, P, i64, i32, P]
        L.oracle_df_hit.argtypes = [P, i32, P, P, i64, P, P, P]
        L.oracle_df_value.argtypes = [P, i32, P, f64, f64, f64]
        L.oracle_df_value.restype = f64
        L.oracle_lipschitz.argtypes = [P, i32, f64]
        L.oracle_lipschitz.restype = f64
        L.oracle_sphere_trace.argtypes = [P, i32, P, f64, P, i64, P, P, f64, i64, P, P]
        L.oracle_query.argtypes = [P, P, i64, P, i32, P, P, i64, P, P, f32, f32, f32, i32, P, P, P, P]
        L.oracle_margin.argtypes = [P, P, i64, P, i32, P, P, i64, P, P, f32, f32, f32, i32, P, P]
        L.oracle_df_grad.argtypes = [P, i32, P, P, i64, P, P, P, P, P]
        L.oracle_sdf_points.argtypes = [P, P, i64, P, P, P, i32, P, i64, P]
        L.oracle_df_values.argtypes = [P, i32, P, P, i64, P]
        L.oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


FMT_F32, FMT_F16, FMT_I8 = 0, 1, 2
SCALE_BLOCK = 8


def _block_exponents(g, nb):
    """e_B of every block of 8^3 cells: the smallest integer e >= -126 with
    max |f| over the block's nodes (cells [8b, 8b + 8) on each axis, so nodes
    [8b, 8b + 8]) <= 127 * 2^e.  Exact: the bound is compared in FP64."""
    n = g.shape[-1]
    a = np.abs(g).astype(np.float64)
    size = SCALE_BLOCK * nb + 1
    a = np.pad(a, [(0, max(size - n, 0))] * 3)
    for ax in range(3):
        sl = [np.take(a, np.arange(off, off + SCALE_BLOCK * nb, SCALE_BLOCK), axis=ax) for off in range(SCALE_BLOCK + 1)]
        a = np.maximum.reduce(sl)
    m = a[:nb, :nb, :nb]
    e = np.full(m.shape, -126, dtype=np.int64)
    pos = m > 0
    e[pos] = np.maximum(np.ceil(np.log2(m[pos] / 127.0)).astype(np.int64), -126)
    # correct the logarithm's rounding: smallest e with m <= 127 2^e
    low = pos & (np.ldexp(127.0, e) < m)
    e[low] += 1
    high = pos & (e > -126) & (np.ldexp(127.0, e - 1) >= m)
    e[high] -= 1
    assert np.all(m <= np.ldexp(127.0, e))
    return e


def quantize(grid, fmt):
    """Compact storage of an FP32 grid (n,n,n) [k,j,i], as the library defines
    it: returns (dequantized float32 grid, stored values, block scales or None).
      F16: round to nearest even half.
      I8:  blocks of 8^3 cells (cells [8b, 8b + 8) on each axis, nodes
           [8b, 8b + 8]: neighbouring blocks share a face of nodes), ceil((n - 1)
           / 8) per axis.  Block scale s_B = 2^e_B (_block_exponents).  A node
           lies in 1 to 8 blocks; with s_max and s_min the largest and smallest
           of their scales, its code is q = rint(f / s_max) (exact division,
           rounding half to even) clamped to +-floor(127 s_min / s_max), and its
           value q s_max (exact in FP32).  In every block holding the node the
           value is then an integer multiple k s_B with |k| <= 127, so a cell's
           8 corners are stored as int8 multiples of the one scale of the cell's
           block, and the interpolant stays continuous across block faces.
           Returns the node codes q (int8) and the block scales (nb, nb, nb)."""
    g = np.ascontiguousarray(grid, dtype=np.float32)
    if fmt == FMT_F32:
        return g, g, None
    if fmt == FMT_F16:
        h = g.astype(np.float16)
        return h.astype(np.float32), h, None
    n = g.shape[-1]
    nb = max((n - 1 + SCALE_BLOCK - 1) // SCALE_BLOCK, 1)
    e = _block_exponents(g, nb)
    # the blocks holding node i along one axis: (i - 1) // 8 (when i is on a
    # face) to i // 8, within [0, nb - 1]
    idx = np.arange(n)
    lo = np.clip((idx - 1) // SCALE_BLOCK, 0, nb - 1)
    hi = np.clip(idx // SCALE_BLOCK, 0, nb - 1)
    emax = np.full((n, n, n), -10 ** 6, dtype=np.int64)
    emin = np.full((n, n, n), 10 ** 6, dtype=np.int64)
    for bk in (lo, hi):
        for bj in (lo, hi):
            for bi in (lo, hi):
                sub = e[np.ix_(bk, bj, bi)]
                emax = np.maximum(emax, sub)
                emin = np.minimum(emin, sub)
    q = np.rint(np.ldexp(g, -emax).astype(np.float32))
    lim = np.floor(np.ldexp(127.0, emin - emax))
    q = np.clip(q, -lim, lim)
    deq = np.ldexp(q, emax).astype(np.float32)
    scales = np.ldexp(np.float32(1.0), e).astype(np.float32)
    return deq, q.astype(np.int8), scales


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(lib().oracle_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _rays(rays_soa):
    r = _f32(rays_soa)
    assert r.ndim == 2 and r.shape[0] == 6
    return r, r.shape[1]


def closest_hit(verts, tris, rays_soa, a, b):
    v, t = _f32(verts), _i32(tris)
    r, n = _rays(rays_soa)
    a = _f64(np.broadcast_to(a, (n,)))
    b = _f64(np.broadcast_to(b, (n,)))
    to, uo, vo = np.empty(n), np.empty(n), np.empty(n)
    po = np.empty(n, dtype=np.int32)
    lib().oracle_closest_hit(_p(v), _p(t), t.shape[0], _p(r), n, _p(a), _p(b), _p(to), _p(po), _p(uo), _p(vo))
    return to, po, uo, vo


def sdf_nodes(scene, grid4, n, nodes=None, prune=True):
    """Exact signed distance (FP64) at node indices i + n(j + n k); all nodes
    when `nodes` is None.  Returns FP64 values; the stored grid is their FP32
    rounding."""
    v, t = _f32(scene.verts), _i32(scene.tris)
    g4 = _f32(grid4)
    if nodes is None:
        nodes = np.arange(n ** 3, dtype=np.int64)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty(len(nodes))
    lib().oracle_sdf_nodes(_p(v), _p(t), t.shape[0], _p(_i32(scene.group_start)), _p(_i32(scene.group_count)),
                           _p(_i32(scene.group_kind)), len(scene.group_kind), _p(g4), n, _p(nodes), len(nodes),
                           1 if prune else 0, _p(out))
    return out


def sdf_grid(scene, grid4, n):
    """Full exact grid, FP32, shape (n,n,n) indexed [k,j,i] (x fastest)."""
    return sdf_nodes(scene, grid4, n).astype(np.float32).reshape(n, n, n)


def _grid(grid):
    """Grid samples as FP64 (FP32 grids are promoted exactly)."""
    return _f64(grid)


def sdf_points(scene, pts):
    """Exact signed distance (FP64) at arbitrary points (n,3)."""
    v, t = _f32(scene.verts), _i32(scene.tris)
    p = _f64(pts).reshape(-1, 3)
    out = np.empty(len(p))
    lib().oracle_sdf_points(_p(v), _p(t), t.shape[0], _p(_i32(scene.group_start)), _p(_i32(scene.group_count)),
                            _p(_i32(scene.group_kind)), len(scene.group_kind), _p(p), len(p), _p(out))
    return out


def df_hit(grid, grid4, rays_soa, a, b):
    g = _grid(grid)
    N = g.shape[-1]
    r, n = _rays(rays_soa)
    a = _f64(np.broadcast_to(a, (n,)))
    b = _f64(np.broadcast_to(b, (n,)))
    out = np.empty(n)
    lib().oracle_df_hit(_p(g), N, _p(_f32(grid4)), _p(r), n, _p(a), _p(b), _p(out))
    return out


def df_value(grid, grid4, p):
    g = _grid(grid)
    return lib().oracle_df_value(_p(g), g.shape[-1], _p(_f32(grid4)), float(p[0]), float(p[1]), float(p[2]))


def df_values(grid, grid4, pts):
    """Interpolant at points (n,3)."""
    g = _grid(grid)
    p = _f64(pts).reshape(-1, 3)
    out = np.empty(len(p))
    lib().oracle_df_values(_p(g), g.shape[-1], _p(_f32(grid4)), _p(p), len(p), _p(out))
    return out


def lipschitz(grid, h):
    g = _grid(grid)
    return lib().oracle_lipschitz(_p(g), g.shape[-1], float(h))


def sphere_trace(grid, grid4, L, rays_soa, a, b, eps, max_steps=1_000_000):
    g = _grid(grid)
    r, n = _rays(rays_soa)
    a = _f64(np.broadcast_to(a, (n,)))
    b = _f64(np.broadcast_to(b, (n,)))
    out = np.empty(n)
    st = np.empty(n, dtype=np.int32)
    lib().oracle_sphere_trace(_p(g), g.shape[-1], _p(_f32(grid4)), float(L), _p(r), n, _p(a), _p(b),
                              float(eps), int(max_steps), _p(out), _p(st))
    return out, st


def query(verts, tris, grid, grid4, rays_soa, tmax, tau, mode=MODE_COMBINED, tmin=None, tmax_ray=None,
          tau_end=0.0):
    """O-4 (mode 0), triangles only (1), DF only (2), shadow any-hit (3).
    Returns (t, prim, u, v); prim -1 miss, -2 distance-field hit."""
    v, t = _f32(verts), _i32(tris)
    g = None if grid is None else _grid(grid)
    N = 0 if g is None else g.shape[-1]
    r, n = _rays(rays_soa)
    tm = None if tmin is None else _f32(tmin)
    tx = None if tmax_ray is None else _f32(tmax_ray)
    to, uo, vo = np.empty(n), np.empty(n), np.empty(n)
    po = np.empty(n, dtype=np.int32)
    lib().oracle_query(_p(v), _p(t), t.shape[0], _p(g), N, None if grid4 is None else _p(_f32(grid4)),
                       _p(r), n, _p(tm), _p(tx), np.float32(tmax), np.float32(tau), np.float32(tau_end), mode,
                       _p(to), _p(po), _p(uo), _p(vo))
    return to, po, uo, vo


def margin(verts, tris, grid, grid4, rays_soa, tmax, tau, mode=MODE_COMBINED, tmin=None, tmax_ray=None,
           tau_end=0.0):
    """Per-ray (margin, conditioning) of query(): see oracle.c."""
    v, t = _f32(verts), _i32(tris)
    g = None if grid is None else _grid(grid)
    N = 0 if g is None else g.shape[-1]
    r, n = _rays(rays_soa)
    tm = None if tmin is None else _f32(tmin)
    tx = None if tmax_ray is None else _f32(tmax_ray)
    mo, co = np.empty(n), np.empty(n)
    lib().oracle_margin(_p(v), _p(t), t.shape[0], _p(g), N, None if grid4 is None else _p(_f32(grid4)),
                        _p(r), n, _p(tm), _p(tx), np.float32(tmax), np.float32(tau), np.float32(tau_end), mode,
                        _p(mo), _p(co))
    return mo, co


def df_grad(grid, grid4, rays_soa, t_hit, a=0.0, b=np.inf):
    """O-6: per ray, 8 node indices and d t_hit / d sample (node -1: none) for
    DF hits on the segments [a,b]."""
    g = _grid(grid)
    r, n = _rays(rays_soa)
    th = _f64(t_hit)
    a = _f64(np.broadcast_to(a, (n,)))
    b = _f64(np.broadcast_to(b, (n,)))
    nodes = np.empty((n, 8), dtype=np.int64)
    dt = np.empty((n, 8))
    lib().oracle_df_grad(_p(g), g.shape[-1], _p(_f32(grid4)), _p(r), n, _p(a), _p(b), _p(th), _p(nodes), _p(dt))
    return nodes, dt


def sdf_grid_sparse(scene, grid4, n, rays_o, rays_d, tmax, progress=None):
    """Exact samples (sdf_nodes) at every node of the cells that segments
    [0, tmax] of the given rays can cross, NaN elsewhere, so that a query
    reading any other node shows it.  The cells are found by sampling each
    segment every h/16 and adding all 26 neighbours of every cell met.
    Returns (grid (n,n,n) float32, number of nodes computed)."""
    h = np.float64(grid4[3])
    lo = np.asarray(grid4[:3], np.float64)
    ts = np.arange(0.0, tmax + h / 16, h / 16)
    o, d = np.asarray(rays_o, np.float64), np.asarray(rays_d, np.float64)
    cells = []
    for c0 in range(0, len(o), 256):
        if progress:
            progress("oracle cells: rays %d / %d" % (c0, len(o)))
        p = o[c0:c0 + 256, None, :] + ts[None, :, None] * d[c0:c0 + 256, None, :]
        c = np.floor((p - lo) / h).astype(np.int64).reshape(-1, 3)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    cc = np.clip(c + np.array([dx, dy, dz]), 0, n - 2)
                    cells.append(np.unique(cc[:, 0] + n * (cc[:, 1] + n * cc[:, 2])))
    cells = np.unique(np.concatenate(cells))
    ci, cj, ck = cells % n, (cells // n) % n, cells // (n * n)
    nodes = np.unique(np.concatenate([(ci + dx) + n * ((cj + dy) + n * (ck + dz))
                                      for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]))
    grid = np.full(n ** 3, np.nan, dtype=np.float32)
    step = 1 << 18
    for c0 in range(0, len(nodes), step):
        if progress:
            progress("oracle samples: %d / %d nodes" % (c0, len(nodes)))
        grid[nodes[c0:c0 + step]] = sdf_nodes(scene, grid4, n, nodes=nodes[c0:c0 + step]).astype(np.float32)
    return grid.reshape(n, n, n), len(nodes)


def _segment_cells(o, d, a, b, grid4, n, chunk=256):
    """(ray index, cell) pairs covering every cell a segment o + t d, t in
    [a_i, b_i], can cross: the points t = a_i + k h/8 <= b_i and, for each
    point, the neighbouring cells across every face within h/8 of it.  (A
    cell the segment enters after a point and before the next, or before b_i,
    is entered within h/8 of that point, so it differs from the point's cell
    only along axes whose face lies within h/8 of the point.)  The points of
    [a, b'] are those of [a, b] up to b', so a shorter segment's cells are a
    subset.  Cells are flat indices i + n (j + n k), clamped to [0, n - 2]."""
    h = np.float64(grid4[3])
    lo = np.asarray(grid4[:3], np.float64)
    step, band = h / 8, 1.0 / 8 + 1e-9
    o, d = np.asarray(o, np.float64), np.asarray(d, np.float64)
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    keys = []
    for c0 in range(0, len(o), chunk):
        sl = slice(c0, c0 + chunk)
        aa, bb = a[sl], np.maximum(b[sl], a[sl])
        if not len(aa):
            continue
        cnt = np.floor((bb - aa) / step).astype(np.int64) + 1  # points a + k step, k < cnt
        m = int(cnt.max())
        k = np.arange(m)[None, :]
        keep = (k < cnt[:, None]).reshape(-1)
        ts = aa[:, None] + k * step
        x = ((o[sl, None, :] + ts[:, :, None] * d[sl, None, :] - lo) / h).reshape(-1, 3)[keep]
        ray = np.repeat(np.arange(c0, c0 + len(aa), dtype=np.int64), m)[keep]
        c = np.floor(x)
        f = x - c
        c = c.astype(np.int64)
        for k in range(3):
            lo_k, hi_k = f[:, k] < band, f[:, k] > 1.0 - band
            cl, ch = c[lo_k].copy(), c[hi_k].copy()
            cl[:, k] -= 1
            ch[:, k] += 1
            c = np.concatenate([c, cl, ch])
            f = np.concatenate([f, f[lo_k], f[hi_k]])
            ray = np.concatenate([ray, ray[lo_k], ray[hi_k]])
        c = np.clip(c, 0, n - 2)
        keys.append(np.unique(ray * (n ** 3) + c[:, 0] + n * (c[:, 1] + n * c[:, 2])))
    if not keys:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    pair = np.unique(np.concatenate(keys))
    return pair // (n ** 3), pair % (n ** 3)


def _cell_nodes(cells, n):
    ci, cj, ck = cells % n, (cells // n) % n, cells // (n * n)
    return np.stack([(ci + dx) + n * ((cj + dy) + n * (ck + dz))
                     for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], axis=1)


def sdf_grid_on_paths(scene, grid4, n, rays_soa, a, b, progress=None):
    """Exact samples (sdf_nodes) at the nodes of every cell that each ray's
    distance-field segment [a_i, b_i] crosses up to its first root, NaN
    elsewhere, so that any read of another node shows.  Rays are extended
    from a short reach, doubling it, until the first root that df_hit finds
    on the sampled nodes lies beyond no unsampled cell (a root inside an
    unsampled cell cannot be skipped unnoticed: the walk up to a later root
    would cross that cell).  Returns (grid (n,n,n) float32, nodes computed)."""
    r = np.ascontiguousarray(rays_soa, np.float32)
    nr = r.shape[1]
    o, d = r[:3].T.astype(np.float64), r[3:].T.astype(np.float64)
    a = np.broadcast_to(np.asarray(a, np.float64), (nr,)).copy()
    b = np.broadcast_to(np.asarray(b, np.float64), (nr,)).copy()
    h = np.float64(grid4[3])
    grid = np.full(n ** 3, np.nan, dtype=np.float32)
    reach = np.full(nr, 8 * h)
    pending = np.arange(nr)
    computed = 0
    while len(pending):
        p = pending
        ri, cells = _segment_cells(o[p], d[p], a[p], np.minimum(a[p] + reach[p], b[p]), grid4, n)
        nodes = np.unique(_cell_nodes(cells, n).reshape(-1))
        new = nodes[np.isnan(grid[nodes])]
        for c0 in range(0, len(new), 1 << 18):
            grid[new[c0:c0 + (1 << 18)]] = sdf_nodes(scene, grid4, n, nodes=new[c0:c0 + (1 << 18)]).astype(np.float32)
        computed += len(new)
        t = df_hit(grid.reshape(n, n, n), grid4, r[:, p], a[p], b[p])
        tend = np.minimum(np.where(np.isfinite(t), t, b[p]), b[p])
        ri, cells = _segment_cells(o[p], d[p], a[p], tend, grid4, n)
        bad = np.isnan(grid[_cell_nodes(cells, n)]).any(axis=1)
        ok = np.ones(len(p), bool)
        ok[ri[bad]] = False
        if progress:
            progress("oracle samples: %d nodes, %d of %d rays pending" % (computed, (~ok).sum(), nr))
        # a segment sampled to its end covers every cell its walk can visit
        assert np.all(a[p[~ok]] + reach[p[~ok]] < b[p[~ok]]), "a fully sampled segment read an unsampled cell"
        reach[p[~ok]] *= 2
        pending = p[~ok]
    return grid.reshape(n, n, n), computed
