"""Seeded synthetic scenes and rays for the combined ray query.

This module only *creates inputs*: triangle meshes of a room filled with boxes
and icospheres, ray origins and directions, and the screen-space G-buffer that
the paper's experiments start from (Section 3: one ray per pixel, its origin
taken from an initial rasterization of the scene, directions randomised within
screen tiles).  It holds none of the ray-query arithmetic: no ray/triangle
test, no BVH, no distance field and no marching.  The G-buffer comes from a
z-buffer rasterizer (edge functions plus perspective-correct depth), which is
how the paper obtains its ray origins.

Both the GPU library and the CPU oracle consume what this module returns; it
imports neither of them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------
# scene description
# ----------------------------------------------------------------------------

KIND_ROOM = 0  # the enclosing room: normals point inwards, exterior is solid
KIND_BOX = 1
KIND_ICO = 2

CAMERA_EYE = np.array([0.5, 0.45, 0.05])
CAMERA_TARGET = np.array([0.5, 0.5, 1.0])
CAMERA_UP = np.array([0.0, 1.0, 0.0])
CAMERA_VFOV_DEG = 60.0
CAMERA_CLEARANCE = 0.05


@dataclasses.dataclass
class Scene:
    verts: np.ndarray        # (V,3) float32
    tris: np.ndarray         # (T,3) int32, counter-clockwise seen from free space
    group_start: np.ndarray  # (G,) int32: first triangle of each object
    group_count: np.ndarray  # (G,) int32
    group_kind: np.ndarray   # (G,) int32: KIND_ROOM / KIND_BOX / KIND_ICO
    centers: np.ndarray      # (G,3) float64 object centres
    rots: np.ndarray         # (G,3,3) float64 local->world rotations
    extents: np.ndarray      # (G,3) float64 box half-extents, or (r,r,r) for icospheres
    seed: int

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    def triangle_soup(self) -> np.ndarray:
        """(T,3,3) float32 vertex positions per triangle."""
        return self.verts[self.tris]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _box_mesh(n: int):
    """Closed cube [-1,1]^3 split into n x n quads per face, shared vertices,
    outward counter-clockwise winding."""
    keys = {}
    verts = []
    tris = []

    def vid(i, j, k):
        key = (i, j, k)
        if key not in keys:
            keys[key] = len(verts)
            verts.append((-1.0 + 2.0 * i / n, -1.0 + 2.0 * j / n, -1.0 + 2.0 * k / n))
        return keys[key]

    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in (0, n):
            for u in range(n):
                for w in range(n):
                    quad = []
                    for du, dw in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        idx = [0, 0, 0]
                        idx[a] = side
                        idx[b] = u + du
                        idx[c] = w + dw
                        quad.append(vid(*idx))
                    if side == 0:  # e_b x e_c = +e_a, so reverse on the negative face
                        quad = quad[::-1]
                    tris.append((quad[0], quad[1], quad[2]))
                    tris.append((quad[0], quad[2], quad[3]))
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int64)


def _icosphere_mesh(splits: int):
    """Unit icosphere: icosahedron with `splits` 4:1 midpoint subdivisions."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0),
         (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(splits):
        mid = {}

        def midpoint(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                p = verts[i] + verts[j]
                verts.append(p / np.linalg.norm(p))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for (a, b, c) in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts)
    F = np.array(faces, dtype=np.int64)
    # orient outward: the face normal must agree with the centroid direction
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    cen = V[F].mean(axis=1)
    flip = np.einsum("ij,ij->i", n, cen) < 0
    F[flip] = F[flip][:, ::-1]
    return V, F


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a uniform unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.random(3)
    x = math.sqrt(1 - u1) * math.sin(2 * math.pi * u2)
    y = math.sqrt(1 - u1) * math.cos(2 * math.pi * u2)
    z = math.sqrt(u1) * math.sin(2 * math.pi * u3)
    w = math.sqrt(u1) * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def make_scene(seed: int, n_objects: int, s_min: float, s_max: float,
               box_subdiv: int = 6, ico_splits: int = 2,
               kinds: np.ndarray | None = None) -> Scene:
    """Room (unit cube, 12 inward-facing triangles) plus `n_objects` boxes and
    icospheres: centres uniform in [0.05,0.95]^3, size log-uniform in
    [s_min,s_max], box half-extents s*(a_x,a_y,a_z) with a_i ~ U[0.2,1],
    uniform random rotation; overlaps allowed, none within 0.05 of the camera.
    `kinds` fixes the object types; otherwise each is a fair coin."""
    rng = _rng(seed)
    box_v, box_f = _box_mesh(box_subdiv)
    ico_v, ico_f = _icosphere_mesh(ico_splits)
    room_v, room_f = _box_mesh(1)

    verts = [0.5 + 0.5 * room_v]
    tris = [room_f[:, ::-1].copy()]  # inward-facing
    group_start, group_count, group_kind = [0], [len(room_f)], [KIND_ROOM]
    centers, rots, extents = [np.full(3, 0.5)], [np.eye(3)], [np.full(3, 0.5)]
    nv, nt = len(room_v), len(room_f)

    if kinds is None:
        kinds = np.where(rng.random(n_objects) < 0.5, KIND_BOX, KIND_ICO)
    for i in range(n_objects):
        kind = int(kinds[i])
        while True:
            c = 0.05 + 0.9 * rng.random(3)
            s = math.exp(rng.uniform(math.log(s_min), math.log(s_max)))
            if kind == KIND_BOX:
                ext = s * rng.uniform(0.2, 1.0, 3)
                radius = float(np.linalg.norm(ext))
            else:
                ext = np.full(3, s)
                radius = s
            R = _random_rotation(rng)
            if np.linalg.norm(c - CAMERA_EYE) >= CAMERA_CLEARANCE + radius:
                break
        if kind == KIND_BOX:
            lv, lf = box_v * ext, box_f
        else:
            lv, lf = ico_v * s, ico_f
        verts.append(c + lv @ R.T)
        tris.append(lf + nv)
        group_start.append(nt)
        group_count.append(len(lf))
        group_kind.append(kind)
        centers.append(c)
        rots.append(R)
        extents.append(ext)
        nv += len(lv)
        nt += len(lf)

    return Scene(
        verts=np.concatenate(verts).astype(np.float32),
        tris=np.concatenate(tris).astype(np.int32),
        group_start=np.array(group_start, dtype=np.int32),
        group_count=np.array(group_count, dtype=np.int32),
        group_kind=np.array(group_kind, dtype=np.int32),
        centers=np.array(centers), rots=np.array(rots), extents=np.array(extents),
        seed=seed,
    )


def tiny_scene(seed: int = 1) -> Scene:
    """Room + 20 boxes (12 triangles) + 10 icospheres (80 triangles): 1,052
    triangles in the unit cube."""
    kinds = np.array([KIND_BOX] * 20 + [KIND_ICO] * 10)
    return make_scene(seed, 30, 0.03, 0.12, box_subdiv=1, ico_splits=1, kinds=kinds)


def gi_scene(seed: int = 2) -> Scene:
    """Room + 500 objects (432-triangle boxes / 320-triangle icospheres),
    about 188k triangles."""
    return make_scene(seed, 500, 0.006, 0.06, box_subdiv=6, ico_splits=2)


def precision_scene(seed: int = 3) -> Scene:
    """Room + 5,000 objects, about 1.88M triangles."""
    return make_scene(seed, 5000, 0.003, 0.03, box_subdiv=6, ico_splits=2)


# ----------------------------------------------------------------------------
# grid placement (configuration, shared by both sides so they sample the same nodes)
# ----------------------------------------------------------------------------

def default_grid(verts: np.ndarray, n: int) -> np.ndarray:
    """Node-centred n^3 grid over the scene AABB padded by 2 voxels per side:
    returns float32 [lo_x, lo_y, lo_z, h] with h = extent/(n-5)."""
    v = verts.astype(np.float64)
    lo, hi = v.min(axis=0), v.max(axis=0)
    h = np.float32((hi - lo).max() / (n - 5))
    lo32 = (lo - 2.0 * np.float64(h)).astype(np.float32)
    return np.array([lo32[0], lo32[1], lo32[2], h], dtype=np.float32)


def room_grid(n: int) -> np.ndarray:
    """Node-centred n^3 grid over the unit room padded by 2 voxels per side:
    float32 [lo, lo, lo, h] with h = 1/(n-5) (1/27 at 32^3, 1/123 at 128^3)."""
    h = np.float32(1.0 / (n - 5))
    lo = np.float32(-2.0 * np.float64(h))
    return np.array([lo, lo, lo, h], dtype=np.float32)


# ----------------------------------------------------------------------------
# rays
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Rays:
    o: np.ndarray  # (n,3) float32
    d: np.ndarray  # (n,3) float32, unit length in float32 arithmetic

    @property
    def n(self) -> int:
        return int(self.o.shape[0])

    def soa(self) -> np.ndarray:
        """(6,n) float32: ox,oy,oz,dx,dy,dz rows."""
        return np.ascontiguousarray(np.concatenate([self.o.T, self.d.T]).astype(np.float32))

    def subset(self, idx) -> "Rays":
        return Rays(self.o[idx].copy(), self.d[idx].copy())


def _normalize32(d: np.ndarray) -> np.ndarray:
    d = d.astype(np.float32)
    nrm = np.sqrt((d * d).sum(axis=1, dtype=np.float32)).astype(np.float32)
    return (d / nrm[:, None]).astype(np.float32)


def _inside_object_bounds(scene: Scene, p: np.ndarray, skip_group=None) -> np.ndarray:
    """Conservative solid test used only for rejection sampling: inside any
    box (exact, local frame) or any icosphere's circumscribed sphere."""
    inside = np.zeros(len(p), dtype=bool)
    for g in range(1, len(scene.group_kind)):
        loc = (p - scene.centers[g]) @ scene.rots[g]
        if scene.group_kind[g] == KIND_BOX:
            hit = np.all(np.abs(loc) <= scene.extents[g] * (1 + 1e-6), axis=1)
        else:
            hit = (loc * loc).sum(axis=1) <= (scene.extents[g][0] * (1 + 1e-6)) ** 2
        if skip_group is not None:
            hit &= skip_group != g
        inside |= hit
    return inside


def uniform_rays(scene: Scene, n: int, seed: int) -> Rays:
    """Origins uniform in the room, rejected when inside an object's bounding
    shape; directions uniform on the sphere."""
    rng = _rng(seed)
    out = np.zeros((0, 3))
    while len(out) < n:
        p = rng.random((2 * n, 3))
        p = p[~_inside_object_bounds(scene, p)]
        out = np.concatenate([out, p])
    o = out[:n]
    d = rng.standard_normal((n, 3))
    return Rays(o.astype(np.float32), _normalize32(d))


def cosine_hemisphere(n_world: np.ndarray, u1: np.ndarray, u2: np.ndarray) -> np.ndarray:
    """Cosine-weighted directions about unit normals (Malley's method, with the
    branchless orthonormal basis of Duff et al. 2017)."""
    r = np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    lx, ly, lz = r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))
    nx, ny, nz = n_world[:, 0], n_world[:, 1], n_world[:, 2]
    sign = np.where(nz >= 0, 1.0, -1.0)
    a = -1.0 / (sign + nz)
    b = nx * ny * a
    t = np.stack([1.0 + sign * nx * nx * a, sign * b, -sign * nx], axis=1)
    bt = np.stack([b, sign + ny * ny * a, -ny], axis=1)
    return lx[:, None] * t + ly[:, None] * bt + lz[:, None] * n_world


def _tri_normals(scene: Scene) -> np.ndarray:
    v = scene.verts.astype(np.float64)[scene.tris]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


@dataclasses.dataclass
class SurfacePoints:
    p: np.ndarray     # (n,3) float64 point on a triangle
    n: np.ndarray     # (n,3) float64 unit normal pointing into free space
    tri: np.ndarray   # (n,) int32 source triangle


def surface_points(scene: Scene, n: int, seed: int) -> SurfacePoints:
    """Area-uniform points on the mesh, outside other objects' bounds and the
    room's exterior."""
    rng = _rng(seed)
    v = scene.verts.astype(np.float64)[scene.tris]
    area = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    cdf = np.cumsum(area)
    cdf /= cdf[-1]
    group_of_tri = np.searchsorted(scene.group_start, np.arange(scene.n_tris), side="right") - 1
    normals = _tri_normals(scene)
    ps, ns, ts = [], [], []
    got = 0
    while got < n:
        m = 2 * n
        tri = np.minimum(np.searchsorted(cdf, rng.random(m)), scene.n_tris - 1)
        s1 = np.sqrt(rng.random(m))
        s2 = rng.random(m)
        b0, b1, b2 = 1 - s1, s1 * (1 - s2), s1 * s2
        p = b0[:, None] * v[tri, 0] + b1[:, None] * v[tri, 1] + b2[:, None] * v[tri, 2]
        g = group_of_tri[tri]
        ok = ~_inside_object_bounds(scene, p, skip_group=g)
        ok &= (g == 0) | np.all((p > 0) & (p < 1), axis=1)
        ps.append(p[ok]); ns.append(normals[tri[ok]]); ts.append(tri[ok])
        got += int(ok.sum())
    return SurfacePoints(np.concatenate(ps)[:n], np.concatenate(ns)[:n],
                         np.concatenate(ts)[:n].astype(np.int32))


def offset_rays(pts: SurfacePoints, eps: float, seed: int) -> Rays:
    """Diffuse rays leaving surface points: origin p + eps*n, cosine directions."""
    rng = _rng(seed)
    u = rng.random((len(pts.p), 2))
    d = cosine_hemisphere(pts.n, u[:, 0], u[:, 1])
    o = pts.p + eps * pts.n
    return Rays(o.astype(np.float32), _normalize32(d))


# ----------------------------------------------------------------------------
# G-buffer by rasterization (pinhole camera, z-buffer)
# ----------------------------------------------------------------------------

def _camera_basis():
    fwd = CAMERA_TARGET - CAMERA_EYE
    fwd = fwd / np.linalg.norm(fwd)
    right = np.cross(fwd, CAMERA_UP)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return right, up, fwd


def _clip_near(cam: np.ndarray, z_near: float):
    """Clip one triangle (3,3) in camera space against z >= z_near; returns a
    list of triangles."""
    poly = [cam[0], cam[1], cam[2]]
    out = []
    for i in range(3):
        a, b = poly[i], poly[(i + 1) % 3]
        ina, inb = a[2] >= z_near, b[2] >= z_near
        if ina:
            out.append(a)
        if ina != inb:
            s = (z_near - a[2]) / (b[2] - a[2])
            out.append(a + s * (b - a))
    return [np.array([out[0], out[k], out[k + 1]]) for k in range(1, len(out) - 1)]


def rasterize(scene: Scene, width: int, height: int):
    """Z-buffer rasterization of every triangle at pixel centres.

    Returns (tri_id (H*W,) int32 with -1 where nothing covers the pixel,
    depth (H*W,) float64 camera-space depth) in row-major pixel order."""
    right, up, fwd = _camera_basis()
    f = (height / 2.0) / math.tan(math.radians(CAMERA_VFOV_DEG) / 2.0)
    z_near = 1e-4
    v = scene.verts.astype(np.float64)[scene.tris] - CAMERA_EYE
    cam = np.stack([v @ right, v @ up, v @ fwd], axis=-1)  # (T,3,3)
    zc = cam[..., 2]
    all_in = (zc >= z_near).all(axis=1)
    some_in = (zc >= z_near).any(axis=1)
    tri_cam = [cam[all_in]]
    tri_ids = [np.nonzero(all_in)[0]]
    for t in np.nonzero(some_in & ~all_in)[0]:
        for piece in _clip_near(cam[t], z_near):
            tri_cam.append(piece[None])
            tri_ids.append(np.array([t]))
    tc = np.concatenate(tri_cam)
    tid = np.concatenate(tri_ids)
    sx = width / 2.0 + f * tc[..., 0] / tc[..., 2]
    sy = height / 2.0 - f * tc[..., 1] / tc[..., 2]
    inv_z = 1.0 / tc[..., 2]

    x0 = np.clip(np.ceil(sx.min(axis=1) - 0.5), 0, width).astype(np.int64)
    x1 = np.clip(np.floor(sx.max(axis=1) - 0.5), -1, width - 1).astype(np.int64)
    y0 = np.clip(np.ceil(sy.min(axis=1) - 0.5), 0, height).astype(np.int64)
    y1 = np.clip(np.floor(sy.max(axis=1) - 0.5), -1, height - 1).astype(np.int64)
    bw = x1 - x0 + 1
    bh = y1 - y0 + 1
    live = (bw > 0) & (bh > 0)

    pix_all, z_all, t_all = [], [], []
    size = np.maximum(bw, bh)
    for lo_s, hi_s in ((1, 4), (5, 8), (9, 16), (17, 32), (33, 64), (65, 128), (129, 1 << 30)):
        sel = np.nonzero(live & (size >= lo_s) & (size <= hi_s))[0]
        if len(sel) == 0:
            continue
        B = hi_s if hi_s < (1 << 30) else None
        if B is None:
            for t in sel:  # very large triangles: one at a time, in row bands
                for ys in range(int(y0[t]), int(y1[t]) + 1, 64):
                    ye = min(int(y1[t]), ys + 63)
                    py, px = np.mgrid[ys:ye + 1, x0[t]:x1[t] + 1]
                    _raster_batch(np.array([t]), px[None], py[None], sx, sy, inv_z, tid,
                                  width, pix_all, z_all, t_all)
            continue
        chunk = max(1, (1 << 22) // (B * B))
        oy, ox = np.mgrid[0:B, 0:B]
        for c0 in range(0, len(sel), chunk):
            s = sel[c0:c0 + chunk]
            px = x0[s][:, None, None] + ox[None]
            py = y0[s][:, None, None] + oy[None]
            valid = (px <= x1[s][:, None, None]) & (py <= y1[s][:, None, None])
            _raster_batch(s, px, py, sx, sy, inv_z, tid, width, pix_all, z_all, t_all, valid)

    pix = np.concatenate(pix_all)
    z = np.concatenate(z_all)
    tt = np.concatenate(t_all)
    order = np.lexsort((tt, z, pix))
    pix, z, tt = pix[order], z[order], tt[order]
    first = np.ones(len(pix), dtype=bool)
    first[1:] = pix[1:] != pix[:-1]
    tri_id = np.full(width * height, -1, dtype=np.int32)
    depth = np.full(width * height, np.inf)
    tri_id[pix[first]] = tt[first]
    depth[pix[first]] = z[first]
    return tri_id, depth


def _raster_batch(s, px, py, sx, sy, inv_z, tid, width, pix_all, z_all, t_all, valid=None):
    cx = px + 0.5
    cy = py + 0.5
    ax, ay = sx[s, 0][:, None, None], sy[s, 0][:, None, None]
    bx, by = sx[s, 1][:, None, None], sy[s, 1][:, None, None]
    qx, qy = sx[s, 2][:, None, None], sy[s, 2][:, None, None]
    w0 = (qx - bx) * (cy - by) - (qy - by) * (cx - bx)  # opposite vertex 0
    w1 = (ax - qx) * (cy - qy) - (ay - qy) * (cx - qx)  # opposite vertex 1
    w2 = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)  # opposite vertex 2
    area = w0 + w1 + w2
    inside = (((w0 >= 0) & (w1 >= 0) & (w2 >= 0)) | ((w0 <= 0) & (w1 <= 0) & (w2 <= 0))) & (area != 0)
    if valid is not None:
        inside &= valid
    k, yy, xx = np.nonzero(inside)
    if len(k) == 0:
        return
    ar = area[k, yy, xx]
    l0, l1, l2 = w0[k, yy, xx] / ar, w1[k, yy, xx] / ar, w2[k, yy, xx] / ar
    iz = l0 * inv_z[s[k], 0] + l1 * inv_z[s[k], 1] + l2 * inv_z[s[k], 2]
    pix_all.append(py[k, yy, xx] * width + px[k, yy, xx])
    z_all.append(1.0 / iz)
    t_all.append(tid[s[k]].astype(np.int32))


@dataclasses.dataclass
class GBuffer:
    width: int
    height: int
    p: np.ndarray     # (H*W,3) float64 visible point, tile-major order
    n: np.ndarray     # (H*W,3) float64 geometric normal facing the camera
    tri: np.ndarray   # (H*W,) int32 visible triangle
    order: np.ndarray  # (H*W,) row-major pixel index of each tile-major slot


def tile_major_order(width: int, height: int, tile: int = 8) -> np.ndarray:
    """Row-major pixel index for each slot of an 8x8-tile-major ordering."""
    ty, tx, ly, lx = np.meshgrid(np.arange(height // tile), np.arange(width // tile),
                                 np.arange(tile), np.arange(tile), indexing="ij")
    return ((ty * tile + ly) * width + (tx * tile + lx)).reshape(-1)


def gbuffer(scene: Scene, width: int, height: int) -> GBuffer:
    """Visible surface point and normal per pixel of the pinhole camera, in
    8x8-tile-major order (one 64-wide wavefront per tile)."""
    assert width % 8 == 0 and height % 8 == 0
    tri_id, depth = rasterize(scene, width, height)
    # a pixel centre that fell exactly on a shared edge in both neighbours'
    # edge tests can be left uncovered: borrow the left (else upper) neighbour
    miss = np.nonzero(tri_id < 0)[0]
    for m in miss:
        for nb in (m - 1, m - width, m + 1, m + width):
            if 0 <= nb < len(tri_id) and tri_id[nb] >= 0:
                tri_id[m], depth[m] = tri_id[nb], depth[nb]
                break
    assert (tri_id >= 0).all(), "camera sees outside the scene"
    right, up, fwd = _camera_basis()
    f = (height / 2.0) / math.tan(math.radians(CAMERA_VFOV_DEG) / 2.0)
    order = tile_major_order(width, height)
    py, px = np.divmod(order, width)
    xc = (px + 0.5 - width / 2.0) / f
    yc = (height / 2.0 - (py + 0.5)) / f
    z = depth[order]
    p = CAMERA_EYE + z[:, None] * (xc[:, None] * right + yc[:, None] * up + fwd)
    tri = tri_id[order]
    n = _tri_normals(scene)[tri]
    flip = np.einsum("ij,ij->i", n, CAMERA_EYE - p) < 0
    n[flip] *= -1.0
    return GBuffer(width, height, p, n, tri, order)


def gbuffer_rays(gb: GBuffer, seed: int, eps: float = 1e-5, spp: int = 1) -> Rays:
    """`spp` cosine-hemisphere diffuse rays per G-buffer pixel, origin p+eps*n.
    With spp > 1 the samples of one pixel are adjacent."""
    rng = _rng(seed)
    p = np.repeat(gb.p, spp, axis=0)
    n = np.repeat(gb.n, spp, axis=0)
    u = rng.random((len(p), 2))
    d = cosine_hemisphere(n, u[:, 0], u[:, 1])
    return Rays((p + eps * n).astype(np.float32), _normalize32(d))


LIGHT_CORNER = np.array([0.35, 0.97, 0.35])
LIGHT_EDGES = (np.array([0.3, 0.0, 0.0]), np.array([0.0, 0.0, 0.3]))


def shadow_rays(p: np.ndarray, n: np.ndarray, seed: int, eps: float = 1e-5):
    """Shadow rays from surface points p (normals n) to uniform samples on a
    0.3 x 0.3 area light just below the ceiling.  Returns (Rays, tmax) with
    tmax = the float32 distance to the light sample (rays from points that face
    away from the light are kept; they are simply occluded by their own
    surface's neighbourhood or not)."""
    rng = _rng(seed)
    u = rng.random((len(p), 2))
    q = LIGHT_CORNER + u[:, :1] * LIGHT_EDGES[0] + u[:, 1:] * LIGHT_EDGES[1]
    o = p + eps * n
    v = q - o
    dist = np.linalg.norm(v, axis=1)
    d = _normalize32(v / dist[:, None])
    return Rays(o.astype(np.float32), d), dist.astype(np.float32)


def rebias(rays: Rays, gb: GBuffer, eps: float, spp: int = 1) -> Rays:
    """Same directions as `rays`, origins moved to p + eps*n (the large normal
    bias a distance-field-only trace needs against self-intersection)."""
    p = np.repeat(gb.p, spp, axis=0)
    n = np.repeat(gb.n, spp, axis=0)
    return Rays((p + eps * n).astype(np.float32), rays.d.copy())


# ----------------------------------------------------------------------------
# many scenes of uneven size (batched tracing)
# ----------------------------------------------------------------------------

TRIS_PER_OBJECT = 376  # mean of the 432-triangle boxes and 320-triangle icospheres


@dataclasses.dataclass
class BatchSceneSpec:
    seed: int
    n_objects: int
    s_min: float
    s_max: float
    n_grid: int
    width: int
    height: int

    @property
    def n_rays(self) -> int:
        return self.width * self.height


def batch_specs(seed: int = 4, n_scenes: int = 64, tris=(1e3, 5e5), rays=(1e3, 2e6)) -> list:
    """Scenes of log-uniform size in `tris` triangles, each with a log-uniform
    number of rays in `rays` (one diffuse ray per pixel of a 16:9 G-buffer
    whose sides are multiples of 8) and a grid of 32^3 at the smallest size
    to 128^3 at the largest, log-linear in the triangle count (multiples of 8).
    Object sizes grow as objects get fewer, so every scene fills the room
    about as densely as the GI-shaped scene."""
    rng = _rng(seed)
    out = []
    lt, lr = np.log(tris), np.log(rays)
    for s in range(n_scenes):
        t = math.exp(rng.uniform(lt[0], lt[1]))
        r = math.exp(rng.uniform(lr[0], lr[1]))
        n_obj = max(2, int(round((t - 12) / TRIS_PER_OBJECT)))
        s_max = min(0.25, 0.06 * (500.0 / n_obj) ** (1.0 / 3.0))
        frac = (math.log(t) - lt[0]) / (lt[1] - lt[0])
        n_grid = int(min(128, max(32, 8 * round(32 * 4.0 ** frac / 8))))
        w = max(8, 8 * int(round(math.sqrt(r * 16.0 / 9.0) / 8)))
        h = max(8, 8 * int(round(r / w / 8)))
        out.append(BatchSceneSpec(1000 * seed + s, n_obj, s_max / 10.0, s_max, n_grid, w, h))
    return out


def batch_scene(spec: BatchSceneSpec) -> Scene:
    return make_scene(spec.seed, spec.n_objects, spec.s_min, spec.s_max)
