"""Element-wise parity rule between a kernel result and the FP64 oracle.

A ray is *decided* when its oracle margin exceeds MARGIN (1e-5: in scene units
for triangle edges and near misses, relative for t gaps, in voxels for the
distance field's near-tangent minima).  On decided rays:
  - prim must match exactly (triangle id, -2 distance-field hit, -1 miss);
  - t must agree to 1e-5 relative, |dt| <= 1e-5 max(t_ref, 0.05), wherever the
    hit is also well conditioned (|cos| or |g'| >= 1e-2);
  - barycentrics must agree to UV_TOL;
  - misses report t = +inf and distance-field hits u = v = 0.
The excluded fraction is reported so a test can bound it.
"""
from __future__ import annotations

import numpy as np

MARGIN = 1e-5
COND = 1e-2
T_REL = 1e-5
T_FLOOR = 0.05
UV_TOL = 1e-4


def check(got, ref, margin, cond, label="", max_excluded=0.05, uv_tol=UV_TOL):
    t, prim, u, v = (np.asarray(x) for x in got[:4])
    rt, rp, ru, rv = (np.asarray(x) for x in ref[:4])
    n = len(t)
    dec = margin > MARGIN
    excl = 1.0 - dec.mean() if n else 0.0
    msgs = []
    bad_prim = dec & (prim != rp)
    if bad_prim.any():
        i = np.nonzero(bad_prim)[0][:5]
        msgs.append("%d prim mismatches, e.g. rays %s got %s ref %s (t %s ref %s, margin %s)" % (
            bad_prim.sum(), i.tolist(), prim[i].tolist(), rp[i].tolist(), t[i].tolist(), rt[i].tolist(),
            margin[i].tolist()))
    hit = dec & (rp != -1) & (prim == rp) & (cond >= COND)
    with np.errstate(invalid="ignore"):  # misses: inf - inf
        err = np.abs(t.astype(np.float64) - rt)
    tol = T_REL * np.maximum(rt, T_FLOOR)
    bad_t = hit & ~(err <= tol)
    if bad_t.any():
        i = np.nonzero(bad_t)[0][:5]
        msgs.append("%d t mismatches, e.g. rays %s got %s ref %s" % (bad_t.sum(), i.tolist(), t[i].tolist(),
                                                                    rt[i].tolist()))
    tri = dec & (rp >= 0) & (prim == rp)
    duv = np.maximum(np.abs(u - ru), np.abs(v - rv))
    bad_uv = tri & ~(duv <= uv_tol)
    if bad_uv.any():
        i = np.nonzero(bad_uv)[0][:5]
        msgs.append("%d uv mismatches, e.g. rays %s dmax %s" % (bad_uv.sum(), i.tolist(), duv[i].tolist()))
    miss = prim == -1
    if not np.all(np.isinf(t[miss])) or np.any(u[miss] != 0) or np.any(v[miss] != 0):
        msgs.append("miss encoding broken")
    dfh = prim == -2
    if np.any(u[dfh] != 0) or np.any(v[dfh] != 0) or not np.all(np.isfinite(t[dfh])):
        msgs.append("distance-field hit encoding broken")
    if excl > max_excluded:
        msgs.append("excluded fraction %.4f > %.4f" % (excl, max_excluded))
    stats = dict(n=n, excluded=float(excl), max_rel_t=float(np.max(err[hit] / np.maximum(rt[hit], T_FLOOR)))
                 if hit.any() else 0.0, max_duv=float(duv[tri].max()) if tri.any() else 0.0,
                 tri_hits=int((prim >= 0).sum()), df_hits=int((prim == -2).sum()), misses=int(miss.sum()))
    assert not msgs, "%s: %s\n%s" % (label, stats, "\n".join(msgs))
    return stats


def check_shadow(got, ref, margin, orc, verts, tris, rays_soa, segs, label="", max_excluded=0.05):
    """Any-hit parity: occlusion (prim != -1) and the distance-field class
    (prim == -2) match on decided rays; a reported triangle occluder must be hit
    by the ray in one of the triangle segments `segs` = [(a, b), (a, b)]."""
    t, prim = np.asarray(got[0]), np.asarray(got[1])
    rp = np.asarray(ref[1])
    dec = margin > MARGIN
    msgs = []
    bad = dec & ((prim != -1) != (rp != -1))
    if bad.any():
        i = np.nonzero(bad)[0][:5]
        msgs.append("%d occlusion mismatches, e.g. %s got %s ref %s" % (bad.sum(), i.tolist(), prim[i].tolist(),
                                                                       rp[i].tolist()))
    bad = dec & ((prim == -2) != (rp == -2))
    if bad.any():
        msgs.append("%d distance-field class mismatches" % bad.sum())
    tri = np.nonzero(dec & (prim >= 0))[0]
    for i in tri[:512]:
        r1 = np.ascontiguousarray(np.asarray(rays_soa)[:, i:i + 1])
        ok = False
        for a, b in segs:
            ai, bi = np.broadcast_to(a, (len(t),))[i], np.broadcast_to(b, (len(t),))[i]
            if bi < ai:
                continue
            h = orc.closest_hit(verts, np.asarray(tris)[prim[i]:prim[i] + 1], r1, ai, bi)
            ok |= h[1][0] == 0 and abs(h[0][0] - t[i]) <= 1e-5 * max(h[0][0], 0.05)
        if not ok:
            msgs.append("ray %d reports triangle %d at t=%s, not hit in the triangle segments" % (i, prim[i], t[i]))
            break
    excl = 1.0 - dec.mean()
    if excl > max_excluded:
        msgs.append("excluded fraction %.4f" % excl)
    assert not msgs, label + "\n" + "\n".join(msgs)
    return dict(n=len(t), excluded=float(excl), occluded=int((prim != -1).sum()), df=int((prim == -2).sum()))


def split_t1(tau, h, tmax):
    """The combined query's split point for rays with tmin = 0:
    t1 = min(fl32(0 + tau h), tmax) (one FP32 rounding, as an FMA gives)."""
    with np.errstate(over="ignore"):
        t1 = np.float32(tau) * np.float32(h) if np.isfinite(tau) else np.float32(np.inf)
    return np.float32(min(t1, np.float32(tmax)))


def combined_oracle(orc, verts, tris, grids, g4, rays_soa, tmax, tau):
    """The oracle's combined query (Eq. 2, first hit, sub-queries in order)
    for rays with tmin = 0 over several grids of one scene, its triangle
    sub-query computed once: triangles on [0, t1] (oracle mode 1), then, for
    the rays they missed, the distance field on [t1, tmax] (mode 2), with the
    margin composed the way the oracle's combined margin is (the triangle
    margin alone after a triangle hit, else the smaller of both, and the
    conditioning of the part that decides).  Returns [(ref, margin, cond)]
    per grid."""
    n = np.asarray(rays_soa).shape[1]
    t1 = split_t1(tau, g4[3], tmax)
    if t1 > 0:
        tm = np.full(n, t1, np.float32)
        tri = orc.query(verts, tris, None, None, rays_soa, tmax, 0.0, mode=orc.MODE_BVH, tmax_ray=tm)
        mt, ct = orc.margin(verts, tris, None, None, rays_soa, tmax, 0.0, mode=orc.MODE_BVH, tmax_ray=tm)
        hit = tri[1] >= 0
    else:
        tri, hit = None, np.zeros(n, bool)
    out = []
    for grid in grids:
        if t1 < np.float32(tmax) or tau == 0.0:
            t0 = np.full(n, t1, np.float32)
            df = orc.query(None, np.zeros((0, 3), np.int32), grid, g4, rays_soa, tmax, 0.0, mode=orc.MODE_DF, tmin=t0)
            md, cd = orc.margin(None, np.zeros((0, 3), np.int32), grid, g4, rays_soa, tmax, 0.0, mode=orc.MODE_DF,
                                tmin=t0)
        else:
            df = (np.full(n, np.inf), np.full(n, -1, np.int32), np.zeros(n), np.zeros(n))
            md, cd = np.full(n, np.inf), np.ones(n)
        if tri is None:
            out.append((df, md, cd))
            continue
        ref = tuple(np.where(hit, a, b) for a, b in zip(tri, df))
        m = np.where(hit, mt, np.minimum(mt, md))
        c = np.where(hit, ct, cd)
        out.append((ref, m, c))
    return out


def lossless_grid(grid):
    """The grid rounded to integer multiples q s of one power of two s with
    |q| <= 127 (s the smallest with 127 s >= max |grid|): F16 holds every
    such value exactly, and so does I8, whose scale of any block is a power
    of two dividing s (codes q s / scale stay within 127, also on the faces
    blocks share), so all formats store the same samples."""
    g = np.asarray(grid, np.float32)
    m = float(np.abs(g).max())
    s = 2.0 ** int(np.ceil(np.log2(m / 127.0))) if m > 0 else 1.0
    q = np.clip(np.rint(g.astype(np.float64) / s), -127, 127)
    return (q * s).astype(np.float32)
