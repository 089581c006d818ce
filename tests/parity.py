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
