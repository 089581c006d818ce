// Exact signed distance at one grid node (internal header): the per-node body
// of the distance-field build kernel, host+device so a CPU build can check it.
//   distance  nearest-triangle query over the BVH in FP64: children in order of
//             their box distance, a subtree skipped once its box is no closer
//             than the best triangle; point/triangle distance = plane distance
//             when the projection falls inside, else the nearest edge segment;
//   sign      winding number from signed ray crossings along a fixed generic
//             direction (leaving through the front of a face +1, entering -1),
//             plus 1 when the exterior is solid; solid iff the total is >= 1.
#pragma once

#include "bvh_build.hpp"
#include "hyb_device.hpp"

namespace hyb {

struct D3 {
    double x, y, z;
};

HYB_HD D3 d3(double x, double y, double z) { return D3{x, y, z}; }
HYB_HD D3 dsub(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
HYB_HD double ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
HYB_HD D3 dcross(D3 a, D3 b) {
    return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
HYB_HD D3 dvert(float4 v) { return d3(v.x, v.y, v.z); }

// squared distance from p to the segment [a, b]
HYB_HD double seg_dist2(D3 p, D3 a, D3 b) {
    const D3 e = dsub(b, a), w = dsub(p, a);
    const double ee = ddot(e, e);
    double s = ee > 0.0 ? ddot(w, e) / ee : 0.0;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    const D3 r = d3(w.x - s * e.x, w.y - s * e.y, w.z - s * e.z);
    return ddot(r, r);
}

// squared distance from p to triangle abc
HYB_HD double tri_dist2(D3 p, D3 a, D3 b, D3 c) {
    const D3 n = dcross(dsub(b, a), dsub(c, a));
    const double nn = ddot(n, n);
    if (nn > 0.0) {
        // the projection of p lies inside iff p is on the inner side of all
        // three edge planes (each contains an edge and the normal)
        const bool in_ab = ddot(dcross(dsub(b, a), dsub(p, a)), n) >= 0.0;
        const bool in_bc = ddot(dcross(dsub(c, b), dsub(p, b)), n) >= 0.0;
        const bool in_ca = ddot(dcross(dsub(a, c), dsub(p, c)), n) >= 0.0;
        if (in_ab && in_bc && in_ca) {
            const double h = ddot(dsub(p, a), n);
            return h * h / nn;
        }
    }
    return fmin(seg_dist2(p, a, b), fmin(seg_dist2(p, b, c), seg_dist2(p, c, a)));
}

HYB_HD double box_dist2(D3 p, float lx, float hx, float ly, float hy, float lz, float hz) {
    const double dx = fmax(fmax((double)lx - p.x, 0.0), p.x - (double)hx);
    const double dy = fmax(fmax((double)ly - p.y, 0.0), p.y - (double)hy);
    const double dz = fmax(fmax((double)lz - p.z, 0.0), p.z - (double)hz);
    return dx * dx + dy * dy + dz * dz;
}

// ray (o + t D, t > 0) against a box, FP64
HYB_HD bool ray_box64(D3 o, D3 inv, float lx, float hx, float ly, float hy, float lz, float hz) {
    const double t0x = ((double)lx - o.x) * inv.x, t1x = ((double)hx - o.x) * inv.x;
    const double t0y = ((double)ly - o.y) * inv.y, t1y = ((double)hy - o.y) * inv.y;
    const double t0z = ((double)lz - o.z) * inv.z, t1z = ((double)hz - o.z) * inv.z;
    const double tn = fmax(fmax(fmin(t0x, t1x), fmin(t0y, t1y)), fmax(fmin(t0z, t1z), 0.0));
    const double tf = fmin(fmin(fmax(t0x, t1x), fmax(t0y, t1y)), fmax(t0z, t1z));
    return tn <= tf * (1.0 + 1e-12);
}

// signed crossing of the ray o + t D (t > 0) with triangle abc: +1 when the ray
// leaves through the front side (D . n > 0), -1 when it enters, 0 when it misses
// (edge functions of the triangle seen along D, all of one sign)
HYB_HD int crossing(D3 o, D3 D, D3 a, D3 b, D3 c) {
    const D3 pa = dsub(a, o), pb = dsub(b, o), pc = dsub(c, o);
    const double wa = ddot(D, dcross(pb, pc));
    const double wb = ddot(D, dcross(pc, pa));
    const double wc = ddot(D, dcross(pa, pb));
    if (!((wa >= 0.0 && wb >= 0.0 && wc >= 0.0) || (wa <= 0.0 && wb <= 0.0 && wc <= 0.0))) return 0;
    const double s = wa + wb + wc;
    if (s == 0.0) return 0;
    const D3 n = dcross(dsub(b, a), dsub(c, a));
    const double t = ddot(n, pa) / ddot(n, D);
    if (!(t > 0.0)) return 0;
    return ddot(D, n) > 0.0 ? 1 : -1;
}

// BVH2 queries push at most one entry per level, and the BVH2 is at most 64 deep.
constexpr int kStack2 = 64;

HYB_HD double sdf_node_value(const float4* __restrict__ nodes, const float4* __restrict__ tris, D3 p,
                             int exterior_solid) {
    int stack[kStack2];

    // nearest triangle: children in order of box distance; a popped subtree is
    // skipped when its box is no closer than the best triangle found since
    double best = __builtin_inf();
    double dstack[kStack2];
    int sp = 0;
    int ref = 0;
    for (;;) {
        if (ref >= 0) {
            const float4* nd = nodes + 4 * (int64_t)ref;
            const float4 A = nd[0], B = nd[1], C = nd[2], E = nd[3];
            const double d0 = box_dist2(p, A.x, A.y, A.z, A.w, C.x, C.y);
            const double d1 = box_dist2(p, B.x, B.y, B.z, B.w, C.z, C.w);
            const int r0 = bits_i(E.x), r1 = bits_i(E.y);
            const bool h0 = d0 < best && r0 != kEmptyRef, h1 = d1 < best && r1 != kEmptyRef;
            if (h0 && h1) {
                const bool first0 = d0 <= d1;
                dstack[sp] = first0 ? d1 : d0;
                stack[sp++] = first0 ? r1 : r0;
                ref = first0 ? r0 : r1;
                continue;
            }
            if (h0) { ref = r0; continue; }
            if (h1) { ref = r1; continue; }
        } else {
            const int info = ~ref;
            const int first = info >> 3, count = info & 7;
            for (int q = 0; q < count; ++q) {
                const float4* tp = tris + 3 * (int64_t)(first + q);
                best = fmin(best, tri_dist2(p, dvert(tp[0]), dvert(tp[1]), dvert(tp[2])));
            }
        }
        bool found = false;
        while (sp > 0) {
            --sp;
            if (dstack[sp] < best) {
                ref = stack[sp];
                found = true;
                break;
            }
        }
        if (!found) break;
    }

    // winding number along a fixed direction that no mesh edge is likely to contain
    const double Dn = sqrt(0.61 * 0.61 + 0.5177 * 0.5177 + 0.6003 * 0.6003);
    const D3 D = d3(0.61 / Dn, 0.5177 / Dn, 0.6003 / Dn);
    const D3 inv = d3(1.0 / D.x, 1.0 / D.y, 1.0 / D.z);
    int wind = exterior_solid ? 1 : 0;
    sp = 0;
    ref = 0;
    for (;;) {
        if (ref >= 0) {
            const float4* nd = nodes + 4 * (int64_t)ref;
            const float4 A = nd[0], B = nd[1], C = nd[2], E = nd[3];
            const int r0 = bits_i(E.x), r1 = bits_i(E.y);
            const bool h0 = r0 != kEmptyRef && ray_box64(p, inv, A.x, A.y, A.z, A.w, C.x, C.y);
            const bool h1 = r1 != kEmptyRef && ray_box64(p, inv, B.x, B.y, B.z, B.w, C.z, C.w);
            if (h0 && h1) {
                stack[sp++] = r1;
                ref = r0;
                continue;
            }
            if (h0) { ref = r0; continue; }
            if (h1) { ref = r1; continue; }
        } else {
            const int info = ~ref;
            const int first = info >> 3, count = info & 7;
            for (int q = 0; q < count; ++q) {
                const float4* tp = tris + 3 * (int64_t)(first + q);
                wind += crossing(p, D, dvert(tp[0]), dvert(tp[1]), dvert(tp[2]));
            }
        }
        if (sp == 0) break;
        ref = stack[--sp];
    }
    const double dist = sqrt(best);
    return wind >= 1 ? -dist : dist;
}

}  // namespace hyb
