/*
 * oracle.c - plain FP64 CPU reference for the combined ray query of
 * Bartels & Harada, "Combining GPU Tracing Methods within a Single Ray Query"
 * (SIGGRAPH Asia 2022 Technical Communications).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct definition the
 * GPU library is checked against.  Only the test suite, the package smoke check
 * and the CPU-baseline leg of the benchmark load it; the product path never
 * does.  It shares no source, header, helper or table with the GPU library.
 *
 * All inputs are the FP32 values the GPU sees (vertices, rays, grid samples,
 * tmin/tmax/threshold), promoted exactly to FP64; all arithmetic is FP64.
 *
 * Parts (each cites the passage it follows):
 *   O-1  closest triangle hit on [a,b]        Section 2, Eq. (1) on a sub-interval
 *   O-2  trilinear distance-field interpolant  (distance-field tracing, Sections 1 and 3)
 *   O-3  first distance-field root on [a,b]    (same; first-hit semantics of Section 2)
 *   O-4  combined query                        Section 2, Eq. (2), first-hit in order;
 *                                              Section 3 (AO): t1 from voxel size x multiplier
 *   O-5  exact signed distance grid from the mesh (input construction for O-3)
 *   O-6  d(hit t)/d(grid sample) at a DF hit   implicit differentiation of g(t*)=0
 *   margins used by the parity tests to exclude ill-posed rays
 */
#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Number of OpenMP threads the parallel loops use. */
int oracle_threads(void) { return omp_get_max_threads(); }

typedef struct { double x, y, z; } vec;

static vec mk(double x, double y, double z) { vec r = {x, y, z}; return r; }
static vec sub(vec a, vec b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static vec add(vec a, vec b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static vec scl(vec a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(vec a, vec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static vec cross(vec a, vec b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double norm(vec a) { return sqrt(dot(a, a)); }
static double comp(vec a, int axis) { return axis == 0 ? a.x : (axis == 1 ? a.y : a.z); }

static vec vert(const float* verts, int32_t i) {
    return mk((double)verts[3 * (int64_t)i], (double)verts[3 * (int64_t)i + 1], (double)verts[3 * (int64_t)i + 2]);
}

/* rays are SoA float32: rows ox,oy,oz,dx,dy,dz each of length n */
static vec ray_o(const float* r, int64_t n, int64_t i) { return mk(r[i], r[n + i], r[2 * n + i]); }
static vec ray_d(const float* r, int64_t n, int64_t i) { return mk(r[3 * n + i], r[4 * n + i], r[5 * n + i]); }

/* ------------------------------------------------------------------------- */
/* O-1: closest triangle hit                                                  */
/* ------------------------------------------------------------------------- */

/* Moller-Trumbore (1997), no back-face culling.  Returns 1 when the line
 * o + t d meets the closed triangle; (t,u,v) with hit = (1-u-v) a + u b + v c. */
static int mt_hit(vec o, vec d, vec a, vec b, vec c, double* t, double* u, double* v) {
    vec e1 = sub(b, a), e2 = sub(c, a);
    vec P = cross(d, e2);
    double det = dot(e1, P);
    if (det == 0.0) return 0;
    vec T = sub(o, a);
    double uu = dot(T, P) / det;
    vec Q = cross(T, e1);
    double vv = dot(d, Q) / det;
    double tt = dot(e2, Q) / det;
    if (!(uu >= 0.0 && vv >= 0.0 && uu + vv <= 1.0)) return 0;
    *t = tt; *u = uu; *v = vv;
    return 1;
}

/* Closest hit over every triangle with a <= t <= b; equal t goes to the
 * smallest triangle index.  prim = -1 and t = +inf on a miss. */
static void closest_one(const float* verts, const int32_t* tris, int64_t ntri, vec o, vec d,
                        double a, double b, double* t_out, int32_t* prim_out, double* u_out, double* v_out) {
    double bt = INFINITY, bu = 0.0, bv = 0.0;
    int32_t bp = -1;
    for (int64_t k = 0; k < ntri; ++k) {
        double t, u, v;
        if (!mt_hit(o, d, vert(verts, tris[3 * k]), vert(verts, tris[3 * k + 1]), vert(verts, tris[3 * k + 2]), &t, &u, &v))
            continue;
        if (t < a || t > b) continue;
        if (t < bt) { bt = t; bu = u; bv = v; bp = (int32_t)k; }
    }
    *t_out = bt; *prim_out = bp; *u_out = bu; *v_out = bv;
}

void oracle_closest_hit(const float* verts, const int32_t* tris, int64_t ntri,
                        const float* rays, int64_t n, const double* a, const double* b,
                        double* t_out, int32_t* prim_out, double* u_out, double* v_out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        closest_one(verts, tris, ntri, ray_o(rays, n, i), ray_d(rays, n, i), a[i], b[i],
                    &t_out[i], &prim_out[i], &u_out[i], &v_out[i]);
}

/* ------------------------------------------------------------------------- */
/* O-5: exact signed distance at grid nodes                                   */
/* ------------------------------------------------------------------------- */

/* Closest point on triangle abc to p by Voronoi regions (Ericson, Real-Time
 * Collision Detection, 5.1.5). */
static vec closest_on_tri(vec p, vec a, vec b, vec c) {
    vec ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return a;
    vec bp = sub(p, b);
    double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) return b;
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return add(a, scl(ab, d1 / (d1 - d3)));
    vec cp = sub(p, c);
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return c;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return add(a, scl(ac, d2 / (d2 - d6)));
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0)
        return add(b, scl(sub(c, b), (d4 - d3) / ((d4 - d3) + (d5 - d6))));
    double den = 1.0 / (va + vb + vc);
    return add(a, add(scl(ab, vb * den), scl(ac, vc * den)));
}

static double dist_tri(vec p, const float* verts, const int32_t* t) {
    vec q = closest_on_tri(p, vert(verts, t[0]), vert(verts, t[1]), vert(verts, t[2]));
    return norm(sub(p, q));
}

/* Solid test from the object records: each object group is a closed convex
 * polytope with outward faces; the room group (kind 0) faces inwards and
 * everything not strictly inside it is solid.  With `bound` (per group a
 * sphere holding every vertex, so the whole polytope) an object group whose
 * sphere does not hold p is skipped: p cannot be inside it. */
static int is_solid(vec p, const float* verts, const int32_t* tris,
                    const int32_t* gstart, const int32_t* gcount, const int32_t* gkind, int ngroups,
                    const double* bound) {
    for (int g = 0; g < ngroups; ++g) {
        if (bound && gkind[g] != 0 &&
            norm(sub(p, mk(bound[4 * g], bound[4 * g + 1], bound[4 * g + 2]))) > bound[4 * g + 3])
            continue;
        int inside_all = 1, strictly = 1;
        for (int32_t k = gstart[g]; k < gstart[g] + gcount[g]; ++k) {
            const int32_t* t = tris + 3 * (int64_t)k;
            vec a = vert(verts, t[0]);
            vec nrm = cross(sub(vert(verts, t[1]), a), sub(vert(verts, t[2]), a));
            double s = dot(sub(p, a), nrm);
            if (gkind[g] == 0) { if (!(s > 0.0)) { strictly = 0; break; } }
            else if (s > 0.0) { inside_all = 0; break; }
        }
        if (gkind[g] == 0 && !strictly) return 1;
        if (gkind[g] != 0 && inside_all) return 1;
    }
    return 0;
}

typedef struct {
    const float* verts;
    const int32_t* tris;
    int64_t ntri;
    const int32_t *gstart, *gcount, *gkind;
    int ngroups;
    double* bound; /* per group: bounding-sphere centre xyz and radius */
} mesh_t;

static void mesh_init(mesh_t* M, const float* verts, const int32_t* tris, int64_t ntri,
                      const int32_t* gstart, const int32_t* gcount, const int32_t* gkind, int ngroups) {
    M->verts = verts; M->tris = tris; M->ntri = ntri;
    M->gstart = gstart; M->gcount = gcount; M->gkind = gkind; M->ngroups = ngroups;
    M->bound = (double*)malloc(sizeof(double) * 4 * (size_t)(ngroups > 0 ? ngroups : 1));
    for (int g = 0; g < ngroups; ++g) {
        vec lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
        for (int32_t k = gstart[g]; k < gstart[g] + gcount[g]; ++k)
            for (int c = 0; c < 3; ++c) {
                vec v = vert(verts, tris[3 * (int64_t)k + c]);
                lo = mk(fmin(lo.x, v.x), fmin(lo.y, v.y), fmin(lo.z, v.z));
                hi = mk(fmax(hi.x, v.x), fmax(hi.y, v.y), fmax(hi.z, v.z));
            }
        vec cen = scl(add(lo, hi), 0.5);
        double r = 0.0;
        for (int32_t k = gstart[g]; k < gstart[g] + gcount[g]; ++k)
            for (int c = 0; c < 3; ++c) r = fmax(r, norm(sub(vert(verts, tris[3 * (int64_t)k + c]), cen)));
        M->bound[4 * g] = cen.x; M->bound[4 * g + 1] = cen.y; M->bound[4 * g + 2] = cen.z;
        M->bound[4 * g + 3] = r * (1.0 + 1e-12);
    }
}

typedef struct {
    double lb;
    int g;
} group_lb;

static int cmp_group_lb(const void* a, const void* b) {
    double x = ((const group_lb*)a)->lb, y = ((const group_lb*)b)->lb;
    return (x > y) - (x < y);
}

/* Signed distance at p: minimum Euclidean distance over every triangle,
 * negative when solid.  With prune != 0 the group whose bounding sphere is
 * nearest is measured first, then the groups whose sphere lies within the best
 * distance so far, in order of that distance, stopping at the first whose
 * sphere already lies farther than the best distance found;
 * this cannot change the minimum (every triangle of a group is at least as far
 * as its bounding sphere, and the minimum of exact values does not depend on
 * their order).  The solid test skips the groups whose sphere excludes p. */
static double signed_dist(const mesh_t* M, vec p, int prune) {
    double best = INFINITY;
    if (!prune) {
        for (int64_t t = 0; t < M->ntri; ++t) best = fmin(best, dist_tri(p, M->verts, M->tris + 3 * t));
        return is_solid(p, M->verts, M->tris, M->gstart, M->gcount, M->gkind, M->ngroups, NULL) ? -best : best;
    }
    group_lb* order = (group_lb*)malloc(sizeof(group_lb) * (size_t)(M->ngroups > 0 ? M->ngroups : 1));
    int g0 = 0;
    for (int g = 0; g < M->ngroups; ++g) {
        order[g].lb = norm(sub(p, mk(M->bound[4 * g], M->bound[4 * g + 1], M->bound[4 * g + 2]))) - M->bound[4 * g + 3];
        order[g].g = g;
        if (order[g].lb < order[g0].lb) g0 = g;
    }
    /* the nearest sphere's group first; then only the groups whose sphere
     * lies within that distance, nearest first */
    if (M->ngroups > 0)
        for (int32_t t = M->gstart[g0]; t < M->gstart[g0] + M->gcount[g0]; ++t)
            best = fmin(best, dist_tri(p, M->verts, M->tris + 3 * (int64_t)t));
    int nc = 0;
    for (int g = 0; g < M->ngroups; ++g)
        if (g != g0 && order[g].lb <= best * (1.0 + 1e-12)) order[nc++] = order[g];
    qsort(order, (size_t)nc, sizeof(group_lb), cmp_group_lb);
    for (int q = 0; q < nc; ++q) {
        if (order[q].lb > best * (1.0 + 1e-12)) break;
        const int g = order[q].g;
        for (int32_t t = M->gstart[g]; t < M->gstart[g] + M->gcount[g]; ++t)
            best = fmin(best, dist_tri(p, M->verts, M->tris + 3 * (int64_t)t));
    }
    free(order);
    return is_solid(p, M->verts, M->tris, M->gstart, M->gcount, M->gkind, M->ngroups, M->bound) ? -best : best;
}

/* Exact signed distance at the listed nodes p = lo + (i,j,k) h, node index
 * i + N (j + N k). */
void oracle_sdf_nodes(const float* verts, const int32_t* tris, int64_t ntri,
                      const int32_t* gstart, const int32_t* gcount, const int32_t* gkind, int ngroups,
                      const float* grid4, int N, const int64_t* nodes, int64_t nn, int prune,
                      double* f_out) {
    mesh_t M;
    mesh_init(&M, verts, tris, ntri, gstart, gcount, gkind, ngroups);
    vec lo = mk(grid4[0], grid4[1], grid4[2]);
    double h = grid4[3];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < nn; ++q) {
        int64_t id = nodes[q];
        int64_t i = id % N, j = (id / N) % N, k = id / ((int64_t)N * N);
        vec p = mk(lo.x + (double)i * h, lo.y + (double)j * h, lo.z + (double)k * h);
        f_out[q] = signed_dist(&M, p, prune);
    }
    free(M.bound);
}

/* Exact signed distance at arbitrary points (n x 3, FP64). */
void oracle_sdf_points(const float* verts, const int32_t* tris, int64_t ntri,
                       const int32_t* gstart, const int32_t* gcount, const int32_t* gkind, int ngroups,
                       const double* pts, int64_t n, double* f_out) {
    mesh_t M;
    mesh_init(&M, verts, tris, ntri, gstart, gcount, gkind, ngroups);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < n; ++q) f_out[q] = signed_dist(&M, mk(pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]), 1);
    free(M.bound);
}

/* ------------------------------------------------------------------------- */
/* O-2 / O-3: trilinear interpolant and its first root along a ray            */
/* ------------------------------------------------------------------------- */

typedef struct {
    const double* g;
    int N;
    vec lo;
    double h;
} grid_t;

static double sample(const grid_t* G, int i, int j, int k) {
    return G->g[(int64_t)i + (int64_t)G->N * ((int64_t)j + (int64_t)G->N * k)];
}

/* Cell of a point: floor((p - lo)/h) clamped to [0, N-2] per axis. */
static void cell_of(const grid_t* G, vec p, int c[3]) {
    for (int a = 0; a < 3; ++a) {
        double x = (comp(p, a) - comp(G->lo, a)) / G->h;
        double f = floor(x);
        if (f < 0.0) f = 0.0;
        if (f > G->N - 2) f = G->N - 2;
        c[a] = (int)f;
    }
}

/* Trilinear blend of the 8 corners of cell c at point p. */
static double trilerp(const grid_t* G, const int c[3], vec p) {
    double fx = (p.x - G->lo.x) / G->h - c[0];
    double fy = (p.y - G->lo.y) / G->h - c[1];
    double fz = (p.z - G->lo.z) / G->h - c[2];
    double r = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                r += sample(G, c[0] + dx, c[1] + dy, c[2] + dz) * (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) *
                     (dz ? fz : 1.0 - fz);
    return r;
}

double oracle_df_value(const double* grid, int N, const float* grid4, double px, double py, double pz) {
    grid_t G = {grid, N, mk(grid4[0], grid4[1], grid4[2]), grid4[3]};
    int c[3];
    vec p = mk(px, py, pz);
    cell_of(&G, p, c);
    return trilerp(&G, c, p);
}

/* Interpolant at many points (n x 3). */
void oracle_df_values(const double* grid, int N, const float* grid4, const double* pts, int64_t n, double* out) {
    grid_t G = {grid, N, mk(grid4[0], grid4[1], grid4[2]), grid4[3]};
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int c[3];
        vec p = mk(pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]);
        cell_of(&G, p, c);
        out[q] = trilerp(&G, c, p);
    }
}

/* Clip [a,b] to the grid box [lo, lo+(N-1)h]^3 (slab test). Returns 0 if empty. */
static int clip_box(const grid_t* G, vec o, vec d, double* a, double* b) {
    double t0 = *a, t1 = *b;
    for (int ax = 0; ax < 3; ++ax) {
        double lo = comp(G->lo, ax), hi = lo + (G->N - 1) * G->h;
        double oa = comp(o, ax), da = comp(d, ax);
        if (da == 0.0) {
            if (oa < lo || oa > hi) return 0;
            continue;
        }
        double ta = (lo - oa) / da, tb = (hi - oa) / da;
        if (ta > tb) { double s = ta; ta = tb; tb = s; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (t0 > t1) return 0;
    *a = t0; *b = t1;
    return 1;
}

/* Coefficients of g(s) = trilinear(o + (t0+s) d) inside cell c as a cubic
 * k[0] + k[1] s + k[2] s^2 + k[3] s^3: every corner weight is a product of
 * three factors linear in s. */
static void cell_cubic(const grid_t* G, const int c[3], vec o, vec d, double t0, double k[4]) {
    vec p0 = add(o, scl(d, t0));
    double x0[3], dx[3];
    for (int a = 0; a < 3; ++a) {
        x0[a] = (comp(p0, a) - comp(G->lo, a)) / G->h - c[a];
        dx[a] = comp(d, a) / G->h;
    }
    k[0] = k[1] = k[2] = k[3] = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                int bit[3] = {cx, cy, cz};
                double al[3], be[3];
                for (int a = 0; a < 3; ++a) {
                    al[a] = bit[a] ? x0[a] : 1.0 - x0[a];
                    be[a] = bit[a] ? dx[a] : -dx[a];
                }
                /* (al0 + be0 s)(al1 + be1 s)(al2 + be2 s) */
                double p0c = al[0] * al[1] * al[2];
                double p1c = be[0] * al[1] * al[2] + al[0] * be[1] * al[2] + al[0] * al[1] * be[2];
                double p2c = be[0] * be[1] * al[2] + be[0] * al[1] * be[2] + al[0] * be[1] * be[2];
                double p3c = be[0] * be[1] * be[2];
                double f = sample(G, c[0] + cx, c[1] + cy, c[2] + cz);
                k[0] += f * p0c; k[1] += f * p1c; k[2] += f * p2c; k[3] += f * p3c;
            }
}

static double cub(const double k[4], double s) { return ((k[3] * s + k[2]) * s + k[1]) * s + k[0]; }
static double dcub(const double k[4], double s) { return (3.0 * k[3] * s + 2.0 * k[2]) * s + k[1]; }

/* Real roots of g'(s) = 3k3 s^2 + 2k2 s + k1 strictly inside (0,S), sorted. */
static int crit_points(const double k[4], double S, double r[2]) {
    double A = 3.0 * k[3], B = 2.0 * k[2], C = k[1];
    double cand[2];
    int m = 0;
    if (A == 0.0) {
        if (B != 0.0) cand[m++] = -C / B;
    } else {
        double disc = B * B - 4.0 * A * C;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -0.5 * (B + (B >= 0.0 ? sq : -sq));
            if (q != 0.0) { cand[m++] = q / A; cand[m++] = C / q; }
            else cand[m++] = 0.0; /* B = 0 and disc = 0: double root at 0 */
        }
    }
    int nr = 0;
    for (int i = 0; i < m; ++i)
        if (cand[i] > 0.0 && cand[i] < S) r[nr++] = cand[i];
    if (nr == 2 && r[0] > r[1]) { double s = r[0]; r[0] = r[1]; r[1] = s; }
    return nr;
}

/* Smallest s in (s0, s1] with g(s) <= 0 when g(s0) > 0 >= g(s1) and g is
 * monotone on [s0, s1]: bisection to FP64 resolution. */
static double bisect(const double k[4], double s0, double s1) {
    double lo = s0, hi = s1;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (cub(k, mid) <= 0.0) hi = mid; else lo = mid;
    }
    return hi;
}

/* One DDA step state (Amanatides & Woo 1987). */
typedef struct {
    int c[3], step[3];
    double tnext[3], tdelta[3];
} dda_t;

static void dda_init(const grid_t* G, vec o, vec d, double t, dda_t* s) {
    cell_of(G, add(o, scl(d, t)), s->c);
    for (int a = 0; a < 3; ++a) {
        double da = comp(d, a), oa = comp(o, a), lo = comp(G->lo, a);
        if (da > 0.0) {
            s->step[a] = 1;
            s->tnext[a] = (lo + (s->c[a] + 1) * G->h - oa) / da;
            s->tdelta[a] = G->h / da;
        } else if (da < 0.0) {
            s->step[a] = -1;
            s->tnext[a] = (lo + s->c[a] * G->h - oa) / da;
            s->tdelta[a] = -G->h / da;
        } else {
            s->step[a] = 0;
            s->tnext[a] = INFINITY;
            s->tdelta[a] = INFINITY;
        }
    }
}

static int dda_next_axis(const dda_t* s) {
    int a = 0;
    if (s->tnext[1] < s->tnext[a]) a = 1;
    if (s->tnext[2] < s->tnext[a]) a = 2;
    return a;
}

/* O-3: the first t in [a,b] (clipped to the grid box) where the trilinear
 * interpolant is <= 0; +inf when there is none.  Walks every cell the segment
 * crosses; inside a cell the interpolant is the cubic above, split into
 * monotone pieces at the roots of its derivative. */
static double df_first_root(const grid_t* G, vec o, vec d, double a, double b) {
    if (!clip_box(G, o, d, &a, &b)) return INFINITY;
    dda_t s;
    dda_init(G, o, d, a, &s);
    double t_in = a;
    for (;;) {
        int ax = dda_next_axis(&s);
        double t_out = s.tnext[ax] < b ? s.tnext[ax] : b;
        if (t_out < t_in) t_out = t_in;
        double k[4];
        cell_cubic(G, s.c, o, d, t_in, k);
        double S = t_out - t_in;
        if (cub(k, 0.0) <= 0.0) return t_in;
        double r[2];
        int nr = crit_points(k, S, r);
        double ends[3];
        int ne = 0;
        for (int i = 0; i < nr; ++i) ends[ne++] = r[i];
        ends[ne++] = S;
        double prev = 0.0;
        for (int i = 0; i < ne; ++i) {
            if (cub(k, ends[i]) <= 0.0) return t_in + bisect(k, prev, ends[i]);
            prev = ends[i];
        }
        if (t_out >= b) return INFINITY;
        /* advance to the neighbouring cell */
        s.c[ax] += s.step[ax];
        if (s.c[ax] < 0 || s.c[ax] > G->N - 2) return INFINITY;
        t_in = t_out;
        s.tnext[ax] += s.tdelta[ax];
    }
}

void oracle_df_hit(const double* grid, int N, const float* grid4, const float* rays, int64_t n,
                   const double* a, const double* b, double* t_out) {
    grid_t G = {grid, N, mk(grid4[0], grid4[1], grid4[2]), grid4[3]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        t_out[i] = df_first_root(&G, ray_o(rays, n, i), ray_d(rays, n, i), a[i], b[i]);
}

/* Lipschitz bound of the interpolant: max over cells of
 * sqrt(max|dx|^2 + max|dy|^2 + max|dz|^2) / h, where max|dx| is the largest
 * sample difference along the four x-edges of the cell (and so on): inside a
 * cell each partial derivative is a convex blend of its edge differences / h. */
double oracle_lipschitz(const double* grid, int N, double h) {
    grid_t G = {grid, N, mk(0, 0, 0), h};
    double L = 0.0;
    for (int k = 0; k + 1 < N; ++k)
        for (int j = 0; j + 1 < N; ++j)
            for (int i = 0; i + 1 < N; ++i) {
                double mx = 0, my = 0, mz = 0;
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) {
                        mx = fmax(mx, fabs(sample(&G, i + 1, j + u, k + v) - sample(&G, i, j + u, k + v)));
                        my = fmax(my, fabs(sample(&G, i + u, j + 1, k + v) - sample(&G, i + u, j, k + v)));
                        mz = fmax(mz, fabs(sample(&G, i + u, j + v, k + 1) - sample(&G, i + u, j + v, k)));
                    }
                L = fmax(L, sqrt(mx * mx + my * my + mz * mz) / h);
            }
    return L;
}

/* Cross-check for O-3: the straightforward sphere tracer.  Steps g/L from a
 * (clipped), stops once g <= eps (then finishes with bisection between the last
 * two positions) or when t passes b.  status: 0 ok, 1 step budget exhausted. */
void oracle_sphere_trace(const double* grid, int N, const float* grid4, double L, const float* rays, int64_t n,
                         const double* a, const double* b, double eps, int64_t max_steps,
                         double* t_out, int32_t* status) {
    grid_t G = {grid, N, mk(grid4[0], grid4[1], grid4[2]), grid4[3]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        vec o = ray_o(rays, n, i), d = ray_d(rays, n, i);
        double lo = a[i], hi = b[i];
        status[i] = 0;
        t_out[i] = INFINITY;
        if (!clip_box(&G, o, d, &lo, &hi)) continue;
        double t = lo;
        int64_t it;
        for (it = 0; it < max_steps; ++it) {
            int c[3];
            vec p = add(o, scl(d, t));
            cell_of(&G, p, c);
            double g = trilerp(&G, c, p);
            if (g <= 0.0) { t_out[i] = t; break; }
            if (g <= eps) {
                /* the root lies within a few g/|g'| ahead: bracket it and bisect */
                double step = g / L, tl = t, th = t;
                double gh = g;
                while (gh > 0.0 && th <= hi) {
                    tl = th;
                    th += step;
                    step *= 2.0;
                    vec q = add(o, scl(d, th));
                    cell_of(&G, q, c);
                    gh = trilerp(&G, c, q);
                }
                if (gh > 0.0) break; /* grazed: no root before hi */
                for (int r = 0; r < 200; ++r) {
                    double mid = 0.5 * (tl + th);
                    if (mid <= tl || mid >= th) break;
                    vec q = add(o, scl(d, mid));
                    cell_of(&G, q, c);
                    if (trilerp(&G, c, q) <= 0.0) th = mid; else tl = mid;
                }
                t_out[i] = th;
                break;
            }
            t += g / L;
            if (t > hi) break;
        }
        if (it == max_steps) status[i] = 1;
    }
}

/* ------------------------------------------------------------------------- */
/* O-4: combined query                                                        */
/* ------------------------------------------------------------------------- */

/* The split point: t1 = tmin + threshold * h rounded once to FP32, capped at
 * tmax; the same FP32 value the query is specified with.  threshold = +inf
 * gives t1 = tmax. */
static double split_point(float tmin, float tmax, float tau, float h) {
    float t1 = fmaf(tau, h, tmin);
    return (double)(t1 < tmax ? t1 : tmax);
}

/* Second split point of the shadow query: t2 = max(fl32(tmax - tau_end h), t1). */
static double split_end(float tmax, float tau_end, float h, double t1) {
    float t2 = fmaf(-tau_end, h, tmax);
    return (double)t2 > t1 ? (double)t2 : t1;
}

/* mode 0: combined (BVH on [tmin,t1] first, DF on [t1,tmax] only after a miss)
 * mode 1: triangles only on [tmin,tmax];  mode 2: distance field only on [tmin,tmax]
 * mode 3: shadow query, any hit: triangles on [tmin,t1] and [t2,tmax], DF on
 *         [t1,t2]; reported: the DF's first root if it has one, else the
 *         closest triangle of the first part, else of the last part.
 * Ray i ends at min(tmax_ray[i], tmax) when tmax_ray is given.
 * prim: >= 0 triangle, -2 distance-field hit, -1 miss (t = +inf). */
void oracle_query(const float* verts, const int32_t* tris, int64_t ntri,
                  const double* grid, int N, const float* grid4,
                  const float* rays, int64_t n, const float* tmin, const float* tmax_ray, float tmax_all,
                  float tau, float tau_end, int mode,
                  double* t_out, int32_t* prim_out, double* u_out, double* v_out) {
    grid_t G = {grid, N, mk(grid4 ? grid4[0] : 0, grid4 ? grid4[1] : 0, grid4 ? grid4[2] : 0), grid4 ? grid4[3] : 1.0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        vec o = ray_o(rays, n, i), d = ray_d(rays, n, i);
        float t0 = tmin ? tmin[i] : 0.0f;
        float tmax = tmax_ray ? fminf(tmax_ray[i], tmax_all) : tmax_all;
        double t, u, v;
        int32_t prim;
        t_out[i] = INFINITY; prim_out[i] = -1; u_out[i] = 0.0; v_out[i] = 0.0;
        if (!(t0 <= tmax)) continue;
        if (mode == 1) {
            closest_one(verts, tris, ntri, o, d, t0, tmax, &t, &prim, &u, &v);
            if (prim >= 0) { t_out[i] = t; prim_out[i] = prim; u_out[i] = u; v_out[i] = v; }
            continue;
        }
        if (mode == 2) {
            t = df_first_root(&G, o, d, t0, tmax);
            if (t < INFINITY) { t_out[i] = t; prim_out[i] = -2; }
            continue;
        }
        double t1 = split_point(t0, tmax, tau, (float)G.h);
        if (mode == 3) {
            double t2 = split_end(tmax, tau_end, (float)G.h, t1);
            if (t2 > t1 || (tau == 0.0f && tau_end == 0.0f)) {
                t = df_first_root(&G, o, d, t1, t2);
                if (t < INFINITY) { t_out[i] = t; prim_out[i] = -2; continue; }
            }
            if (t1 > t0) {
                closest_one(verts, tris, ntri, o, d, t0, t1, &t, &prim, &u, &v);
                if (prim >= 0) { t_out[i] = t; prim_out[i] = prim; u_out[i] = u; v_out[i] = v; continue; }
            }
            if ((double)tmax > t2) {
                closest_one(verts, tris, ntri, o, d, t2, tmax, &t, &prim, &u, &v);
                if (prim >= 0) { t_out[i] = t; prim_out[i] = prim; u_out[i] = u; v_out[i] = v; }
            }
            continue;
        }
        if (t1 > t0) {
            closest_one(verts, tris, ntri, o, d, t0, t1, &t, &prim, &u, &v);
            if (prim >= 0) { t_out[i] = t; prim_out[i] = prim; u_out[i] = u; v_out[i] = v; continue; }
        }
        if (t1 < tmax || tau == 0.0f) {
            t = df_first_root(&G, o, d, t1, tmax);
            if (t < INFINITY) { t_out[i] = t; prim_out[i] = -2; }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* O-6: gradient of the DF hit distance with respect to the grid samples      */
/* ------------------------------------------------------------------------- */

/* At a DF hit t* with g(t*; theta) = 0, implicit differentiation gives
 * dt_hit / dtheta_j = -w_j(p_hit) / (grad f~(p_hit) . d) for the 8 corners j of the
 * cell holding p_hit = o + t_hit d (w_j: trilinear weights) and 0 elsewhere.
 * A hit at the (clipped) segment start a' is not a root of g (the segment
 * began at or below zero), so t_hit = a' does not move with theta: zero.
 * For each ray writes the 8 node indices and 8 derivatives (node -1 when the
 * ray has no DF crossing or the denominator vanishes). */
void oracle_df_grad(const double* grid, int N, const float* grid4, const float* rays, int64_t n,
                    const double* a, const double* b, const double* t_hit, int64_t* node_out, double* dt_out) {
    grid_t G = {grid, N, mk(grid4[0], grid4[1], grid4[2]), grid4[3]};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < 8; ++j) { node_out[8 * i + j] = -1; dt_out[8 * i + j] = 0.0; }
        if (!(t_hit[i] < INFINITY)) continue;
        vec o = ray_o(rays, n, i), d = ray_d(rays, n, i);
        double a0 = a[i], b0 = b[i];
        if (!clip_box(&G, o, d, &a0, &b0) || t_hit[i] <= a0) continue;
        vec p = add(o, scl(d, t_hit[i]));
        int c[3];
        cell_of(&G, p, c);
        double f[3] = {(p.x - G.lo.x) / G.h - c[0], (p.y - G.lo.y) / G.h - c[1], (p.z - G.lo.z) / G.h - c[2]};
        double w[8], grad[3] = {0, 0, 0};
        for (int j = 0; j < 8; ++j) {
            int bx = j & 1, by = (j >> 1) & 1, bz = (j >> 2) & 1;
            double wx = bx ? f[0] : 1 - f[0], wy = by ? f[1] : 1 - f[1], wz = bz ? f[2] : 1 - f[2];
            double val = sample(&G, c[0] + bx, c[1] + by, c[2] + bz);
            w[j] = wx * wy * wz;
            grad[0] += val * (bx ? 1.0 : -1.0) * wy * wz / G.h;
            grad[1] += val * wx * (by ? 1.0 : -1.0) * wz / G.h;
            grad[2] += val * wx * wy * (bz ? 1.0 : -1.0) / G.h;
        }
        double gd = grad[0] * d.x + grad[1] * d.y + grad[2] * d.z;
        if (gd == 0.0) continue;
        for (int j = 0; j < 8; ++j) {
            int bx = j & 1, by = (j >> 1) & 1, bz = (j >> 2) & 1;
            node_out[8 * i + j] = (int64_t)(c[0] + bx) + (int64_t)N * ((int64_t)(c[1] + by) + (int64_t)N * (c[2] + bz));
            dt_out[8 * i + j] = -w[j] / gd;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Margins: how far each ray is from a decision boundary                      */
/* ------------------------------------------------------------------------- */

/* Distance between the line o + t d and the segment p + s (q - p), s in [0,1].
 * The squared distance is a convex quadratic in s once t is optimal, so the
 * minimum is at its stationary point when that lies inside, else at an end. */
static double line_seg_dist(vec o, vec d, vec p, vec q) {
    vec e = sub(q, p), w = sub(p, o);
    double a = dot(d, d), b = dot(d, e), c = dot(e, e), wd = dot(w, d), we = dot(w, e);
    double den = a * c - b * b;
    double cand[3] = {0.0, 1.0, 0.0};
    int nc = 2;
    if (den > 1e-30 * a * c) {
        cand[2] = (b * wd - a * we) / den;
        if (cand[2] > 0.0 && cand[2] < 1.0) nc = 3;
    }
    double best = INFINITY;
    for (int i = 0; i < nc; ++i) {
        vec x = add(w, scl(e, cand[i]));
        best = fmin(best, norm(sub(x, scl(d, dot(x, d) / a))));
    }
    return best;
}

static double rel_gap(double x, double y) { return fabs(x - y) / fmax(fabs(y), 0.05); }

/* Triangle margin on [a,b]: min over the winner's edges and every triangle the
 * line passes within reach of before the winner, of the distance from the ray
 * line to that triangle's boundary; plus relative gaps of the winner to a, b and
 * to the next hit, and of inside hits just outside [a,b] to a and b.
 * cond = |d . n_winner| (1 for a miss). */
static void tri_margin(const float* verts, const int32_t* tris, int64_t ntri, vec o, vec d, double a, double b,
                       double* m_out, double* cond_out, int32_t* win_out, double* twin_out) {
    double tw, uw, vw;
    int32_t w;
    closest_one(verts, tris, ntri, o, d, a, b, &tw, &w, &uw, &vw);
    double m = INFINITY, cond = 1.0;
    double tlim = w >= 0 ? tw : b;
    for (int64_t k = 0; k < ntri; ++k) {
        vec A = vert(verts, tris[3 * k]), B = vert(verts, tris[3 * k + 1]), C = vert(verts, tris[3 * k + 2]);
        vec nrm = cross(sub(B, A), sub(C, A));
        double den = dot(nrm, d);
        if (den == 0.0) continue;
        double tk = dot(nrm, sub(A, o)) / den;
        double t, u, v;
        int inside = mt_hit(o, d, A, B, C, &t, &u, &v);
        if (k == w) {
            double e = fmin(line_seg_dist(o, d, A, B), fmin(line_seg_dist(o, d, B, C), line_seg_dist(o, d, C, A)));
            m = fmin(m, fmin(e, fmin(rel_gap(tk, a), rel_gap(tk, b))));
            cond = fabs(den) / norm(nrm);
            continue;
        }
        if (inside) {
            if (tk >= a && tk <= b) m = fmin(m, rel_gap(tk, tw)); /* a later (or tied) hit */
            else m = fmin(m, fmin(rel_gap(tk, a), rel_gap(tk, b)));
        } else if (tk >= a - 1e-3 && tk <= tlim + 1e-3) {
            double e = fmin(line_seg_dist(o, d, A, B), fmin(line_seg_dist(o, d, B, C), line_seg_dist(o, d, C, A)));
            m = fmin(m, e);
        }
    }
    *m_out = m; *cond_out = cond; *win_out = w; *twin_out = tw;
}

/* DF margin on [a,b]: the smallest local minimum of g/h before the hit (or over
 * the whole clipped segment for a miss), |g(a')|/h when the segment starts at or
 * below zero, and the relative gap of a hit to the segment end.
 * cond = |g'(t*)| for a hit (1 for a miss). */
static void df_margin(const grid_t* G, vec o, vec d, double a, double b, double* m_out, double* cond_out,
                      double* thit_out) {
    double m = INFINITY, cond = 1.0;
    double thit = df_first_root(G, o, d, a, b);
    *thit_out = thit;
    if (!clip_box(G, o, d, &a, &b)) { *m_out = m; *cond_out = cond; return; }
    dda_t s;
    dda_init(G, o, d, a, &s);
    double t_in = a;
    double prev_slope = NAN;  /* derivative at the end of the previous cell */
    double tend = thit < INFINITY ? thit : b;
    for (;;) {
        int ax = dda_next_axis(&s);
        double t_out = s.tnext[ax] < b ? s.tnext[ax] : b;
        if (t_out < t_in) t_out = t_in;
        double k[4];
        cell_cubic(G, s.c, o, d, t_in, k);
        double S = t_out - t_in;
        double g0 = cub(k, 0.0), d0 = dcub(k, 0.0);
        if (t_in == a) {
            if (g0 <= 0.0) { m = fabs(g0) / G->h; break; }
            if (d0 >= 0.0) m = fmin(m, g0 / G->h);
        } else if (prev_slope <= 0.0 && d0 >= 0.0) {
            m = fmin(m, g0 / G->h); /* kink minimum at a cell face */
        }
        double r[2];
        int nr = crit_points(k, S, r);
        for (int i = 0; i < nr; ++i)
            if (t_in + r[i] < tend && 6.0 * k[3] * r[i] + 2.0 * k[2] >= 0.0) m = fmin(m, cub(k, r[i]) / G->h);
        if (t_out >= tend) {
            if (thit < INFINITY) {
                cond = fabs(dcub(k, thit - t_in));
                m = fmin(m, rel_gap(thit, b));
            } else if (dcub(k, S) <= 0.0) {
                m = fmin(m, cub(k, S) / G->h); /* still falling at the far end */
            }
            break;
        }
        prev_slope = dcub(k, S);
        s.c[ax] += s.step[ax];
        if (s.c[ax] < 0 || s.c[ax] > G->N - 2) break;
        t_in = t_out;
        s.tnext[ax] += s.tdelta[ax];
    }
    *m_out = m; *cond_out = cond;
}

/* Per-ray margin and conditioning of a query (mode as in oracle_query). */
void oracle_margin(const float* verts, const int32_t* tris, int64_t ntri,
                   const double* grid, int N, const float* grid4,
                   const float* rays, int64_t n, const float* tmin, const float* tmax_ray, float tmax_all,
                   float tau, float tau_end, int mode, double* margin_out, double* cond_out) {
    grid_t G = {grid, N, mk(grid4 ? grid4[0] : 0, grid4 ? grid4[1] : 0, grid4 ? grid4[2] : 0), grid4 ? grid4[3] : 1.0};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        vec o = ray_o(rays, n, i), d = ray_d(rays, n, i);
        float t0 = tmin ? tmin[i] : 0.0f;
        float tmax = tmax_ray ? fminf(tmax_ray[i], tmax_all) : tmax_all;
        double m = INFINITY, cnd = 1.0, mt, ct, tw, md, cd, td;
        int32_t w;
        if (!(t0 <= tmax)) { margin_out[i] = m; cond_out[i] = cnd; continue; }
        if (mode == 1) {
            tri_margin(verts, tris, ntri, o, d, t0, tmax, &m, &cnd, &w, &tw);
        } else if (mode == 2) {
            df_margin(&G, o, d, t0, tmax, &m, &cnd, &td);
        } else if (mode == 3) {
            /* any hit: the DF part decides alone when it has a root; otherwise
             * both triangle parts take part in the decision */
            double t1 = split_point(t0, tmax, tau, (float)G.h);
            double t2 = split_end(tmax, tau_end, (float)G.h, t1);
            int decided = 0;
            if (t2 > t1 || (tau == 0.0f && tau_end == 0.0f)) {
                df_margin(&G, o, d, t1, t2, &md, &cd, &td);
                m = md; cnd = cd;
                if (td < INFINITY) decided = 1;
            }
            if (!decided) {
                if (t1 > t0) { tri_margin(verts, tris, ntri, o, d, t0, t1, &mt, &ct, &w, &tw); m = fmin(m, mt); cnd = ct; }
                if ((double)tmax > t2) { tri_margin(verts, tris, ntri, o, d, t2, tmax, &mt, &ct, &w, &tw); m = fmin(m, mt); }
            }
        } else {
            double t1 = split_point(t0, tmax, tau, (float)G.h);
            int done = 0;
            if (t1 > t0) {
                tri_margin(verts, tris, ntri, o, d, t0, t1, &mt, &ct, &w, &tw);
                m = mt; cnd = ct;
                if (w >= 0) done = 1;
            }
            if (!done && (t1 < tmax || tau == 0.0f)) {
                df_margin(&G, o, d, t1, tmax, &md, &cd, &td);
                m = fmin(m, md);
                cnd = cd;
            }
        }
        margin_out[i] = m; cond_out[i] = cnd;
    }
}
