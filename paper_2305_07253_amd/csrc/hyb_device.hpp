// Device-side building blocks of the combined ray query (internal header).
//
// Everything here runs one ray per lane of a 64-wide CDNA wavefront:
//   - robust ray/box slab test (Ize, "Robust BVH ray traversal", JCGT 2013)
//   - watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013)
//   - closest-hit four-wide BVH traversal with a per-lane stack in LDS (+ rare spill)
//   - distance-field marching: conservative sphere-tracing steps g/L far from
//     the surface, exact first root of the per-cell trilinear cubic near it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

// Per-ray functions are host+device so that a CPU build can run the exact
// kernel logic (bounds-checked) against the oracle without a GPU.
#define HYB_HD __host__ __device__ __forceinline__

namespace hyb {

// Threads per block of the trace kernels: one wavefront.  A block keeps its
// slot and LDS until its last wavefront ends, and the march's wavefronts end
// at very different times, so with one wavefront per block none waits on
// another's long rays (measured against 4 and 2 wavefronts per block: 1-5%
// faster on every timed query, the same hits).
constexpr int kBlock = 64;
constexpr int kBatchBlock = 256;  // the persistent batch kernel's blocks: 4 wavefronts
constexpr int kXcds = 8;         // MI355X: 8 accelerator dies of 32 CUs, one L2 each
constexpr int kLdsDepth = 16;    // stack entries per lane held in LDS
constexpr int kStackDepth = 96;  // total stack entries per lane (LDS + spill); the BVH builder bounds the need
constexpr float kGamma3 = 3.0f * 5.9604645e-8f / (1.0f - 3.0f * 5.9604645e-8f);
constexpr float kBoxPad = 1.0f + 2.0f * kGamma3;

struct Counters {
    int nodes = 0, tris = 0, df = 0;
};

HYB_HD int bits_i(float v) { return __builtin_bit_cast(int, v); }

HYB_HD float pick3(float a, float b, float c, int k) { return k == 0 ? a : (k == 1 ? b : c); }

// a * b + c for a, b < 2^24 (low 32 bits, as the full-rate 24-bit multiply-add
// forms it; the 32-bit integer multiply is a quarter-rate instruction).
// Nested as mad24(a, b, mad24(c, d, e)), never as an operand of another
// multiply: only the low 24 bits of such an operand matter, so the compiler
// drops its masks and falls back to the quarter-rate form.
HYB_HD uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) { return (a & 0xffffffu) * (b & 0xffffffu) + c; }

// The dispatcher hands workgroup b of a launch to die b mod kXcds.  Returns
// the block this workgroup should process: the blocks are cut into groups of
// kXcds * run, and within a group each die gets `run` consecutive blocks, so
// neighbouring rays, which fetch the same cells and nodes, share one L2.  A
// short run keeps every die working across the whole launch (for work whose
// cost varies over the image); run = nb / kXcds gives each die one
// contiguous eighth.  The last, partial group keeps its order.  A bijection
// on [0, nb) for any run >= 1.
HYB_HD uint32_t xcd_block(uint32_t b, uint32_t nb, uint32_t run) {
    const uint32_t group = kXcds * run;
    if (b >= nb / group * group) return b;
    const uint32_t k = b / kXcds;  // this die's k-th block
    return (k / run * kXcds + b % kXcds) * run + k % run;
}

// Run length of the trace kernels: consecutive blocks (one wavefront each)
// a die takes at a time.  64 blocks (4,096 rays) on the GI rays: 3% faster
// than plain order at threshold 0, and faster than runs of 1,024 to 32,768
// rays (one contiguous eighth per die made the triangle-only query 4% slower,
// the dies finishing unevenly).  Grids whose kernel copy passes 128 MiB, half
// the MALL, take runs of 8,192 rays: on the 256^3 grid F32 3% and I8 6%
// faster at threshold 0 (F16 in its 128 MiB two-cell copy the same either
// way).
constexpr uint32_t kXcdRun = 64;
constexpr uint32_t kXcdRunLargeGrid = 128;

inline uint32_t xcd_run_for(int64_t copy_bytes) {
    return copy_bytes > (int64_t(128) << 20) ? kXcdRunLargeGrid : kXcdRun;
}

// ---------------------------------------------------------------------------
// triangle test
// ---------------------------------------------------------------------------

// Per-ray shear of the watertight test: the ray becomes the +z axis.
struct ShearRay {
    int kx, ky, kz;
    float sx, sy, sz;
};

HYB_HD ShearRay make_shear(float dx, float dy, float dz) {
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    ShearRay s;
    s.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    s.kx = s.kz == 2 ? 0 : s.kz + 1;
    s.ky = s.kx == 2 ? 0 : s.kx + 1;
    const float dkz = pick3(dx, dy, dz, s.kz);
    if (dkz < 0.0f) {
        int t = s.kx;
        s.kx = s.ky;
        s.ky = t;
    }
    s.sx = pick3(dx, dy, dz, s.kx) / dkz;
    s.sy = pick3(dx, dy, dz, s.ky) / dkz;
    s.sz = 1.0f / dkz;
    return s;
}

// Watertight test of one triangle against the ray on [t_lo, t_hi].  On a hit
// returns true with t and barycentrics (u: weight of v1, v: weight of v2).
// Contraction into FMA is disabled so that the edge functions of an edge shared
// by two triangles are exact negations of each other.
HYB_HD bool tri_hit(const ShearRay& s, float ox, float oy, float oz, float4 v0, float4 v1,
                                        float4 v2, float t_lo, float t_hi, float& t, float& u, float& v) {
#pragma clang fp contract(off)
    const float Ax0 = v0.x - ox, Ay0 = v0.y - oy, Az0 = v0.z - oz;
    const float Bx0 = v1.x - ox, By0 = v1.y - oy, Bz0 = v1.z - oz;
    const float Cx0 = v2.x - ox, Cy0 = v2.y - oy, Cz0 = v2.z - oz;
    const float Akz = pick3(Ax0, Ay0, Az0, s.kz), Bkz = pick3(Bx0, By0, Bz0, s.kz), Ckz = pick3(Cx0, Cy0, Cz0, s.kz);
    const float Ax = pick3(Ax0, Ay0, Az0, s.kx) - s.sx * Akz;
    const float Ay = pick3(Ax0, Ay0, Az0, s.ky) - s.sy * Akz;
    const float Bx = pick3(Bx0, By0, Bz0, s.kx) - s.sx * Bkz;
    const float By = pick3(Bx0, By0, Bz0, s.ky) - s.sy * Bkz;
    const float Cx = pick3(Cx0, Cy0, Cz0, s.kx) - s.sx * Ckz;
    const float Cy = pick3(Cx0, Cy0, Cz0, s.ky) - s.sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        // exact signs from double products of the FP32 sheared coordinates
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = U + V + W;
    if (det == 0.0f) return false;
    const float T = U * (s.sz * Akz) + V * (s.sz * Bkz) + W * (s.sz * Ckz);
    const float inv = 1.0f / det;
    const float tt = T * inv;
    if (!(tt >= t_lo && tt <= t_hi)) return false;
    t = tt;
    u = V * inv;
    v = W * inv;
    return true;
}

// ---------------------------------------------------------------------------
// BVH traversal
// ---------------------------------------------------------------------------

struct BoxRay {
    float ox, oy, oz, ix, iy, iz;
};

HYB_HD float safe_inv(float d) {
    // a zero component becomes a tiny value of the same sign: the slab then
    // spans +-huge instead of producing 0 * inf = NaN
    return 1.0f / (fabsf(d) > 1e-30f ? d : copysignf(1e-30f, d));
}

// 1 / d per component, formed once per ray for the slab tests of both
// techniques (the BVH's boxes, the distance field's grid box).
struct RayInv {
    float x, y, z;
};

HYB_HD RayInv ray_inv(float dx, float dy, float dz) { return {safe_inv(dx), safe_inv(dy), safe_inv(dz)}; }

// Conservative slab test: tn/tf of the box clipped to [lo, hi]; hit iff tn <= tf.
HYB_HD void box_clip(const BoxRay& r, float lx, float hx, float ly, float hy, float lz, float hz,
                                         float seg_lo, float seg_hi, float& tn, float& tf) {
    const float t0x = (lx - r.ox) * r.ix, t1x = (hx - r.ox) * r.ix;
    const float t0y = (ly - r.oy) * r.iy, t1y = (hy - r.oy) * r.iy;
    const float t0z = (lz - r.oz) * r.iz, t1z = (hz - r.oz) * r.iz;
    tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), seg_lo));
    tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), seg_hi)) * kBoxPad;
}

struct Hit {
    float t;
    int prim;
    float u, v;
};

// Orders two (key, ref) pairs by key.
HYB_HD void order2(float& ka, int& ra, float& kb, int& rb) {
    const bool sw = kb < ka;
    const float k = sw ? kb : ka;
    const int r = sw ? rb : ra;
    kb = sw ? ka : kb;
    rb = sw ? ra : rb;
    ka = k;
    ra = r;
}

// Closest triangle hit on [seg_lo, seg_hi] (both inclusive) through the
// four-wide BVH (nodes4 layout, 128-byte nodes).  Equal t goes to the smallest
// original triangle id, independent of traversal order.  With ANY the
// traversal stops at the first intersection it finds (any-hit).  With `sort`
// the children a node's ray hits are visited nearest first (the nearest is
// entered, the others are pushed farthest first), which lets a closest hit
// prune farther boxes early on long segments; without it they go in slot
// order, which costs fewer instructions and gives the same hit (the order
// only changes which boxes a closer hit prunes, never the result).  `stack`
// points at this lane's first LDS slot; consecutive entries are `stride` ints
// apart (one slot per thread of the block, no bank conflicts); entries beyond
// LDS go to a private spill area.
template <bool COUNT, bool ANY = false, int LDS = kLdsDepth>
HYB_HD Hit bvh_closest(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                       float ox, float oy, float oz, float dx, float dy, float dz, const RayInv& inv,
                       float seg_lo, float seg_hi, int* stack, int stride, Counters& cnt, int start = 0,
                       bool sort = true) {
    Hit best;
    best.t = seg_hi;
    best.prim = -1;
    best.u = 0.0f;
    best.v = 0.0f;
    const BoxRay br = {ox, oy, oz, inv.x, inv.y, inv.z};
    const ShearRay sr = make_shear(dx, dy, dz);
    static_assert(LDS > 0 && LDS < kStackDepth, "LDS part of the stack out of range");
    int spill[kStackDepth - LDS];
    int sp = 0;
    int ref = start;  // the root, or a subtree holding every triangle the segment can reach
    for (;;) {
        if (ref >= 0) {
            const float4* n = nodes + 8 * (int64_t)ref;
            const float4 lx = n[0], hx = n[1], ly = n[2], hy = n[3], lz = n[4], hz = n[5], rf = n[6];
            if (COUNT) cnt.nodes++;
            const float hi = best.t * kBoxPad;
            constexpr float kNone = __builtin_inff();
            float tn, tf;
            box_clip(br, lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, seg_lo, hi, tn, tf);
            float k0 = tn <= tf ? tn : kNone;
            box_clip(br, lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, seg_lo, hi, tn, tf);
            float k1 = tn <= tf ? tn : kNone;
            box_clip(br, lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, seg_lo, hi, tn, tf);
            float k2 = tn <= tf ? tn : kNone;
            box_clip(br, lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, seg_lo, hi, tn, tf);
            float k3 = tn <= tf ? tn : kNone;
            int r0 = bits_i(rf.x), r1 = bits_i(rf.y), r2 = bits_i(rf.z), r3 = bits_i(rf.w);
            if (sort) {
                // sorting network, nearest first; misses (+inf) sink to the end
                order2(k0, r0, k1, r1);
                order2(k2, r2, k3, r3);
                order2(k0, r0, k2, r2);
                order2(k1, r1, k3, r3);
                order2(k1, r1, k2, r2);
                if (k0 < kNone) {
                    const int push[3] = {r3, r2, r1};
                    const bool take[3] = {k3 < kNone, k2 < kNone, k1 < kNone};
                    for (int c = 0; c < 3; ++c) {
                        if (!take[c]) continue;
                        if (sp < LDS) stack[sp * stride] = push[c];
                        else spill[sp - LDS] = push[c];
                        ++sp;
                    }
                    ref = r0;
                    continue;
                }
            } else {
                // slot order: enter the first child hit, push the others
                const int rr[4] = {r3, r2, r1, r0};
                const bool hh[4] = {k3 < kNone, k2 < kNone, k1 < kNone, k0 < kNone};
                int next = 0;
                bool have = false;
                for (int c = 0; c < 4; ++c) {
                    if (!hh[c]) continue;
                    if (have) {
                        if (sp < LDS) stack[sp * stride] = next;
                        else spill[sp - LDS] = next;
                        ++sp;
                    }
                    next = rr[c];
                    have = true;
                }
                if (have) {
                    ref = next;
                    continue;
                }
            }
        } else {
            const int info = ~ref;
            const int first = info >> 3, count = info & 7;
            for (int k = 0; k < count; ++k) {
                const float4* tp = tris + 3 * (int64_t)(first + k);
                const float4 v0 = tp[0], v1 = tp[1], v2 = tp[2];
                if (COUNT) cnt.tris++;
                float t, u, v;
                if (tri_hit(sr, ox, oy, oz, v0, v1, v2, seg_lo, best.t, t, u, v)) {
                    const int id = bits_i(v0.w);
                    if (t < best.t || best.prim < 0 || id < best.prim) {
                        best.t = t;
                        best.prim = id;
                        best.u = u;
                        best.v = v;
                    }
                    if (ANY) return best;
                }
            }
        }
        if (sp == 0) break;
        --sp;
        ref = sp < LDS ? stack[sp * stride] : spill[sp - LDS];
    }
    if (best.prim < 0) best.t = __builtin_inff();
    return best;
}

// ---------------------------------------------------------------------------
// distance field
// ---------------------------------------------------------------------------

// Storage format and brick layout of the kernels' copy: kF16B2 is F16 in the
// bricks of 2^3 cells that FP32 uses, for grids whose one-cell F16 copy would
// crowd the 256 MB MALL (f16_layout).
enum SdfFormat : int { kF32 = 0, kF16 = 1, kI8 = 2, kF16B2 = 3 };
constexpr int kScaleBlock = 8;  // I8: one scale per block of 8^3 cells

// I8 scale blocks per axis of an n^3 grid: ceil((n - 1) / 8) blocks of cells.
HYB_HD int i8_blocks(int n) { return (n - 1 + kScaleBlock - 1) / kScaleBlock; }

struct Grid {
    const void* __restrict__ v;  // samples in the bricked layout Brick<FMT> (float, _Float16 or int8_t)
    int n;                       // samples per axis
    float lo_x, lo_y, lo_z, h, inv_h;
    float inv_l;    // 1 / Lipschitz bound of the interpolant (slightly reduced)
    float two_e;    // 2 x (interpolation error bound + storage error), +inf if uncertified
    float slope_x, slope_y, slope_z;  // bounds of |df/dx|, |df/dy|, |df/dz| over the grid
    double inv_hd;  // 1 / h in FP64
};

// The 8 corner samples of cell (i, j, k), dequantized to FP32:
// f[dx + 2 dy + 4 dz] = sample(i + dx, j + dy, k + dz).
// Kernel-side layout of the samples: the cells are grouped into bricks of
// C^3 cells, and each brick stores all (C + 1)^3 nodes of its cells (the faces
// it shares with neighbouring bricks are duplicated), x fastest inside a
// brick, bricks x fastest.  The 8 corners of any cell then lie in one brick at
// fixed offsets from one address: a fetch is a few wide loads with immediate
// offsets inside one or two cache lines, and the nodes around a ray share
// lines.  C per format (fastest measured on the GI-shaped workload):
//   F32: C = 2, the 27 samples of a brick padded to 32 (4x the n^3 samples):
//        each brick is one 128-byte cache line, so a fetch touches exactly one
//        (unpadded, 43% of the 56-byte fetches straddled two)
//   F16: C = 1, the 8 corners of each cell contiguous (16 B, one load)
//   I8: C = 1, the 8 codes of each cell, then the scale of the cell's block
//        (a float in slots 8-11): 12 B, one load per fetch with no table
//        lookup; the block's scale repeats in each of its cells (1.5x the
//        bytes of codes alone, three quarters of one-cell F16)
//   F16 of large grids (kF16B2): C = 2, 27 halves padded to 32 (64 B): half
//        the footprint of one-cell bricks, eight 2-byte loads per fetch
// Slots of nodes beyond the grid are padding and never read.
template <int FMT>
struct Brick {
    static constexpr int kCells = FMT == kF32 || FMT == kF16B2 ? 2 : 1;
    static constexpr int kSide = kCells + 1;
    static constexpr int kNodes = kSide * kSide * kSide;
    // slots per brick: padding at the end (two-cell bricks), the scale (I8)
    static constexpr int kStride = kCells == 2 ? 32 : (FMT == kI8 ? kNodes + 4 : kNodes);

    HYB_HD static int per_axis(int n) { return (n - 1 + kCells - 1) / kCells; }

    HYB_HD static int64_t storage(int n) {
        const int64_t b = per_axis(n);
        return b * b * b * kStride;
    }

    // Storage slot of corner 0 (the node (i, j, k)) of cell (i, j, k); cells
    // are never negative.  With n <= 1024 a grid has fewer than 2^30 bricks
    // and nb^2 < 2^20, so the brick index fits 32 bits; only the slot (brick
    // times a power of two) needs 64 bits.  One-cell bricks form it with two
    // 24-bit multiply-adds (I8 queries 3-6% faster); for two-cell bricks the
    // compiler's own form measured faster in the combined kernel.
    HYB_HD static int64_t cell_slot(int i, int j, int k, int nbk) {
        const uint32_t ui = (uint32_t)i, uj = (uint32_t)j, uk = (uint32_t)k, nb = (uint32_t)nbk;
        const uint32_t bi = ui / kCells, bj = uj / kCells, bk = uk / kCells;
        const uint32_t r = (ui - bi * kCells) + kSide * ((uj - bj * kCells) + kSide * (uk - bk * kCells));
        const uint32_t brick = kCells == 1 ? mad24(bk, nb * nb, mad24(bj, nb, bi)) : (bk * nb + bj) * nb + bi;
        return (int64_t)((uint64_t)brick * (uint32_t)kStride + r);
    }

    // The node stored in slot s; false for a padding slot.
    HYB_HD static bool slot_node(int64_t s, int n, int& i, int& j, int& k) {
        const int nbk = per_axis(n);
        const int64_t b = s / kStride;
        const int r = (int)(s - b * kStride);
        if (r >= kNodes) {
            i = j = k = 0;
            return false;
        }
        const int bi = (int)(b % nbk), bj = (int)((b / nbk) % nbk), bk = (int)(b / ((int64_t)nbk * nbk));
        i = bi * kCells + r % kSide;
        j = bj * kCells + (r / kSide) % kSide;
        k = bk * kCells + r / (kSide * kSide);
        return i < n && j < n && k < n;
    }
};

// Slots of the bricked storage of an n^3 grid in format fmt (runtime format).
inline int64_t brick_storage(int fmt, int n) {
    switch (fmt) {
        case kF32: return Brick<kF32>::storage(n);
        case kF16: return Brick<kF16>::storage(n);
        case kF16B2: return Brick<kF16B2>::storage(n);
        default: return Brick<kI8>::storage(n);
    }
}

// Kernel layout of an F16 grid of n^3 samples: two-cell bricks once the
// one-cell copy ((n - 1)^3 cells of 16 B) passes 128 MiB, half the MALL.
// Measured: at 128^3 (33 MB) one-cell bricks are 6% faster on the GI rays, at
// 256^3 (265 MB) two-cell bricks 20% faster.
inline int f16_layout(int n) {
    const int64_t c = n - 1;
    return c * c * c * 16 > (int64_t(128) << 20) ? kF16B2 : kF16;
}

// The 8 samples of cell (i, j, k), corner c = (i + (c & 1), j + (c >> 1 & 1), k + (c >> 2)),
// as f[c] times the returned factor: 1, except for I8 (f the integer codes,
// the factor their block's scale, which the caller applies after
// interpolating: a power of two, it changes no rounding in between).
template <int FMT>
HYB_HD float corners(const Grid& g, int i, int j, int k, float f[8]) {
    using B = Brick<FMT>;
    constexpr int S = B::kSide, S2 = B::kSide * B::kSide;
    constexpr int off[8] = {0, 1, S, S + 1, S2, S2 + 1, S2 + S, S2 + S + 1};
    const int64_t slot = B::cell_slot(i, j, k, B::per_axis(g.n));
    if constexpr (FMT == kF32) {
        const float* p = static_cast<const float*>(g.v) + slot;
        for (int c = 0; c < 8; ++c) f[c] = p[off[c]];
        return 1.0f;
    } else if constexpr (FMT == kF16 || FMT == kF16B2) {
        const _Float16* p = static_cast<const _Float16*>(g.v) + slot;
        for (int c = 0; c < 8; ++c) f[c] = (float)p[off[c]];
        return 1.0f;
    } else {
        // the 8 codes, then the scale of the cell's block: 12 bytes at a
        // 4-aligned address (slot = 12 x brick), one load
        struct Cell {
            int8_t q[8];
            float s;
        };
        Cell c8;
        __builtin_memcpy(&c8, __builtin_assume_aligned(static_cast<const int8_t*>(g.v) + slot, 4), sizeof(Cell));
        for (int c = 0; c < 8; ++c) f[c] = (float)c8.q[off[c]];
        return c8.s;
    }
}

// Trilinear interpolation inside one cell at in-cell fractions (x, y, z),
// keeping the differences it forms: with them the cubic along a ray through
// the point (cell_cubic) costs a few more operations.
struct CellLerp {
    float val;                // the interpolant at (x, y, z)
    float dx0, dx1, dx2, dx3; // f1 - f0, f3 - f2, f5 - f4, f7 - f6: x-differences of the 4 x-edges
    float dy0, dy1;           // y-differences of the x-lerps at z = 0 and z = 1
    float dz;                 // z-difference of the y-lerps: df/dz at the point
};

HYB_HD CellLerp lerp_cell(const float f[8], float x, float y, float z) {
    CellLerp L;
    L.dx0 = f[1] - f[0];
    L.dx1 = f[3] - f[2];
    L.dx2 = f[5] - f[4];
    L.dx3 = f[7] - f[6];
    const float a = f[0] + x * L.dx0, b = f[2] + x * L.dx1;
    const float c = f[4] + x * L.dx2, d = f[6] + x * L.dx3;
    L.dy0 = b - a;
    L.dy1 = d - c;
    const float e = a + y * L.dy0, q = c + y * L.dy1;
    L.dz = q - e;
    L.val = e + z * L.dz;
    return L;
}

// Cubic g(s) = k0 + k1 s + k2 s^2 + k3 s^3 of the trilinear interpolant along
// (x + qx s, y + qy s, z + qz s) inside one cell.  A trilinear function equals
// its Taylor expansion about any point, f(p + u) = f + fx ux + fy uy + fz uz +
// fxy ux uy + fxz ux uz + fyz uy uz + fxyz ux uy uz, and every partial
// derivative at p is a lerp of differences formed by lerp_cell.
HYB_HD void cell_cubic(const CellLerp& L, float y, float z, float qx, float qy, float qz, float k[4]) {
    const float hx0 = L.dx1 - L.dx0, hx1 = L.dx3 - L.dx2;     // fxy at z = 0 and z = 1
    const float gx0 = L.dx0 + y * hx0, gx1 = L.dx2 + y * hx1; // fx at z = 0 and z = 1
    const float fxz = gx1 - gx0, fyz = L.dy1 - L.dy0, fxyz = hx1 - hx0;
    const float fx = gx0 + z * fxz, fy = L.dy0 + z * fyz, fxy = hx0 + z * fxyz;
    k[0] = L.val;
    k[1] = fx * qx + fy * qy + L.dz * qz;
    k[2] = fxy * (qx * qy) + fxz * (qx * qz) + fyz * (qy * qz);
    k[3] = fxyz * (qx * qy) * qz;
}

HYB_HD float cubic_at(const float k[4], float s) { return fmaf(fmaf(fmaf(k[3], s, k[2]), s, k[1]), s, k[0]); }

// Approximate reciprocal (about 1 ulp) where it only places a guess inside a
// bracket; exact division in the CPU build of these functions.
HYB_HD float approx_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

HYB_HD float cubic_slope(const float k[4], float s) { return fmaf(fmaf(3.0f * k[3], s, 2.0f * k[2]), s, k[1]); }

// Root of the cubic inside (a, b] where g(a) > 0 >= g(b) and g is monotone
// there: Newton from the secant guess, any step leaving the bracket replaced by
// bisection, until the step or the bracket is below `tol`.
HYB_HD float refine_root(const float k[4], float a, float b, float tol) {
    const float fa = cubic_at(k, a), fb = cubic_at(k, b);
    float x = b - fb * (b - a) * approx_rcp(fb - fa);
    if (!(x > a && x <= b)) x = 0.5f * (a + b);
    for (int it = 0; it < 16; ++it) {
        const float fx = cubic_at(k, x);
        if (fx <= 0.0f) b = x;
        else a = x;
        if (b - a <= tol) return b;
        float nx = x - fx * approx_rcp(cubic_slope(k, x));
        if (fabsf(nx - x) <= tol) return fminf(fmaxf(nx, a), b);
        if (!(nx > a && nx <= b)) nx = 0.5f * (a + b);
        x = nx;
    }
    return b;
}

// Exact rejection: on [0, S] the cubic is a blend of its four Bernstein
// coefficients, so if they are all positive g stays positive.  True when the
// span may hold a root.
HYB_HD bool cubic_may_vanish(const float k[4], float S) {
    if (!(S > 0.0f)) return false;
    const float k1 = k[1] * S, k2 = k[2] * S * S, k3 = k[3] * S * S * S;
    const float b1 = fmaf(k1, 1.0f / 3.0f, k[0]);
    const float b2 = fmaf(k2, 1.0f / 3.0f, fmaf(k1, 2.0f / 3.0f, k[0]));
    const float b3 = k[0] + k1 + k2 + k3;
    return !(b1 > 0.0f && b2 > 0.0f && b3 > 0.0f);
}

// First s in (0, S] with g(s) <= 0 given g(0) > 0, or -1: g is split into
// monotone pieces at the roots of g'; the first piece ending at or below zero
// holds the first root.
HYB_HD float cubic_first_root(const float k[4], float S) {
    float r0 = S, r1 = S;
    const float A = 3.0f * k[3], B = 2.0f * k[2], C = k[1];
    if (A != 0.0f) {
        const float disc = B * B - 4.0f * A * C;
        if (disc >= 0.0f) {
            const float q = -0.5f * (B + copysignf(sqrtf(disc), B));
            float a = q * approx_rcp(A), b = q != 0.0f ? C * approx_rcp(q) : S;
            if (a > b) {
                const float t = a;
                a = b;
                b = t;
            }
            r0 = (a > 0.0f && a < S) ? a : S;
            r1 = (b > 0.0f && b < S) ? b : S;
            if (r0 == S) r0 = r1;
        }
    } else if (B != 0.0f) {
        const float a = -C * approx_rcp(B);
        r0 = r1 = (a > 0.0f && a < S) ? a : S;
    }
    float lo = 0.0f, hi = S;
    if (cubic_at(k, r0) <= 0.0f) hi = r0;
    else if (r1 > r0 && cubic_at(k, r1) <= 0.0f) {
        lo = r0;
        hi = r1;
    } else if (cubic_at(k, S) <= 0.0f) {
        lo = r1;
    } else {
        return -1.0f;
    }
    return refine_root(k, lo, hi, 1e-6f * S);
}

// Marching state of one ray (see df_first_root).
struct DfRay {
    double px, py, pz;  // origin in cell units, (o - lo) / h
    double qx, qy, qz;  // direction in cell units, d / h
    float qxf, qyf, qzf;
    float inv_l;        // sphere-step factor: 1 / bound of |d/dt f(o + t d)|
    // time to the cell's exit face along each axis from in-cell fraction f is
    // f m + e: with c the time to cross one cell, (1 - f) c moving up (m = -c,
    // e = c), f c moving down (m = c, e = 0); c = inf when not moving
    float mx, my, mz, ex, ey, ez;
    float t, b;         // current position and segment end
    float cover;        // [start, cover] is verified free of roots
    int ci, cj, ck;     // current cell while walking
    bool walk;
    bool relax;         // the next sphere step may be over-relaxed
    bool walk_only;     // cell steps only (the bounded fall-back of df_first_root)
    // a cell span [t, t + span] whose cubic k may vanish, left for df_resolve
    float k[4], span, t_exit;
    int axis;           // exit face of that cell: 0, 1, 2
};

enum DfStatus : int { kDfContinue = 0, kDfHit = 1, kDfMiss = 2, kDfSolve = 3 };

// Moves to the neighbouring cell across the exit face `axis` at t_exit.
HYB_HD int df_advance(const Grid& g, DfRay& r, int axis, float t_exit) {
    if (t_exit >= r.b) return kDfMiss;
    r.cover = t_exit;  // the cell's span was checked
    if (axis == 0) r.ci += r.qxf > 0.0f ? 1 : -1;
    else if (axis == 1) r.cj += r.qyf > 0.0f ? 1 : -1;
    else r.ck += r.qzf > 0.0f ? 1 : -1;
    const int nm2 = g.n - 2;
    if (r.ci < 0 || r.cj < 0 || r.ck < 0 || r.ci > nm2 || r.cj > nm2 || r.ck > nm2) return kDfMiss;
    r.t = t_exit;
    return kDfContinue;
}

// Clips [a, b] to the grid box and prepares the marching state; false when the
// segment misses the box.
HYB_HD bool df_init(const Grid& g, float ox, float oy, float oz, float dx, float dy, float dz, const RayInv& inv,
                    float a, float b, DfRay& r) {
    const float ext = (float)(g.n - 1) * g.h;
    const float ix = inv.x, iy = inv.y, iz = inv.z;
    const float t0x = (g.lo_x - ox) * ix, t1x = (g.lo_x + ext - ox) * ix;
    const float t0y = (g.lo_y - oy) * iy, t1y = (g.lo_y + ext - oy) * iy;
    const float t0z = (g.lo_z - oz) * iz, t1z = (g.lo_z + ext - oz) * iz;
    a = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), a));
    b = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), b));
    if (!(a <= b)) return false;
    const double ih = g.inv_hd;
    r.px = ((double)ox - (double)g.lo_x) * ih;
    r.py = ((double)oy - (double)g.lo_y) * ih;
    r.pz = ((double)oz - (double)g.lo_z) * ih;
    r.qx = (double)dx * ih;
    r.qy = (double)dy * ih;
    r.qz = (double)dz * ih;
    r.qxf = (float)r.qx;
    r.qyf = (float)r.qy;
    r.qzf = (float)r.qz;
    // these only size the cell spans of the walk (a span a few ulps long or
    // short moves a cell boundary by as much, on a continuous interpolant)
    const float cx = r.qxf != 0.0f ? approx_rcp(fabsf(r.qxf)) : __builtin_inff();
    const float cy = r.qyf != 0.0f ? approx_rcp(fabsf(r.qyf)) : __builtin_inff();
    const float cz = r.qzf != 0.0f ? approx_rcp(fabsf(r.qzf)) : __builtin_inff();
    r.mx = r.qxf > 0.0f ? -cx : cx;
    r.my = r.qyf > 0.0f ? -cy : cy;
    r.mz = r.qzf > 0.0f ? -cz : cz;
    r.ex = r.qxf > 0.0f ? cx : 0.0f;
    r.ey = r.qyf > 0.0f ? cy : 0.0f;
    r.ez = r.qzf > 0.0f ? cz : 0.0f;
    // the interpolant changes along the ray by at most sum |df/dx_i| |d_i| per
    // unit t (at least 1 keeps steps finite on flat fields), often well below
    // the gradient-norm bound L (1.5 against sqrt(3) for an exact distance
    // field and a random direction); rounded down 2e-6 to stay a bound
    const float ld = fmaf(g.slope_x, fabsf(dx), fmaf(g.slope_y, fabsf(dy), g.slope_z * fabsf(dz)));
    r.inv_l = fmaxf(g.inv_l, approx_rcp(fmaxf(ld, 1.0f)) * (1.0f - 2e-6f));
    r.t = a;
    r.b = b;
    r.cover = a;
    r.ci = r.cj = r.ck = 0;
    r.walk = false;
    r.relax = false;
    r.walk_only = false;
    return true;
}

// Over-relaxed sphere steps (Keinert et al., "Enhanced Sphere Tracing", 2014):
// a step of kOverRelax times the certified radius, kept only when the new
// point's own certified interval reaches back to the end of the verified part
// of the ray; otherwise the march returns there and steps plainly.  On the
// GI-shaped workload this saves a ninth of the iterations (1.3 measured best
// among 1.15 to 1.9).
constexpr float kOverRelax = 1.3f;

// Smallest of the samples' bit patterns read as signed integers: <= 0 exactly
// when some sample is <= 0 (-0 included), for samples that are not NaN.
HYB_HD int min_bits(const float f[8]) {
    int m = __builtin_bit_cast(int, f[0]);
    for (int c = 1; c < 8; ++c) m = min(m, __builtin_bit_cast(int, f[c]));
    return m;
}

HYB_HD float exit_span_of(float ex, float ey, float ez) { return fmaxf(fminf(fminf(ex, ey), ez), 0.0f); }

HYB_HD int exit_axis_of(float ex, float ey, float ez) { return (ex <= ey && ex <= ez) ? 0 : (ey <= ez ? 1 : 2); }

// The cubic k of the interpolant along the ray from r.t inside the cell
// (the lerp of its samples f, times their factor s, see corners), and the
// length of the span it covers, up to the cell's exit or the segment end.
HYB_HD float span_cubic(const CellLerp& L, float s, float fy, float fz, const DfRay& r, float t_exit, float k[4]) {
    cell_cubic(L, fy, fz, r.qxf, r.qyf, r.qzf, k);
    for (int m = 0; m < 4; ++m) k[m] *= s;
    return fminf(t_exit, r.b) - r.t;
}

// One iteration of the march: fetch the 8 corners of one cell, then either a
// sphere step or a cell step (see df_first_root).  On kDfHit the hit is r.t;
// kDfSolve leaves a cell span that may hold the first root for df_resolve.
template <int FMT, bool COUNT>
HYB_HD int df_step(const Grid& g, DfRay& r, Counters& cnt) {
    const int nm2 = g.n - 2;
    const double X = fma((double)r.t, r.qx, r.px), Y = fma((double)r.t, r.qy, r.py), Z = fma((double)r.t, r.qz, r.pz);
    if (!r.walk) {
        r.ci = min(max((int)X, 0), nm2);
        r.cj = min(max((int)Y, 0), nm2);
        r.ck = min(max((int)Z, 0), nm2);
    }
    const float fx = (float)(X - r.ci), fy = (float)(Y - r.cj), fz = (float)(Z - r.ck);
    float f[8];
    const float s = corners<FMT>(g, r.ci, r.cj, r.ck, f);
    if (COUNT) cnt.df++;
    const CellLerp L = lerp_cell(f, fx, fy, fz);
    const float val = L.val * s;
    // no root within `safe` of this point (0 at or below the surface: both
    // bounds are then <= 0)
    const float safe = fmaxf(fmaxf(val * r.inv_l, val - g.two_e), 0.0f);
    if (r.t - safe > r.cover) {
        // an over-relaxed step left (cover, t - safe) unchecked: go back
        r.t = r.cover;
        r.walk = false;
        r.relax = false;
        return kDfContinue;
    }
    if (val <= 0.0f) return kDfHit;
    // span of the ray inside the current cell, from the in-cell fractions
    const float ex = fmaf(fx, r.mx, r.ex);
    const float ey = fmaf(fy, r.my, r.ey);
    const float ez = fmaf(fz, r.mz, r.ez);
    const float exit_span = exit_span_of(ex, ey, ez);
    // A sphere step far from the surface, unless it would be shorter than half
    // a cell (on a grid whose bound L is inflated, one extreme sample anywhere
    // makes every step short, and the exact cell step is longer; for any grid
    // with L < 2, g > h already gives safe > h / 2); and near the surface
    // whenever the certified distance already passes the cell's exit, which
    // covers the cell step's span and more.  Either kind moves the ray at
    // least half a cell or into the next cell.
    if (((val > g.h && safe >= 0.5f * g.h) || safe > exit_span) && !r.walk_only) {
        r.walk = false;
        r.cover = r.t + safe;
        r.t += r.relax ? kOverRelax * safe : safe;
        r.relax = true;
        if (r.t > r.b) {
            if (r.cover >= r.b) return kDfMiss;
            r.t = r.b;
        }
        return kDfContinue;
    }
    r.walk = true;
    const float t_exit = r.t + exit_span;
    const int axis = exit_axis_of(ex, ey, ez);
    if (min_bits(f) <= 0) {
        // some corner at or below zero: the cell's cubic along the ray
        r.span = span_cubic(L, s, fy, fz, r, t_exit, r.k);
        if (cubic_may_vanish(r.k, r.span)) {
            r.t_exit = t_exit;
            r.axis = axis;
            return kDfSolve;
        }
    }
    return df_advance(g, r, axis, t_exit);
}

// Finishes a kDfSolve: the exact first root of the cell's cubic on its span,
// else on to the next cell.
//
// REFORM: the span's cubic, its end and exit face are formed here again from
// r.t and the cell (df_step changed neither) by the functions df_step used
// (the F32 / I8 agreement on samples every format stores exactly checks that
// they give the same numbers); df_step's own copies are then never read, and
// the march no longer holds them.  A lane that stops for a
// solve keeps those seven values in registers while the rest of its
// wavefront marches on; formed again, they cost one more fetch of the cell
// once the wavefront's march has ended, by when its lines may have left the
// caches.  The combined I8 kernel then fits seven wavefronts per SIMD
// instead of six (3-4% faster at threshold 1); kernels that already fit
// seven or more lost more to the fetch than they gained.
template <int FMT, bool REFORM>
HYB_HD int df_resolve(const Grid& g, DfRay& r) {
    if constexpr (REFORM) {
        const double X = fma((double)r.t, r.qx, r.px), Y = fma((double)r.t, r.qy, r.py),
                     Z = fma((double)r.t, r.qz, r.pz);
        const float fx = (float)(X - r.ci), fy = (float)(Y - r.cj), fz = (float)(Z - r.ck);
        float f[8];
        const float s = corners<FMT>(g, r.ci, r.cj, r.ck, f);
        const CellLerp L = lerp_cell(f, fx, fy, fz);
        const float ex = fmaf(fx, r.mx, r.ex);
        const float ey = fmaf(fy, r.my, r.ey);
        const float ez = fmaf(fz, r.mz, r.ez);
        r.t_exit = r.t + exit_span_of(ex, ey, ez);
        r.axis = exit_axis_of(ex, ey, ez);
        r.span = span_cubic(L, s, fy, fz, r, r.t_exit, r.k);
    }
    const float s = cubic_first_root(r.k, r.span);
    if (s >= 0.0f) {
        r.t += s;
        return kDfHit;
    }
    return df_advance(g, r, r.axis, r.t_exit);
}

// Iterations of the mixed march before the walk-only fall-back: sphere steps
// are at least h / 2 long (an over-relaxed step the next iteration takes
// back is followed by a plain one), cell steps enter a new cell along the
// ray, and the clipped segment is at most sqrt(3) (n - 1) h long, so this is
// not reached in practice; it only has to keep the march finite.  (A host
// build of these functions may define a smaller budget to exercise the
// fall-back.)
#ifndef HYB_DF_MIXED_STEPS
#define HYB_DF_MIXED_STEPS(n) (16 * (n) + 64)
#endif
HYB_HD int df_max_steps(const Grid& g) { return HYB_DF_MIXED_STEPS(g.n); }

// Iterations of the walk-only fall-back: every iteration either ends the
// march or moves one of the three cell indices one step in the direction of
// the ray, and each index stays in [0, n - 2].
HYB_HD int df_max_walk(const Grid& g) { return 3 * g.n; }

// First t in [a, b] (clipped to the grid box) where the trilinear interpolant
// of the samples is <= 0, or +inf.
//
// Every iteration fetches the 8 corners of one cell and then takes one of two
// steps, so lanes of a wavefront in different phases still execute the same
// instruction stream:
//   sphere step  g > h: advance by a distance the interpolant cannot cross,
//                max(g / L_d, g - two_e) with L_d the ray's own slope bound
//                (df_init; the second bound only for grids that certify
//                1-Lipschitz samples, two_e = 2 (sqrt(3)/2 h + q)), times
//                kOverRelax after a plain step;
//   cell step    near the surface: the ray's span inside the current cell; a
//                cell whose 8 corners are all positive holds no root (the
//                interpolant is a convex blend of them), otherwise the exact
//                first root of the cell's cubic; then the next cell in DDA order.
// The ray's position in cell units, X(t) = (o - lo)/h + t d/h, is formed in
// FP64 (on MI355X an FP64 FMA issues at the rate of an unpacked FP32 one) so
// the in-cell fraction keeps full FP32 precision tens of cells from the
// origin.
template <int FMT, bool COUNT, bool REFORM = false>
HYB_HD float df_first_root(const Grid& g, float ox, float oy, float oz, float dx, float dy, float dz,
                           const RayInv& inv, float a, float b, Counters& cnt) {
    DfRay r;
    if (!df_init(g, ox, oy, oz, dx, dy, dz, inv, a, b, r)) return __builtin_inff();
    // The cubic solve runs outside the marching loop: a lane leaves the loop
    // at a cell that may hold its root and the wavefront solves all such lanes
    // together (nearly every solve ends its ray).
    int budget = df_max_steps(g);
    for (;;) {
        int st = kDfContinue;
        for (; budget > 0 && st == kDfContinue; --budget) st = df_step<FMT, COUNT>(g, r, cnt);
        if (st == kDfSolve) st = df_resolve<FMT, REFORM>(g, r);
        if (st == kDfHit) return r.t;
        if (st == kDfMiss) return __builtin_inff();
        if (budget <= 0) {
            // Out of iterations without an answer: walk cell by cell from the
            // end of the part of the ray already verified free of roots.  The
            // walk visits each crossed cell once and is exact, so the result
            // is still the first root.  A walk that ran out too (impossible
            // by the bound above) reports NaN, never a miss.
            if (r.walk_only) return __builtin_nanf("");
            r.t = r.cover;
            r.walk = false;
            r.walk_only = true;
            budget = df_max_walk(g);
        }
    }
}

// Implicit derivative of a distance-field hit: for the ray's hit t_hit on its
// segment [a, b], the 8 node indices of the cell holding p = o + t_hit d and
// d t_hit / d sample = -w_j / (grad f~(p) . d).  Returns false when the ray has
// no crossing (no hit, a hit at the clipped segment start, or a vanishing
// directional derivative).
HYB_HD bool df_hit_gradient(const Grid& g, float ox, float oy, float oz, float dx, float dy, float dz, float a,
                            float b, float t_hit, int64_t node[8], float dt[8]) {
    if (!(t_hit < __builtin_inff())) return false;
    DfRay r;
    if (!df_init(g, ox, oy, oz, dx, dy, dz, ray_inv(dx, dy, dz), a, b, r) || !(t_hit > r.t)) return false;
    const int nm2 = g.n - 2;
    const double X = fma((double)t_hit, r.qx, r.px), Y = fma((double)t_hit, r.qy, r.py), Z = fma((double)t_hit, r.qz, r.pz);
    const int ci = min(max((int)X, 0), nm2), cj = min(max((int)Y, 0), nm2), ck = min(max((int)Z, 0), nm2);
    const float fx = (float)(X - ci), fy = (float)(Y - cj), fz = (float)(Z - ck);
    float f[8];
    corners<kF32>(g, ci, cj, ck, f);
    // gradient of the interpolant in cell units, then along d (per unit t)
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    for (int c = 0; c < 8; ++c) {
        const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        gx += f[c] * (bx ? 1.0f : -1.0f) * wy[by] * wz[bz];
        gy += f[c] * wx[bx] * (by ? 1.0f : -1.0f) * wz[bz];
        gz += f[c] * wx[bx] * wy[by] * (bz ? 1.0f : -1.0f);
    }
    const float slope = gx * r.qxf + gy * r.qyf + gz * r.qzf;
    if (slope == 0.0f) return false;
    const float inv = -1.0f / slope;
    const int64_t n = g.n;
    for (int c = 0; c < 8; ++c) {
        const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        node[c] = (int64_t)(ci + bx) + n * ((int64_t)(cj + by) + n * (int64_t)(ck + bz));
        dt[c] = wx[bx] * wy[by] * wz[bz] * inv;
    }
    return true;
}

// Gradient bound of the trilinear interpolant inside one cell (corners f):
// each partial derivative is a convex blend of the cell's four edge differences
// along that axis (divided by h), so |grad| <= sqrt(mx^2 + my^2 + mz^2) / h.
// Largest |edge difference| / h of a cell along x, y and z: bounds of
// |df/dx|, |df/dy|, |df/dz| inside it (each partial derivative of the
// interpolant is a blend of the edge differences along its axis).
HYB_HD void cell_slopes(const float f[8], float inv_h, float m[3]) {
    m[0] = fmaxf(fmaxf(fabsf(f[1] - f[0]), fabsf(f[3] - f[2])), fmaxf(fabsf(f[5] - f[4]), fabsf(f[7] - f[6]))) * inv_h;
    m[1] = fmaxf(fmaxf(fabsf(f[2] - f[0]), fabsf(f[3] - f[1])), fmaxf(fabsf(f[6] - f[4]), fabsf(f[7] - f[5]))) * inv_h;
    m[2] = fmaxf(fmaxf(fabsf(f[4] - f[0]), fabsf(f[5] - f[1])), fmaxf(fabsf(f[6] - f[2]), fabsf(f[7] - f[3]))) * inv_h;
}

HYB_HD float cell_lipschitz(const float f[8], float inv_h) {
    const float mx = fmaxf(fmaxf(fabsf(f[1] - f[0]), fabsf(f[3] - f[2])), fmaxf(fabsf(f[5] - f[4]), fabsf(f[7] - f[6])));
    const float my = fmaxf(fmaxf(fabsf(f[2] - f[0]), fabsf(f[3] - f[1])), fmaxf(fabsf(f[6] - f[4]), fabsf(f[7] - f[5])));
    const float mz = fmaxf(fmaxf(fabsf(f[4] - f[0]), fabsf(f[5] - f[1])), fmaxf(fabsf(f[6] - f[2]), fabsf(f[7] - f[3])));
    return sqrtf(mx * mx + my * my + mz * mz) * inv_h;
}

// Lipschitz bound used for steps, from the largest cell bound of the grid: at
// least 1 (keeps steps finite on flat fields), rounded up a few ulps so it
// stays a bound after FP32 evaluation.
HYB_HD float finish_lipschitz(float cell_max) { return fmaxf(cell_max, 1.0f) * (1.0f + 4e-7f); }

// Per-axis slope bound from the largest cell value, rounded up likewise.
HYB_HD float finish_slope(float cell_max) { return cell_max * (1.0f + 4e-7f); }

// Reciprocal step factor: g * inv_step(L) is a safe sphere-tracing step.
HYB_HD float inv_step(float lipschitz) { return (1.0f / lipschitz) * (1.0f - 1e-6f); }

// Step slack for grids whose samples are FP32 roundings of a 1-Lipschitz
// function f (an exact distance field).  Then |f~ - f| <= E + q with
// E = sqrt(3)/2 h (the largest blend of corner distances inside a cell) and q
// the storage error, so f~ stays positive for a distance g - 2 (E + q) ahead.
// q covers one FP32 rounding of any sample (|f| <= the grid diagonal) plus a
// margin of 1e-4 h.
HYB_HD float certified_slack(float h, int n) {
    const float q = 1e-4f * h + 2.4e-7f * 1.7320508f * (float)(n - 1) * h;
    return 2.0f * (0.8660254f * h * (1.0f + 1e-6f) + q);
}

// Where a traversal of the segment [t0, t1] may start: the entry of the
// finest window of the pyramid (2 x 2 x 2 half-cells, windows overlapping by
// a half-cell) that holds the whole segment, grown by a margin over the FP32
// rounding of its end points (every triangle the segment can hit overlaps
// that window, so it lies under the window's entry), else the root.  Parts of
// the segment outside the pyramid's box reach no triangle, so the end points
// are clamped into it.
HYB_HD int entry_node(const TraceArgs& a, float ox, float oy, float oz, float dx, float dy, float dz, float t0,
                      float t1) {
    // a segment longer than 8 finest voxels almost never fits one window deep
    // enough to skip levels: start at the root without looking
    if (a.entry_res == 0 || !((t1 - t0) * a.entry_inv <= 8.0f)) return 0;
    const int H = 2 * a.entry_res;  // finest half-cells per axis
    int ia[3], ib[3];
    const float o[3] = {ox, oy, oz}, d[3] = {dx, dy, dz}, lo[3] = {a.entry_lo_x, a.entry_lo_y, a.entry_lo_z};
    const float inv_half = 2.0f * a.entry_inv;
    for (int k = 0; k < 3; ++k) {
        const float p0 = fmaf(t0, d[k], o[k]), p1 = fmaf(t1, d[k], o[k]);
        const float m = 1e-6f * (1.0f + fmaxf(fabsf(p0), fabsf(p1)));
        const float u0 = (fminf(p0, p1) - m - lo[k]) * inv_half;
        const float u1 = (fmaxf(p0, p1) + m - lo[k]) * inv_half;
        ia[k] = (int)floorf(fminf(fmaxf(u0, 0.0f), (float)(H - 1)));
        ib[k] = (int)floorf(fminf(fmaxf(u1, 0.0f), (float)(H - 1)));
    }
    int level = 0, off = 0;
    for (; level + 1 < a.entry_levels; ++level) {
        if ((ib[0] >> level) - (ia[0] >> level) <= 1 && (ib[1] >> level) - (ia[1] >> level) <= 1 &&
            (ib[2] >> level) - (ia[2] >> level) <= 1)
            break;
        const int w = (H >> level) - 1;
        off += w * w * w;
    }
    const int w = (H >> level) - 1;
    const int x = min(ia[0] >> level, w - 1), y = min(ia[1] >> level, w - 1), z = min(ia[2] >> level, w - 1);
    return a.entry[off + x + w * (y + w * z)];
}

// Triangle segments at most this many voxels long are traversed without
// ordering the children (their boxes mostly all overlap the short segment, so
// nearest-first order prunes little and costs a sorting network per node).
constexpr float kShortSegment = 4.0f;

// The grid of a query's arguments, with the step bounds of a deferred
// update read from the device (uniform loads) where the arguments point at
// them.
HYB_HD Grid grid_of(const TraceArgs& a) {
    Grid g = {a.sdf, a.n_grid, a.lo_x, a.lo_y, a.lo_z, a.h, a.inv_h, a.inv_l, a.two_e,
              a.slope_x, a.slope_y, a.slope_z, a.inv_hd};
    if (a.bounds) {
        g.inv_l = a.bounds[kBInvL];
        g.slope_x = a.bounds[kBSlopeX];
        g.slope_y = a.bounds[kBSlopeY];
        g.slope_z = a.bounds[kBSlopeZ];
        g.two_e = a.bounds[kBTwoE];
    }
    return g;
}

// A deferred update found a sample that is not finite: the distance-field
// part of every query reports NaN (prim -2) until the next update.
HYB_HD bool df_unusable(const TraceArgs& a) { return a.bounds && a.bounds[kBBad] != 0.0f; }

// One ray of a query (the body of the trace kernels).
template <int MODE, int FMT, bool COUNT, int LDS = kLdsDepth>
HYB_HD void trace_ray(const TraceArgs& a, int64_t i, int* stack, int stride) {
    const float ox = a.ox[i], oy = a.oy[i], oz = a.oz[i];
    const float dx = a.dx[i], dy = a.dy[i], dz = a.dz[i];
    const float tmin = a.tmin ? a.tmin[i] : 0.0f;
    const float tmax = a.tmax_ray ? fminf(a.tmax_ray[i], a.tmax) : a.tmax;
    Counters cnt;
    Hit hit;
    hit.t = __builtin_inff();
    hit.prim = -1;
    hit.u = 0.0f;
    hit.v = 0.0f;
    if (tmin <= tmax) {
        const Grid g = grid_of(a);
        if (MODE != kBvhOnly && df_unusable(a)) {
            hit.t = __builtin_nanf("");
            hit.prim = -2;
        } else if (MODE == kBvhOnly) {
            hit = bvh_closest<COUNT, false, LDS>(a.nodes, a.tris, ox, oy, oz, dx, dy, dz, ray_inv(dx, dy, dz), tmin,
                                                 tmax, stack, stride, cnt,
                                                 entry_node(a, ox, oy, oz, dx, dy, dz, tmin, tmax));
        } else if (MODE == kDfOnly) {
            const float t = df_first_root<FMT, COUNT>(g, ox, oy, oz, dx, dy, dz, ray_inv(dx, dy, dz), tmin, tmax, cnt);
            if (t != __builtin_inff()) {  // NaN: see df_first_root
                hit.t = t;
                hit.prim = -2;
            }
        } else if (MODE == kShadow) {
            // Section 3 shadow rays: triangles near both ends, the distance
            // field in between; any intersection suffices, so the cheap DF part
            // runs first (Section 2, out-of-order any-hit processing).
            const float t1 = fminf(fmaf(a.tau, a.h, tmin), tmax);
            const float t2 = fmaxf(fmaf(-a.tau_end, a.h, tmax), t1);
            const bool sort = !(a.tau <= kShortSegment && a.tau_end <= kShortSegment);
            if (t2 > t1 || (a.tau == 0.0f && a.tau_end == 0.0f)) {
                const float t = df_first_root<FMT, COUNT>(g, ox, oy, oz, dx, dy, dz, ray_inv(dx, dy, dz), t1, t2, cnt);
                if (t != __builtin_inff()) {  // NaN: see df_first_root
                    hit.t = t;
                    hit.prim = -2;
                }
            }
            if (hit.prim == -1 && t1 > tmin)
                hit = bvh_closest<COUNT, true, LDS>(a.nodes, a.tris, ox, oy, oz, dx, dy, dz, ray_inv(dx, dy, dz), tmin,
                                                    t1, stack, stride, cnt,
                                                    entry_node(a, ox, oy, oz, dx, dy, dz, tmin, t1), sort);
            if (hit.prim == -1 && tmax > t2)
                hit = bvh_closest<COUNT, true, LDS>(a.nodes, a.tris, ox, oy, oz, dx, dy, dz, ray_inv(dx, dy, dz), t2,
                                                    tmax, stack, stride, cnt,
                                                    entry_node(a, ox, oy, oz, dx, dy, dz, t2, tmax), sort);
        } else {
            // Eq. (2) with two sub-queries processed in order (first hit):
            // triangles on [tmin, t1]; the distance field on [t1, tmax] only
            // when the first sub-query found nothing.  Both slab tests use
            // the same 1 / d (the other modes form it where they use it: kept
            // across the shadow query's march it cost that kernel a
            // wavefront per SIMD).
            const RayInv inv = ray_inv(dx, dy, dz);
            const float t1 = fminf(fmaf(a.tau, a.h, tmin), tmax);
            if (t1 > tmin)
                hit = bvh_closest<COUNT, false, LDS>(a.nodes, a.tris, ox, oy, oz, dx, dy, dz, inv, tmin, t1, stack,
                                                     stride, cnt, entry_node(a, ox, oy, oz, dx, dy, dz, tmin, t1),
                                                     !(a.tau <= kShortSegment));
            if (hit.prim < 0 && (t1 < tmax || a.tau == 0.0f)) {
                // I8 forms its solves again (df_resolve, REFORM): seven wavefronts per SIMD
                const float t = df_first_root<FMT, COUNT, FMT == kI8>(g, ox, oy, oz, dx, dy, dz, inv, t1, tmax, cnt);
                if (t != __builtin_inff()) {  // NaN: see df_first_root
                    hit.t = t;
                    hit.prim = -2;
                }
            }
        }
    }
    a.t[i] = hit.t;
    a.prim[i] = hit.prim;
    a.u[i] = hit.u;
    a.v[i] = hit.v;
    if (COUNT) {
        a.counts[3 * i + 0] = cnt.nodes;
        a.counts[3 * i + 1] = cnt.tris;
        a.counts[3 * i + 2] = cnt.df;
    }
}

}  // namespace hyb
