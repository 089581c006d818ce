// Internal to the C API: the handle structs behind include/hyb.h's opaque
// handles and the argument helpers shared by the entry-point sources.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hyb.h"
#include "hyb_device.hpp"
#include "kernels.hpp"

struct hyb_bvh_s {
    int device = 0;
    float4* nodes = nullptr;   // binary tree (64-byte nodes): the distance-field build's queries
    float4* nodes4 = nullptr;  // the same tree with four children per node (128 bytes): the trace kernels
    int32_t* entry = nullptr;  // traversal entry pyramid (BvhHost::entry)
    float entry_lo[3] = {0, 0, 0}, entry_size = 0.0f;
    int32_t entry_res = 0, entry_levels = 0;
    float4* tris = nullptr;
    int64_t n_nodes = 0, n_tris = 0;  // n_nodes counts the four-wide nodes
    int32_t depth = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
};

struct hyb_sdf_s {
    int device = 0;
    float* values = nullptr;  // n^3 FP32 samples as the kernels see them (dequantized), x fastest
    void* store = nullptr;    // the samples the kernels read: storage format, bricked layout
    float* scales = nullptr;  // I8 block scales
    int32_t n = 0, nb = 0;
    float grid4[4] = {0, 0, 0, 0};
    float lipschitz = 0.0f;
    float slope[3] = {0, 0, 0};  // per-axis bounds of |df/dx_i|
    bool certified = false;  // samples are FP32 roundings of a 1-Lipschitz function
    hyb_sdf_format fmt = HYB_SDF_F32;
    int32_t layout = 0;  // the kernels' storage format and brick layout (hyb::SdfFormat)
    float* blocks = nullptr;  // per-block maxima of the bound pass (kept for updates)
    uint64_t version = 0;     // bumped whenever the samples and bounds change (batches re-read them)
    float* dev_bounds = nullptr;  // hyb::kDeviceBounds floats: the bounds of a deferred update
    bool deferred = false;        // the last update was deferred: the kernels read dev_bounds
    void* bwd_ws = nullptr;       // hyb_df_backward's sort buffers, grown on demand
    size_t bwd_ws_bytes = 0;
    int64_t bwd_n = 0;            // the ray count whose buffer size bwd_need holds
    size_t bwd_need = 0;
};

namespace hyb_api {

inline hyb_status from_hip(hipError_t e) {
    if (e == hipSuccess) return HYB_OK;
    if (e == hipErrorOutOfMemory) return HYB_ERR_OOM;
    return HYB_ERR_HIP;
}

#define HYB_TRY(expr)                               \
    do {                                            \
        hyb_status s_ = from_hip(expr);             \
        if (s_ != HYB_OK) return s_;                \
    } while (0)

inline bool same_device(int dev) {
    int cur = -1;
    return hipGetDevice(&cur) == hipSuccess && cur == dev;
}

inline bool valid_rays(const hyb_rays* r) {
    return r && r->ox && r->oy && r->oz && r->dx && r->dy && r->dz;
}

inline bool valid_hits(const hyb_hits* h) { return h && h->t && h->prim && h->u && h->v; }

// The bound pass over s->values (n^3, x fastest) into host maxima m[0..4]
// (see launch_lipschitz); synchronous.
inline hyb_status grid_bounds(hyb_sdf_s* s, hipStream_t stream, float m[hyb::kBoundValues]) {
    constexpr int V = hyb::kBoundValues;
    const int32_t nb = hyb::lipschitz_blocks(s->n);
    if (!s->blocks) HYB_TRY(hipMalloc(&s->blocks, sizeof(float) * V * nb));
    int32_t got = 0;
    hipError_t e = hyb::launch_lipschitz(s->values, s->n, s->grid4[3], s->blocks, &got, stream);
    std::vector<float> host(V * static_cast<size_t>(nb), 0.0f);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), s->blocks, sizeof(float) * V * nb, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    HYB_TRY(e);
    for (int c = 0; c < V; ++c) m[c] = 0.0f;
    for (size_t b = 0; b < static_cast<size_t>(nb); ++b)
        for (int c = 0; c < V; ++c) m[c] = std::max(m[c], host[V * b + c]);
    return HYB_OK;
}

// HYB_ERR_INVALID_ARG when some sample in s->values is NaN or infinite.
inline hyb_status check_finite(hyb_sdf_s* s, hipStream_t stream) {
    float m[hyb::kBoundValues];
    const hyb_status rc = grid_bounds(s, stream, m);
    if (rc != HYB_OK) return rc;
    return m[4] != 0.0f ? HYB_ERR_INVALID_ARG : HYB_OK;
}

// Lipschitz bound and per-axis slope bounds of the stored grid: per-block
// maxima on the device, final maxima on the host (build time; synchronous).
// A stored sample that is not finite (e.g. an F16 overflow) is an error.
inline hyb_status compute_lipschitz(hyb_sdf_s* s, hipStream_t stream) {
    float m[hyb::kBoundValues];
    const hyb_status rc = grid_bounds(s, stream, m);
    if (rc != HYB_OK) return rc;
    for (float v : m)
        if (!std::isfinite(v)) return HYB_ERR_INVALID_ARG;
    if (m[4] != 0.0f) return HYB_ERR_INVALID_ARG;
    s->lipschitz = hyb::finish_lipschitz(m[0]);
    for (int c = 0; c < 3; ++c) s->slope[c] = hyb::finish_slope(m[1 + c]);
    s->deferred = false;
    ++s->version;
    return HYB_OK;
}

// The certified-grid step slack of the kernels, or +inf.
inline float two_e_of(const hyb_sdf_s* s) {
    return (s->certified && s->fmt == HYB_SDF_F32) ? hyb::certified_slack(s->grid4[3], s->n) : __builtin_inff();
}

// The bounds of compute_lipschitz (and check_finite for the compact formats,
// on the input before it is quantized) left on the device for the kernels,
// without waiting: the quantization runs between the two passes.
inline hyb_status deferred_bounds(hyb_sdf_s* s, hipStream_t stream) {
    const int32_t nb = hyb::lipschitz_blocks(s->n);
    if (!s->blocks) HYB_TRY(hipMalloc(&s->blocks, sizeof(float) * hyb::kBoundValues * nb));
    int32_t got = 0;
    if (s->fmt != HYB_SDF_F32) {
        HYB_TRY(hyb::launch_lipschitz(s->values, s->n, s->grid4[3], s->blocks, &got, stream));
        HYB_TRY(hyb::launch_finish_bounds(s->blocks, got, 0, 0.0f, s->dev_bounds, stream));
    }
    HYB_TRY(hyb::launch_quantize(s->layout, s->values, s->n, s->store, s->scales, stream));
    HYB_TRY(hyb::launch_lipschitz(s->values, s->n, s->grid4[3], s->blocks, &got, stream));
    HYB_TRY(hyb::launch_finish_bounds(s->blocks, got, s->fmt != HYB_SDF_F32 ? 1 : 2, two_e_of(s), s->dev_bounds,
                                      stream));
    s->deferred = true;
    ++s->version;
    return HYB_OK;
}

// Writes the kernels' copy of the FP32 samples in s->values (storage format,
// bricked layout); for the compact formats the dequantized values replace
// s->values in place.
inline hyb_status quantize(hyb_sdf_s* s, hipStream_t stream) {
    const int fmt = s->fmt == HYB_SDF_F32 ? hyb::kF32 : (s->fmt == HYB_SDF_F16 ? hyb::f16_layout(s->n) : hyb::kI8);
    s->layout = fmt;
    const size_t count = static_cast<size_t>(hyb::brick_storage(fmt, s->n));
    const size_t elem = s->fmt == HYB_SDF_F32 ? 4 : (s->fmt == HYB_SDF_F16 ? 2 : 1);
    s->nb = hyb::i8_blocks(s->n);
    HYB_TRY(hipMalloc(&s->store, count * elem));
    if (s->fmt == HYB_SDF_I8_BRICK)
        HYB_TRY(hipMalloc(&s->scales, sizeof(float) * static_cast<size_t>(s->nb) * s->nb * s->nb));
    return from_hip(hyb::launch_quantize(fmt, s->values, s->n, s->store, s->scales, stream));
}

inline bool valid_fmt(hyb_sdf_format f) { return f == HYB_SDF_F32 || f == HYB_SDF_F16 || f == HYB_SDF_I8_BRICK; }

inline bool valid_grid4(const float* g) {
    return g && std::isfinite(g[0]) && std::isfinite(g[1]) && std::isfinite(g[2]) && std::isfinite(g[3]) &&
           g[3] > 0.0f;
}

inline void fill_trace_args(hyb::TraceArgs& a, const hyb_rays* rays, hyb_hits* hits, int64_t n, float tmax, float tau,
                     float tau_end = 0.0f) {
    std::memset(&a, 0, sizeof(a));
    a.ox = rays->ox; a.oy = rays->oy; a.oz = rays->oz;
    a.dx = rays->dx; a.dy = rays->dy; a.dz = rays->dz;
    a.tmin = rays->tmin;
    a.tmax_ray = rays->tmax;
    a.tau_end = tau_end;
    a.t = hits->t; a.prim = hits->prim; a.u = hits->u; a.v = hits->v;
    a.tmax = tmax;
    a.tau = tau;
    a.n = n;
}

// Bytes of the kernels' bricked copy of a grid.
inline int64_t copy_bytes(const hyb_sdf_s* s) {
    const int64_t elem = s->layout == hyb::kF32 ? 4 : (s->layout == hyb::kI8 ? 1 : 2);
    return hyb::brick_storage(s->layout, s->n) * elem;
}

inline void fill_scene(hyb::TraceArgs& a, const hyb_bvh_s* b, const hyb_sdf_s* s) {
    a.xcd_run = hyb::xcd_run_for(s ? copy_bytes(s) : 0);
    if (b) {
        a.nodes = b->nodes4;
        a.entry = b->entry_res ? b->entry : nullptr;
        a.entry_lo_x = b->entry_lo[0];
        a.entry_lo_y = b->entry_lo[1];
        a.entry_lo_z = b->entry_lo[2];
        a.entry_inv = b->entry_res ? 1.0f / b->entry_size : 0.0f;
        a.entry_res = b->entry_res;
        a.entry_levels = b->entry_levels;
        a.tris = b->tris;
    }
    if (s) {
        a.sdf = s->store;
        a.fmt = s->layout;
        a.n_grid = s->n;
        a.lo_x = s->grid4[0];
        a.lo_y = s->grid4[1];
        a.lo_z = s->grid4[2];
        a.h = s->grid4[3];
        a.inv_h = 1.0f / s->grid4[3];
        a.inv_hd = 1.0 / (double)s->grid4[3];
        a.inv_l = hyb::inv_step(s->lipschitz);
        a.two_e = two_e_of(s);
        a.bounds = s->deferred ? s->dev_bounds : nullptr;
        a.slope_x = s->slope[0];
        a.slope_y = s->slope[1];
        a.slope_z = s->slope[2];
    }
}

inline hyb_status check_query(const hyb_rays* rays, int64_t n, float tmax, hyb_hits* hits) {
    if (n < 0 || n > HYB_MAX_RAYS || std::isnan(tmax) || tmax < 0.0f) return HYB_ERR_INVALID_ARG;
    if (n > 0 && (!valid_rays(rays) || !valid_hits(hits))) return HYB_ERR_INVALID_ARG;
    return HYB_OK;
}

}  // namespace hyb_api
