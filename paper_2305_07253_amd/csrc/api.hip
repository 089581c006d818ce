// C API: argument validation, handle lifetime and launches on the caller's
// stream.  Declared in include/hyb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.hpp"
#include "bvh_build.hpp"

static_assert(hyb::kStackDepth >= hyb::kStackDepth4, "trace stack smaller than the builder's bound");

using namespace hyb_api;

extern "C" {

const char* hyb_status_str(hyb_status s) {
    switch (s) {
        case HYB_OK: return "HYB_OK";
        case HYB_ERR_INVALID_ARG: return "HYB_ERR_INVALID_ARG";
        case HYB_ERR_OOM: return "HYB_ERR_OOM";
        case HYB_ERR_HIP: return "HYB_ERR_HIP";
        case HYB_ERR_UNSUPPORTED: return "HYB_ERR_UNSUPPORTED";
    }
    return "HYB_ERR_UNKNOWN";
}

hyb_status hyb_build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, void* stream,
                         hyb_bvh* out) {
    if (!out) return HYB_ERR_INVALID_ARG;
    *out = nullptr;
    hyb::BvhHost host;
    int rc = hyb::build_bvh_host(verts, n_verts, tris, n_tris, &host);
    if (rc == 1) return HYB_ERR_INVALID_ARG;
    if (rc != 0) return HYB_ERR_UNSUPPORTED;
    hyb_bvh_s* b = new (std::nothrow) hyb_bvh_s;
    if (!b) return HYB_ERR_OOM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&b->device);
    b->n_nodes = static_cast<int64_t>(host.nodes4.size() / 32);
    b->n_tris = n_tris;
    b->depth = host.depth4;
    for (int a = 0; a < 3; ++a) {
        b->lo[a] = host.lo[a];
        b->hi[a] = host.hi[a];
    }
    const size_t node_bytes = host.nodes.size() * sizeof(float);
    const size_t tri_bytes = std::max<size_t>(host.tris.size(), 12) * sizeof(float);
    const size_t node4_bytes = host.nodes4.size() * sizeof(float);
    const size_t entry_bytes = host.entry.size() * sizeof(int32_t);
    b->entry_res = host.entry_res;
    b->entry_levels = host.entry_levels;
    b->entry_size = host.entry_size;
    for (int a = 0; a < 3; ++a) b->entry_lo[a] = host.entry_lo[a];
    if (e == hipSuccess && entry_bytes) e = hipMalloc(&b->entry, entry_bytes);
    if (e == hipSuccess && entry_bytes)
        e = hipMemcpyAsync(b->entry, host.entry.data(), entry_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMalloc(&b->nodes, node_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->nodes4, node4_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->tris, tri_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(b->nodes, host.nodes.data(), node_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->nodes4, host.nodes4.data(), node4_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !host.tris.empty())
        e = hipMemcpyAsync(b->tris, host.tris.data(), host.tris.size() * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        hyb_bvh_destroy(b);
        return from_hip(e);
    }
    *out = b;
    return HYB_OK;
}

hyb_status hyb_bvh_info(hyb_bvh bvh, int64_t* n_nodes, int64_t* n_tris, int32_t* depth) {
    if (!bvh) return HYB_ERR_INVALID_ARG;
    if (n_nodes) *n_nodes = bvh->n_nodes;
    if (n_tris) *n_tris = bvh->n_tris;
    if (depth) *depth = bvh->depth;
    return HYB_OK;
}

hyb_status hyb_bvh_destroy(hyb_bvh bvh) {
    if (!bvh) return HYB_ERR_INVALID_ARG;
    if (bvh->nodes) (void)hipFree(bvh->nodes);
    if (bvh->nodes4) (void)hipFree(bvh->nodes4);
    if (bvh->entry) (void)hipFree(bvh->entry);
    if (bvh->tris) (void)hipFree(bvh->tris);
    delete bvh;
    return HYB_OK;
}

hyb_status hyb_build_sdf(hyb_bvh bvh, int32_t n, const float* grid4, uint32_t flags, hyb_sdf_format fmt,
                         void* stream, hyb_sdf* out) {
    if (!out) return HYB_ERR_INVALID_ARG;
    *out = nullptr;
    if (!bvh || n < 8 || n > 1024 || (flags & ~HYB_SDF_EXTERIOR_SOLID) || !valid_fmt(fmt)) return HYB_ERR_INVALID_ARG;
    if (!same_device(bvh->device)) return HYB_ERR_INVALID_ARG;
    float g4[4];
    if (grid4) {
        if (!valid_grid4(grid4)) return HYB_ERR_INVALID_ARG;
        std::memcpy(g4, grid4, sizeof(g4));
    } else {
        float ext = 0.0f;
        for (int a = 0; a < 3; ++a) ext = std::max(ext, bvh->hi[a] - bvh->lo[a]);
        g4[3] = ext > 0.0f ? ext / static_cast<float>(n - 5) : 1.0f;
        for (int a = 0; a < 3; ++a) g4[a] = bvh->lo[a] - 2.0f * g4[3];
    }
    hyb_sdf_s* s = new (std::nothrow) hyb_sdf_s;
    if (!s) return HYB_ERR_OOM;
    s->device = bvh->device;
    s->n = n;
    s->fmt = fmt;
    s->certified = true;  // exact distances to the mesh
    std::memcpy(s->grid4, g4, sizeof(g4));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = sizeof(float) * static_cast<size_t>(n) * n * n;
    hipError_t e = hipMalloc(&s->values, bytes);
    if (e == hipSuccess) {
        hyb::SdfBuildArgs a;
        a.nodes = bvh->nodes;
        a.tris = bvh->tris;
        a.n_grid = n;
        a.lo_x = g4[0];
        a.lo_y = g4[1];
        a.lo_z = g4[2];
        a.h = g4[3];
        a.exterior_solid = (flags & HYB_SDF_EXTERIOR_SOLID) ? 1 : 0;
        a.out = s->values;
        e = hyb::launch_sdf_build(a, st);
    }
    hyb_status rc = from_hip(e);
    if (rc == HYB_OK) rc = quantize(s, st);
    if (rc == HYB_OK) rc = from_hip(hipMalloc(&s->dev_bounds, sizeof(float) * hyb::kDeviceBounds));
    if (rc == HYB_OK) rc = compute_lipschitz(s, st);
    if (rc != HYB_OK) {
        hyb_sdf_destroy(s);
        return rc;
    }
    *out = s;
    return HYB_OK;
}

hyb_status hyb_sdf_from_grid(const float* values, int32_t n, const float* grid4, uint32_t flags, hyb_sdf_format fmt,
                             void* stream, hyb_sdf* out) {
    if (!out) return HYB_ERR_INVALID_ARG;
    *out = nullptr;
    if (!values || n < 2 || n > 1024 || !valid_grid4(grid4) || (flags & ~HYB_SDF_LIPSCHITZ_SAMPLES) || !valid_fmt(fmt))
        return HYB_ERR_INVALID_ARG;
    hyb_sdf_s* s = new (std::nothrow) hyb_sdf_s;
    if (!s) return HYB_ERR_OOM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&s->device);
    s->n = n;
    s->fmt = fmt;
    s->certified = (flags & HYB_SDF_LIPSCHITZ_SAMPLES) != 0;
    std::memcpy(s->grid4, grid4, sizeof(s->grid4));
    const size_t bytes = sizeof(float) * static_cast<size_t>(n) * n * n;
    if (e == hipSuccess) e = hipMalloc(&s->values, bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(s->values, values, bytes, hipMemcpyDeviceToDevice, st);
    hyb_status rc = from_hip(e);
    // the compact formats would turn a NaN input into a finite code
    if (rc == HYB_OK && fmt != HYB_SDF_F32) rc = check_finite(s, st);
    if (rc == HYB_OK) rc = quantize(s, st);
    if (rc == HYB_OK) rc = from_hip(hipMalloc(&s->dev_bounds, sizeof(float) * hyb::kDeviceBounds));
    if (rc == HYB_OK) rc = compute_lipschitz(s, st);
    if (rc != HYB_OK) {
        hyb_sdf_destroy(s);
        return rc;
    }
    *out = s;
    return HYB_OK;
}

hyb_status hyb_sdf_update(hyb_sdf sdf, const float* values, uint32_t flags, void* stream) {
    if (!sdf || !values || (flags & ~(HYB_SDF_LIPSCHITZ_SAMPLES | HYB_SDF_UPDATE_DEFERRED)) ||
        !same_device(sdf->device))
        return HYB_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = sizeof(float) * static_cast<size_t>(sdf->n) * sdf->n * sdf->n;
    sdf->certified = (flags & HYB_SDF_LIPSCHITZ_SAMPLES) != 0;
    HYB_TRY(hipMemcpyAsync(sdf->values, values, bytes, hipMemcpyDeviceToDevice, st));
    if (flags & HYB_SDF_UPDATE_DEFERRED) return deferred_bounds(sdf, st);
    if (sdf->fmt != HYB_SDF_F32) {
        // the compact formats would turn a NaN input into a finite code
        const hyb_status rc = check_finite(sdf, st);
        if (rc != HYB_OK) return rc;
    }
    HYB_TRY(hyb::launch_quantize(sdf->layout, sdf->values, sdf->n, sdf->store, sdf->scales, st));
    return compute_lipschitz(sdf, st);
}

hyb_status hyb_sdf_voxel_size(hyb_sdf sdf, float* h) {
    if (!sdf || !h) return HYB_ERR_INVALID_ARG;
    *h = sdf->grid4[3];
    return HYB_OK;
}

hyb_status hyb_sdf_info(hyb_sdf sdf, float* grid4, int32_t* n, float* lipschitz) {
    if (!sdf) return HYB_ERR_INVALID_ARG;
    if (grid4) std::memcpy(grid4, sdf->grid4, sizeof(sdf->grid4));
    if (n) *n = sdf->n;
    if (lipschitz) {
        if (sdf->deferred) {
            // the bound of a deferred update is on the device
            HYB_TRY(hipDeviceSynchronize());
            HYB_TRY(hipMemcpy(&sdf->lipschitz, sdf->dev_bounds + hyb::kBLipschitz, sizeof(float),
                              hipMemcpyDeviceToHost));
        }
        *lipschitz = sdf->lipschitz;
    }
    return HYB_OK;
}

hyb_status hyb_sdf_check(hyb_sdf sdf, void* stream) {
    if (!sdf) return HYB_ERR_INVALID_ARG;
    if (!sdf->deferred) return HYB_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float bad = 0.0f;
    HYB_TRY(hipMemcpyAsync(&bad, sdf->dev_bounds + hyb::kBBad, sizeof(float), hipMemcpyDeviceToHost, st));
    HYB_TRY(hipStreamSynchronize(st));
    return bad != 0.0f ? HYB_ERR_INVALID_ARG : HYB_OK;
}

hyb_status hyb_sdf_read(hyb_sdf sdf, float* out, void* stream) {
    if (!sdf || !out) return HYB_ERR_INVALID_ARG;
    const size_t bytes = sizeof(float) * static_cast<size_t>(sdf->n) * sdf->n * sdf->n;
    return from_hip(hipMemcpyAsync(out, sdf->values, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
}

hyb_status hyb_sdf_destroy(hyb_sdf sdf) {
    if (!sdf) return HYB_ERR_INVALID_ARG;
    if (sdf->values) (void)hipFree(sdf->values);
    if (sdf->store) (void)hipFree(sdf->store);
    if (sdf->scales) (void)hipFree(sdf->scales);
    if (sdf->blocks) (void)hipFree(sdf->blocks);
    if (sdf->dev_bounds) (void)hipFree(sdf->dev_bounds);
    if (sdf->bwd_ws) (void)hipFree(sdf->bwd_ws);
    delete sdf;
    return HYB_OK;
}

hyb_status hyb_trace(hyb_bvh bvh, hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, float threshold,
                     hyb_hits* hits, void* stream) {
    if (!bvh || !sdf || std::isnan(threshold) || threshold < 0.0f) return HYB_ERR_INVALID_ARG;
    hyb_status rc = check_query(rays, n, tmax, hits);
    if (rc != HYB_OK || n == 0) return rc;
    if (!same_device(bvh->device) || !same_device(sdf->device)) return HYB_ERR_INVALID_ARG;
    hyb::TraceArgs a;
    fill_trace_args(a, rays, hits, n, tmax, threshold);
    fill_scene(a, bvh, sdf);
    // Threshold 0 leaves the triangle segment empty (t1 = tmin), so the query
    // is the distance-field query on [tmin, tmax]: its own kernel runs it, the
    // same per-ray arithmetic without the traversal code or the LDS stack.
    const int mode = threshold == 0.0f ? hyb::kDfOnly : hyb::kCombined;
    return from_hip(hyb::launch_trace(mode, false, a, static_cast<hipStream_t>(stream)));
}

hyb_status hyb_trace_bvh(hyb_bvh bvh, const hyb_rays* rays, int64_t n, float tmax, hyb_hits* hits, void* stream) {
    if (!bvh) return HYB_ERR_INVALID_ARG;
    hyb_status rc = check_query(rays, n, tmax, hits);
    if (rc != HYB_OK || n == 0) return rc;
    if (!same_device(bvh->device)) return HYB_ERR_INVALID_ARG;
    hyb::TraceArgs a;
    fill_trace_args(a, rays, hits, n, tmax, __builtin_inff());
    fill_scene(a, bvh, nullptr);
    return from_hip(hyb::launch_trace(hyb::kBvhOnly, false, a, static_cast<hipStream_t>(stream)));
}

hyb_status hyb_trace_df(hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, hyb_hits* hits, void* stream) {
    if (!sdf) return HYB_ERR_INVALID_ARG;
    hyb_status rc = check_query(rays, n, tmax, hits);
    if (rc != HYB_OK || n == 0) return rc;
    if (!same_device(sdf->device)) return HYB_ERR_INVALID_ARG;
    hyb::TraceArgs a;
    fill_trace_args(a, rays, hits, n, tmax, 0.0f);
    fill_scene(a, nullptr, sdf);
    return from_hip(hyb::launch_trace(hyb::kDfOnly, false, a, static_cast<hipStream_t>(stream)));
}

hyb_status hyb_trace_shadow(hyb_bvh bvh, hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax,
                            float threshold_start, float threshold_end, hyb_hits* hits, void* stream) {
    if (!bvh || !sdf || std::isnan(threshold_start) || threshold_start < 0.0f || std::isnan(threshold_end) ||
        threshold_end < 0.0f)
        return HYB_ERR_INVALID_ARG;
    hyb_status rc = check_query(rays, n, tmax, hits);
    if (rc != HYB_OK || n == 0) return rc;
    if (!same_device(bvh->device) || !same_device(sdf->device)) return HYB_ERR_INVALID_ARG;
    hyb::TraceArgs a;
    fill_trace_args(a, rays, hits, n, tmax, threshold_start, threshold_end);
    fill_scene(a, bvh, sdf);
    return from_hip(hyb::launch_trace(hyb::kShadow, false, a, static_cast<hipStream_t>(stream)));
}

hyb_status hyb_df_backward(hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, const float* t_hit,
                           const float* grad_t, float* grad_grid, void* stream) {
    if (!sdf || n < 0 || n > HYB_MAX_RAYS || std::isnan(tmax) || tmax < 0.0f) return HYB_ERR_INVALID_ARG;
    if (n == 0) return HYB_OK;
    if (!valid_rays(rays) || !t_hit || !grad_t || !grad_grid) return HYB_ERR_INVALID_ARG;
    if (sdf->fmt != HYB_SDF_F32) return HYB_ERR_UNSUPPORTED;
    if (!same_device(sdf->device)) return HYB_ERR_INVALID_ARG;
    hyb::TraceArgs a;
    hyb_hits none = {nullptr, nullptr, nullptr, nullptr};
    fill_trace_args(a, rays, &none, n, tmax, 0.0f);
    fill_scene(a, nullptr, sdf);
    if (n != sdf->bwd_n) {  // sizing the sort costs host time: once per ray count
        sdf->bwd_need = hyb::df_backward_workspace(n, sdf->n);
        sdf->bwd_n = n;
    }
    const size_t need = sdf->bwd_need;
    if (need == 0) return HYB_ERR_HIP;
    if (sdf->bwd_ws_bytes < need) {
        if (sdf->bwd_ws) (void)hipFree(sdf->bwd_ws);
        sdf->bwd_ws = nullptr;
        sdf->bwd_ws_bytes = 0;
        HYB_TRY(hipMalloc(&sdf->bwd_ws, need));
        sdf->bwd_ws_bytes = need;
    }
    return from_hip(hyb::launch_df_backward(a, t_hit, grad_t, grad_grid, sdf->bwd_ws, need,
                                            static_cast<hipStream_t>(stream)));
}

hyb_status hyb_trace_counters(hyb_bvh bvh, hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, float threshold,
                              int32_t mode, hyb_hits* hits, int32_t* counts, void* stream) {
    if (mode < 0 || mode > 3 || std::isnan(threshold) || threshold < 0.0f) return HYB_ERR_INVALID_ARG;
    if ((mode != 2 && !bvh) || (mode != 1 && !sdf)) return HYB_ERR_INVALID_ARG;
    hyb_status rc = check_query(rays, n, tmax, hits);
    if (rc != HYB_OK || n == 0) return rc;
    if (!counts) return HYB_ERR_INVALID_ARG;
    if ((bvh && !same_device(bvh->device)) || (sdf && !same_device(sdf->device))) return HYB_ERR_INVALID_ARG;
    hyb::TraceArgs a;
    fill_trace_args(a, rays, hits, n, tmax, mode == 1 ? __builtin_inff() : (mode == 2 ? 0.0f : threshold),
                    mode == 3 ? threshold : 0.0f);
    fill_scene(a, mode == 2 ? nullptr : bvh, mode == 1 ? nullptr : sdf);
    a.counts = counts;
    return from_hip(hyb::launch_trace(mode, true, a, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
