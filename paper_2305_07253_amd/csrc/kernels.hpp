// Launchers of the device kernels (internal header shared by the C API).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyb {

enum TraceMode : int { kCombined = 0, kBvhOnly = 1, kDfOnly = 2, kShadow = 3 };

struct TraceArgs {
    // rays (device SoA)
    const float *ox, *oy, *oz, *dx, *dy, *dz, *tmin, *tmax_ray;
    // hits (device SoA)
    float* t;
    int32_t* prim;
    float *u, *v;
    int32_t* counts;  // 3 per ray or null
    // scene
    const float4* nodes;  // four-wide BVH
    const float4* tris;
    const int32_t* entry;  // traversal entry pyramid (null: start at the root)
    float entry_lo_x, entry_lo_y, entry_lo_z, entry_inv;  // origin, 1 / finest voxel side
    int32_t entry_res, entry_levels;
    const void* sdf;  // samples in the grid's storage format
    int32_t fmt;      // SdfFormat
    int32_t n_grid;
    float lo_x, lo_y, lo_z, h, inv_h, inv_l;
    float two_e;  // certified-grid step slack (+inf: use g / L only)
    float slope_x, slope_y, slope_z;  // per-axis bounds of the interpolant's partial derivatives
    // query
    float tmax, tau, tau_end;
    uint32_t xcd_run;  // blocks per die run of the trace kernels (xcd_block)
    int64_t n;
    double inv_hd;  // 1 / h in FP64 (scales the distance field's FP64 ray position)
    // Step bounds on the device (null: the fields above hold them): the grid
    // was last updated without a wait (kDeviceBounds floats, see
    // launch_finish_bounds)
    const float* bounds;
};

hipError_t launch_trace(int mode, bool counters, const TraceArgs& a, hipStream_t stream);

// Persistent multi-scene trace (combined query of every scene).  Work item w
// covers rays [(w - item_start[s]) * rays_per_item, ...) of the scene s with
// item_start[s] <= w < item_start[s + 1]; wavefronts take items from the
// global counter *queue (zero before the launch) until it passes n_items.
struct BatchArgs {
    const TraceArgs* scenes;     // device table, n_scenes entries
    const uint32_t* item_start;  // device, n_scenes + 1 entries, item_start[n_scenes] = n_items
    uint32_t* queue;             // device counter
    int32_t n_scenes;
    uint32_t n_items;
    int32_t rays_per_item;       // multiple of 64
};

// Kernel entry of the persistent trace for a storage format and LDS stack
// depth (8, 16 or 32 entries per lane), for launches and graph nodes; null
// for an unsupported pair.  Its dynamic LDS is batch_lds_bytes(lds_depth).
const void* batch_kernel(int fmt, int lds_depth);
size_t batch_lds_bytes(int lds_depth);
const void* queue_reset_kernel();  // one argument: uint32_t* counter, launch <<<1, 64>>>

// Count of rays whose result differs from a reference result: hit/miss
// differs, or both hit and the hit points are more than `h` apart
// (|t - t_ref| |d| > h).  Adds the count to *count.
hipError_t launch_count_mismatch(const float* t, const int32_t* prim, const float* t_ref, const int32_t* prim_ref,
                                 const float* dx, const float* dy, const float* dz, int64_t n, float h,
                                 unsigned long long* count, hipStream_t stream);

// The kernels' copy of an n^3 FP32 grid (x fastest): `out` receives
// brick_storage(fmt, n) samples in the format's bricked layout (slot s holds
// the node Brick<fmt>::slot_node(s)), in the storage format:
//   F32: the value
//   F16: round-to-nearest-even half of the value
//   I8:  scales[b] = the smallest power of two 2^e (e >= -126) with
//        127 * 2^e >= max |value| over the nodes of 8^3 block b; a node's
//        value becomes q * S, S the largest scale of the blocks holding it and
//        q = rint(value / S) clamped to +-floor(127 * smallest / S), an integer
//        multiple of every holding block's scale; each cell stores the codes of
//        its 8 corners for its own block's scale, then that scale
// For F16 / I8, `values` is then overwritten in place by the dequantized FP32
// values (what the trace kernels interpolate).
hipError_t launch_quantize(int fmt, float* values, int32_t n, void* out, float* scales, hipStream_t stream);

// Scatter of d loss / d grid sample for distance-field hits (hyb_df_backward):
// the rays are sorted by hit cell in `workspace` (device memory of at least
// df_backward_workspace(a.n, a.n_grid) bytes, which is 0 when the sort cannot
// be sized), and each wavefront adds once per cell.
size_t df_backward_workspace(int64_t n, int32_t n_grid);
hipError_t launch_df_backward(const TraceArgs& a, const float* t_hit, const float* grad_t, float* grad_grid,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

struct SdfBuildArgs {
    const float4* nodes;
    const float4* tris;
    int32_t n_grid;
    float lo_x, lo_y, lo_z, h;
    int32_t exterior_solid;
    float* out;  // n^3 floats, x fastest
};

hipError_t launch_sdf_build(const SdfBuildArgs& a, hipStream_t stream);

// Per-block maxima of the cell Lipschitz bounds and of the per-axis cell
// slopes of an n^3 grid (x fastest), and a flag for non-finite samples: block
// b writes block_max[5 b .. 5 b + 5) = (Lipschitz, slope x, slope y, slope z,
// 1 if some sample of its cells is NaN or infinite else 0); returns n_blocks
// through *n_blocks.
constexpr int kBoundValues = 5;
// The step bounds a deferred update leaves on the device: inv_l, slope_x,
// slope_y, slope_z, two_e, a flag (nonzero: a sample was not finite) and the
// Lipschitz bound itself.
constexpr int kDeviceBounds = 8;
enum DeviceBound : int { kBInvL = 0, kBSlopeX = 1, kBSlopeY = 2, kBSlopeZ = 3, kBTwoE = 4, kBBad = 5, kBLipschitz = 6 };
// Reduces the n_blocks per-block maxima of launch_lipschitz into the step
// bounds (out, kDeviceBounds floats), as the host does: pass 0 only the
// non-finite flag (a pass over the input of a compact format, before it is
// quantized), pass 1 all of them with the flag kept set by pass 0, pass 2 all
// of them with a fresh flag.  two_e: the certified-grid slack, or +inf.
hipError_t launch_finish_bounds(const float* block_max, int32_t n_blocks, int pass, float two_e, float* out,
                                hipStream_t stream);
hipError_t launch_lipschitz(const float* grid, int32_t n, float h, float* block_max, int32_t* n_blocks,
                            hipStream_t stream);
int32_t lipschitz_blocks(int32_t n);

}  // namespace hyb
