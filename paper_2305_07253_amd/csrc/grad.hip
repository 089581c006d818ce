// Backward of the distance-field hit distance (hyb_df_backward): one thread
// per ray recomputes its hit point from the forward t, the 8 implicit
// derivatives d t / d sample, and adds grad_t * derivative into the grid
// gradient with float atomics.
#include "hyb_device.hpp"
#include "kernels.hpp"

namespace hyb {
namespace {

__global__ __launch_bounds__(256) void k_df_backward(TraceArgs a, const float* __restrict__ t_hit,
                                                     const float* __restrict__ grad_t, float* __restrict__ grad_grid) {
    // every ray costs about the same here: one contiguous eighth of the rays
    // per die keeps the atomics of neighbouring hits in one L2
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x, max(gridDim.x / kXcds, 1u)) * 256 + threadIdx.x;
    if (i >= a.n) return;
    const float gt = grad_t[i];
    if (gt == 0.0f) return;
    const float tmin = a.tmin ? a.tmin[i] : 0.0f;
    const float tmax = a.tmax_ray ? fminf(a.tmax_ray[i], a.tmax) : a.tmax;
    if (!(tmin <= tmax)) return;
    const Grid g = grid_of(a);
    int64_t node[8];
    float dt[8];
    if (!df_hit_gradient(g, a.ox[i], a.oy[i], a.oz[i], a.dx[i], a.dy[i], a.dz[i], tmin, tmax, t_hit[i], node, dt))
        return;
    for (int c = 0; c < 8; ++c) unsafeAtomicAdd(grad_grid + node[c], gt * dt[c]);
}

}  // namespace

hipError_t launch_df_backward(const TraceArgs& a, const float* t_hit, const float* grad_t, float* grad_grid,
                              hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_df_backward, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, stream, a, t_hit, grad_t,
                       grad_grid);
    return hipGetLastError();
}

}  // namespace hyb
