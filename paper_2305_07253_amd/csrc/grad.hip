// Backward of the distance-field hit distance (hyb_df_backward): for every
// ray with a crossing, the 8 implicit derivatives d t / d sample of the
// corners of its hit cell, times grad_t, added into the grid gradient.
//
// The float atomic adds are nearly the whole cost of a plain scatter (8 per
// hit; recomputing the hits is a few percent of it), and the cost is per add.
// Hits cluster in cells (on a G-buffer-shaped refit several rays end in each
// touched cell), so the rays are keyed by hit cell and radix-sorted, and each
// wavefront sums the contributions of consecutive equal keys before the last
// lane of each run adds them: 8 adds per (wavefront, cell) instead of per
// ray.
#include <rocprim/device/device_radix_sort.hpp>

#include "hyb_device.hpp"
#include "kernels.hpp"

namespace hyb {
namespace {

constexpr int kBwdBlock = 256;

// The (cell, ray) pairs are sorted by rocPRIM's onesweep radix sort from 64k
// pairs up: its default switches to a block sort plus merge passes up to 1M
// pairs, which took 154 us of a 241 us backward on 1M rays (ten merge
// passes) where onesweep takes three passes over 22-bit keys.
using BwdSortConfig =
    rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config, rocprim::default_config, 65536>;

// Contributions of ray i (grad_t times d t / d sample of its cell's 8
// corners, corner order of `corners`) and the linear index of the cell's
// corner 0; false when the ray adds nothing.
HYB_HD bool ray_gradient(const TraceArgs& a, const Grid& g, int64_t i, const float* __restrict__ t_hit,
                         const float* __restrict__ grad_t, int64_t& cell, float v[8]) {
    const float gt = grad_t[i];
    if (gt == 0.0f) return false;
    const float tmin = a.tmin ? a.tmin[i] : 0.0f;
    const float tmax = a.tmax_ray ? fminf(a.tmax_ray[i], a.tmax) : a.tmax;
    if (!(tmin <= tmax)) return false;
    int64_t node[8];
    float dt[8];
    if (!df_hit_gradient(g, a.ox[i], a.oy[i], a.oz[i], a.dx[i], a.dy[i], a.dz[i], tmin, tmax, t_hit[i], node, dt))
        return false;
    for (int c = 0; c < 8; ++c) v[c] = gt * dt[c];
    cell = node[0];
    return true;
}

// Sort keys: the hit cell's corner-0 index (below n^3), or `none` (= n^3) for
// a ray that adds nothing; the values are the ray indices.
__global__ __launch_bounds__(kBwdBlock) void k_bwd_keys(TraceArgs a, const float* __restrict__ t_hit,
                                                        const float* __restrict__ grad_t, uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ rays, uint32_t none) {
    const int64_t i = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x;
    if (i >= a.n) return;
    const Grid g = grid_of(a);
    int64_t cell = 0;
    float v[8];
    keys[i] = ray_gradient(a, g, i, t_hit, grad_t, cell, v) ? (uint32_t)cell : none;
    rays[i] = (uint32_t)i;
}

// Over the sorted keys: each lane recomputes its ray's contributions, the
// wavefront forms inclusive sums over runs of equal keys (the keys are
// sorted, so two lanes with equal keys bound a run of them), and the last
// lane of each run adds the run's sums at the cell's 8 corners.  Every lane
// of a launched wavefront takes part in the shuffles; lanes past n carry
// `none`.
__global__ __launch_bounds__(kBwdBlock) void k_bwd_runs(TraceArgs a, const float* __restrict__ t_hit,
                                                        const float* __restrict__ grad_t,
                                                        const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ rays,
                                                        float* __restrict__ grad_grid, uint32_t none) {
    const int64_t j = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x;
    const uint32_t key = j < a.n ? keys[j] : none;
    float v[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (key != none) {
        const Grid g = grid_of(a);
        int64_t cell = 0;
        // the same computation as for the key: it succeeds again; the corners
        // the run adds at come from the key alone
        if (!ray_gradient(a, g, rays[j], t_hit, grad_t, cell, v))
            for (int c = 0; c < 8; ++c) v[c] = 0.0f;
    }
    // every shuffle runs on all 64 lanes (a lane reads its source's value
    // only while the source is active), so none sits behind a condition
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t up = __shfl_up(key, o);
        const bool same = lane >= o && up == key;
        for (int c = 0; c < 8; ++c) {
            const float w = __shfl_up(v[c], o);
            if (same) v[c] += w;
        }
    }
    const uint32_t next = __shfl_down(key, 1);
    const bool last = lane == 63 || next != key;
    if (key == none || !last) return;
    const int64_t n = a.n_grid;
    for (int c = 0; c < 8; ++c) {
        const int64_t node = (int64_t)key + (c & 1) + n * (((c >> 1) & 1) + n * (c >> 2));
        unsafeAtomicAdd(grad_grid + node, v[c]);
    }
}

uint32_t key_none(int32_t n_grid) { return (uint32_t)((int64_t)n_grid * n_grid * n_grid); }

int key_bits(int32_t n_grid) {
    const uint32_t none = key_none(n_grid);
    return 32 - __builtin_clz(none);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t sort_temp_bytes(int64_t n, int32_t n_grid) {
    size_t bytes = 0;
    rocprim::double_buffer<uint32_t> keys(nullptr, nullptr), rays(nullptr, nullptr);
    const hipError_t e = rocprim::radix_sort_pairs<BwdSortConfig>(nullptr, bytes, keys, rays, static_cast<int>(n), 0,
                                                                  key_bits(n_grid), hipStream_t(nullptr));
    return e == hipSuccess ? bytes : 0;
}

}  // namespace

size_t df_backward_workspace(int64_t n, int32_t n_grid) {
    if (n <= 0) return 0;
    const size_t t = sort_temp_bytes(n, n_grid);
    if (t == 0) return 0;
    return 4 * align256(sizeof(uint32_t) * (size_t)n) + align256(t);
}

hipError_t launch_df_backward(const TraceArgs& a, const float* t_hit, const float* grad_t, float* grad_grid,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    // four arrays of n words (keys and ray indices, each twice for the sort's
    // passes), then the sort's scratch: the caller sized it with
    // df_backward_workspace(a.n, a.n_grid)
    const size_t arr = align256(sizeof(uint32_t) * (size_t)a.n);
    if (!workspace || workspace_bytes <= 4 * arr) return hipErrorInvalidValue;
    char* p = static_cast<char*>(workspace);
    rocprim::double_buffer<uint32_t> keys(reinterpret_cast<uint32_t*>(p), reinterpret_cast<uint32_t*>(p + arr));
    rocprim::double_buffer<uint32_t> rays(reinterpret_cast<uint32_t*>(p + 2 * arr),
                                          reinterpret_cast<uint32_t*>(p + 3 * arr));
    size_t temp_bytes = workspace_bytes - 4 * arr;
    const uint32_t none = key_none(a.n_grid);
    const unsigned blocks = (unsigned)((a.n + kBwdBlock - 1) / kBwdBlock);
    hipLaunchKernelGGL(k_bwd_keys, dim3(blocks), dim3(kBwdBlock), 0, stream, a, t_hit, grad_t, keys.current(),
                       rays.current(), none);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = rocprim::radix_sort_pairs<BwdSortConfig>(p + 4 * arr, temp_bytes, keys, rays, static_cast<int>(a.n), 0,
                                                 key_bits(a.n_grid), stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bwd_runs, dim3(blocks), dim3(kBwdBlock), 0, stream, a, t_hit, grad_t, keys.current(),
                       rays.current(), grad_grid, none);
    return hipGetLastError();
}

}  // namespace hyb
