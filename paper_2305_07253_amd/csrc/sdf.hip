// Distance-field construction from the triangle BVH (build time, not the hot
// path): one thread per grid node computes the exact signed distance in FP64
// (sdf_node_value) and rounds it once to FP32; a second kernel reduces the
// Lipschitz bound of the stored grid.
#include "kernels.hpp"
#include "sdf_device.hpp"

namespace hyb {
namespace {

__global__ __launch_bounds__(256) void k_sdf_build(SdfBuildArgs a) {
    const int64_t n = a.n_grid;
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= n * n * n) return;
    const int64_t i = id % n, j = (id / n) % n, k = id / (n * n);
    const D3 p = d3((double)a.lo_x + (double)i * (double)a.h, (double)a.lo_y + (double)j * (double)a.h,
                    (double)a.lo_z + (double)k * (double)a.h);
    a.out[id] = (float)sdf_node_value(a.nodes, a.tris, p, a.exterior_solid);
}

// Largest cell gradient bound of the grid (cell_lipschitz), one value per block.
__global__ __launch_bounds__(256) void k_lipschitz(const float* __restrict__ g, int32_t n, float inv_h,
                                                   float* __restrict__ block_max) {
    __shared__ float red[256];
    const int64_t m = n - 1;
    float best = 0.0f;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < m * m * m; c += (int64_t)gridDim.x * 256) {
        const int64_t i = c % m, j = (c / m) % m, k = c / (m * m);
        const float* p = g + i + (int64_t)n * (j + (int64_t)n * k);
        const int64_t sy = n, sz = (int64_t)n * n;
        const float f[8] = {p[0], p[1], p[sy], p[sy + 1], p[sz], p[sz + 1], p[sz + sy], p[sz + sy + 1]};
        best = fmaxf(best, cell_lipschitz(f, inv_h));
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

}  // namespace

hipError_t launch_sdf_build(const SdfBuildArgs& a, hipStream_t stream) {
    const int64_t total = (int64_t)a.n_grid * a.n_grid * a.n_grid;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_sdf_build, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

int32_t lipschitz_blocks(int32_t n) {
    const int64_t m = (int64_t)(n - 1) * (n - 1) * (n - 1);
    int64_t b = (m + 255) / 256;
    return (int32_t)(b < 2048 ? b : 2048);
}

hipError_t launch_lipschitz(const float* grid, int32_t n, float h, float* block_max, int32_t* n_blocks,
                            hipStream_t stream) {
    const int32_t b = lipschitz_blocks(n);
    *n_blocks = b;
    hipLaunchKernelGGL(k_lipschitz, dim3(b), dim3(256), 0, stream, grid, n, 1.0f / h, block_max);
    return hipGetLastError();
}

}  // namespace hyb
