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

// Largest cell gradient bound of the grid (cell_lipschitz) and largest
// per-axis slopes (cell_slopes), and whether any sample is not finite (fmaxf
// drops NaN, so that is tested on its own): kBoundValues values per block.
__global__ __launch_bounds__(256) void k_lipschitz(const float* __restrict__ g, int32_t n, float inv_h,
                                                   float* __restrict__ block_max) {
    constexpr int V = kBoundValues;
    __shared__ float red[V][256];
    const int64_t m = n - 1;
    float best[V] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < m * m * m; c += (int64_t)gridDim.x * 256) {
        const int64_t i = c % m, j = (c / m) % m, k = c / (m * m);
        const float* p = g + i + (int64_t)n * (j + (int64_t)n * k);
        const int64_t sy = n, sz = (int64_t)n * n;
        const float f[8] = {p[0], p[1], p[sy], p[sy + 1], p[sz], p[sz + 1], p[sz + sy], p[sz + sy + 1]};
        float s[3];
        cell_slopes(f, inv_h, s);
        best[0] = fmaxf(best[0], cell_lipschitz(f, inv_h));
        for (int a = 0; a < 3; ++a) best[1 + a] = fmaxf(best[1 + a], s[a]);
        for (int q = 0; q < 8; ++q)
            if (!(fabsf(f[q]) <= 3.402823466e38f)) best[4] = 1.0f;  // NaN or +-inf
    }
    for (int a = 0; a < V; ++a) red[a][threadIdx.x] = best[a];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int a = 0; a < V; ++a) red[a][threadIdx.x] = fmaxf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x < V) block_max[V * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// I8 block scales: one thread per block of 8^3 cells (its nodes [8b, 8b + 8]
// on each axis, a face shared with the next block): 2^e with e the smallest
// integer >= -126 such that max |f| <= 127 * 2^e (exact comparisons).
__global__ __launch_bounds__(256) void k_block_scales(const float* __restrict__ in, int32_t n, int32_t nb,
                                                      float* __restrict__ scales) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= (int64_t)nb * nb * nb) return;
    const int bi = (int)(b % nb), bj = (int)((b / nb) % nb), bk = (int)(b / ((int64_t)nb * nb));
    float m = 0.0f;
    for (int k = bk * kScaleBlock; k <= min(n - 1, (bk + 1) * kScaleBlock); ++k)
        for (int j = bj * kScaleBlock; j <= min(n - 1, (bj + 1) * kScaleBlock); ++j)
            for (int i = bi * kScaleBlock; i <= min(n - 1, (bi + 1) * kScaleBlock); ++i)
                m = fmaxf(m, fabsf(in[i + (int64_t)n * (j + (int64_t)n * k)]));
    int e = -126;
    if (m > 0.0f) {
        e = max(ilogbf(m) - 7, -126);  // 127 * 2^e < m here: 127 < 2^7
        while (ldexpf(127.0f, e) < m) ++e;
    }
    scales[b] = ldexpf(1.0f, e);
}

// The I8 blocks holding node i along one axis: lo to hi (equal unless the
// node lies on a face between two blocks).
__device__ inline void node_blocks(int i, int nb, int& lo, int& hi) {
    lo = min(max((i - 1) / kScaleBlock, 0), nb - 1);
    hi = min(i / kScaleBlock, nb - 1);
}

// One storage slot of the bricked layout: the sample of its node in the
// storage format (0 for padding slots).
template <int FMT>
__device__ void store_slot(const float* __restrict__ in, int32_t n, int32_t nb, int64_t s, void* __restrict__ out,
                           const float* __restrict__ scales) {
    int i, j, k;
    const bool node = Brick<FMT>::slot_node(s, n, i, j, k);
    const float f = node ? in[(int64_t)i + (int64_t)n * ((int64_t)j + (int64_t)n * k)] : 0.0f;
    if constexpr (FMT == kF32) {
        static_cast<float*>(out)[s] = f;
    } else if constexpr (FMT == kF16 || FMT == kF16B2) {
        static_cast<_Float16*>(out)[s] = (_Float16)f;
    } else {
        // `in` holds the dequantized values: a node's value is an integer
        // multiple of the scale of every block holding it, here the block of
        // the slot's cell (one-cell bricks: brick = cell); slots 8-11 of the
        // cell hold the bytes of that scale
        using B = Brick<kI8>;
        const int64_t b = s / B::kStride;
        const int r = (int)(s - b * B::kStride);
        const int nc = B::per_axis(n);
        const int ci = (int)(b % nc), cj = (int)((b / nc) % nc), ck = (int)(b / ((int64_t)nc * nc));
        const float sc = scales[ci / kScaleBlock + nb * (cj / kScaleBlock + nb * (ck / kScaleBlock))];
        uint8_t byte;
        if (r >= B::kNodes) byte = (uint8_t)(__builtin_bit_cast(uint32_t, sc) >> (8 * (r - B::kNodes)));
        else byte = node ? (uint8_t)(int8_t)(f / sc) : 0;
        static_cast<uint8_t*>(out)[s] = byte;
    }
}

// Every storage slot, in a grid-stride loop: the compact formats of a 1024^3
// grid have 8.6e9 slots, more work items than a launch can count (32 bits per
// dimension).
template <int FMT>
__global__ __launch_bounds__(256) void k_store(const float* __restrict__ in, int32_t n, int32_t nb, int64_t slots,
                                               void* __restrict__ out, const float* __restrict__ scales) {
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < slots; s += (int64_t)gridDim.x * 256)
        store_slot<FMT>(in, n, nb, s, out, scales);
}

// The dequantized FP32 value of every node, in place (linear order).
template <int FMT>
__global__ __launch_bounds__(256) void k_dequantize(float* __restrict__ values, int32_t n, int32_t nb,
                                                    const float* __restrict__ scales) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nn = (int64_t)n;
    if (id >= nn * nn * nn) return;
    const float f = values[id];
    if constexpr (FMT == kF16) {
        values[id] = (float)(_Float16)f;
    } else {
        // the largest and smallest scale of the 1 to 8 blocks holding the
        // node: code rint(f / s_max), clamped to what the smallest-scale
        // block can hold, times s_max (all exact: powers of two)
        const int i = (int)(id % nn), j = (int)((id / nn) % nn), k = (int)(id / (nn * nn));
        int il, ih, jl, jh, kl, kh;
        node_blocks(i, nb, il, ih);
        node_blocks(j, nb, jl, jh);
        node_blocks(k, nb, kl, kh);
        float smax = 0.0f, smin = __builtin_inff();
        for (int bk = kl; bk <= kh; ++bk)
            for (int bj = jl; bj <= jh; ++bj)
                for (int bi = il; bi <= ih; ++bi) {
                    const float sc = scales[bi + nb * (bj + nb * bk)];
                    smax = fmaxf(smax, sc);
                    smin = fminf(smin, sc);
                }
        const float lim = floorf(127.0f * (smin / smax));
        values[id] = fminf(fmaxf(rintf(f / smax), -lim), lim) * smax;
    }
}

}  // namespace

hipError_t launch_quantize(int fmt, float* values, int32_t n, void* out, float* scales, hipStream_t stream) {
    const int64_t total = (int64_t)n * n * n;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    const int64_t slots = brick_storage(fmt, n);
    const unsigned sblocks = (unsigned)std::min<int64_t>((slots + 255) / 256, int64_t(1) << 20);
    const int32_t nb = i8_blocks(n);
    if (fmt == kF32) {
        hipLaunchKernelGGL(k_store<kF32>, dim3(sblocks), dim3(256), 0, stream, values, n, nb, slots, out, scales);
    } else if (fmt == kF16) {
        hipLaunchKernelGGL(k_store<kF16>, dim3(sblocks), dim3(256), 0, stream, values, n, nb, slots, out, scales);
        hipLaunchKernelGGL(k_dequantize<kF16>, dim3(blocks), dim3(256), 0, stream, values, n, nb, scales);
    } else if (fmt == kF16B2) {
        hipLaunchKernelGGL(k_store<kF16B2>, dim3(sblocks), dim3(256), 0, stream, values, n, nb, slots, out, scales);
        hipLaunchKernelGGL(k_dequantize<kF16>, dim3(blocks), dim3(256), 0, stream, values, n, nb, scales);
    } else if (fmt == kI8) {
        const int64_t nbb = (int64_t)nb * nb * nb;
        hipLaunchKernelGGL(k_block_scales, dim3((unsigned)((nbb + 255) / 256)), dim3(256), 0, stream, values, n, nb,
                           scales);
        hipLaunchKernelGGL(k_dequantize<kI8>, dim3(blocks), dim3(256), 0, stream, values, n, nb, scales);
        hipLaunchKernelGGL(k_store<kI8>, dim3(sblocks), dim3(256), 0, stream, values, n, nb, slots, out, scales);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

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

// The step bounds from the per-block maxima of k_lipschitz, on the device:
// the same maxima and the same finishing as the host's (bit for bit).
// pass 0: only the non-finite flag; 1: bounds, the flag kept set by pass 0;
// 2: bounds and a fresh flag.
__global__ __launch_bounds__(256) void k_finish_bounds(const float* __restrict__ block_max, int32_t n_blocks,
                                                       int32_t pass, float two_e, float* __restrict__ out) {
    constexpr int V = kBoundValues;
    __shared__ float red[V][256];
    float m[V] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int b = threadIdx.x; b < n_blocks; b += 256)
        for (int c = 0; c < V; ++c) m[c] = fmaxf(m[c], block_max[V * b + c]);
    for (int c = 0; c < V; ++c) red[c][threadIdx.x] = m[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < V; ++c) red[c][threadIdx.x] = fmaxf(red[c][threadIdx.x], red[c][threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    bool bad = red[4][0] != 0.0f;
    for (int c = 0; c < 4; ++c) bad = bad || !(red[c][0] <= 3.402823466e38f);
    if (pass == 1) bad = bad || out[kBBad] != 0.0f;
    out[kBBad] = bad ? 1.0f : 0.0f;
    if (pass == 0) return;
    const float L = finish_lipschitz(red[0][0]);
    out[kBLipschitz] = L;
    out[kBInvL] = inv_step(L);
    out[kBSlopeX] = finish_slope(red[1][0]);
    out[kBSlopeY] = finish_slope(red[2][0]);
    out[kBSlopeZ] = finish_slope(red[3][0]);
    out[kBTwoE] = two_e;
}

hipError_t launch_finish_bounds(const float* block_max, int32_t n_blocks, int pass, float two_e, float* out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_finish_bounds, dim3(1), dim3(256), 0, stream, block_max, n_blocks, (int32_t)pass, two_e, out);
    return hipGetLastError();
}

hipError_t launch_lipschitz(const float* grid, int32_t n, float h, float* block_max, int32_t* n_blocks,
                            hipStream_t stream) {
    const int32_t b = lipschitz_blocks(n);
    *n_blocks = b;
    hipLaunchKernelGGL(k_lipschitz, dim3(b), dim3(256), 0, stream, grid, n, 1.0f / h, block_max);
    return hipGetLastError();
}

}  // namespace hyb
