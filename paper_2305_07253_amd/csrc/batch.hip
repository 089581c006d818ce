// Many scenes in one launch: a persistent trace kernel fed by a global work
// queue, the batch handle behind hyb_batch_* (include/hyb.h) with its device
// descriptor table and HIP graph, and the autotuner that picks each scene's
// switch threshold and the launch shape.
//
// The combined query itself (Section 2, Eq. (2)) is the same per-ray code as
// hyb_trace; only the mapping of rays to wavefronts differs.  Every wavefront
// takes work items (a run of rays_per_item consecutive rays of one scene) from
// a device counter until the counter passes the last item, so scenes of very
// different sizes share the chip without a tail per scene.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "api_internal.hpp"

namespace hyb {

namespace {

constexpr int kWave = 64;

// FP32: six wavefronts per SIMD (at most 80 VGPRs); left to itself the
// compiler takes 83 registers and runs five, 6% slower on the 64-scene batch.
// The compact formats would spill at six and keep five.
template <int FMT, int LDS>
__global__ __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(FMT == kF32 ? 6 : 5))) void k_trace_batch(
    BatchArgs b, const TraceArgs* __restrict__ scenes) {
    extern __shared__ int s_stack[];
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        uint32_t w = 0;
        if (lane == 0) w = atomicAdd(b.queue, 1u);
        w = __builtin_amdgcn_readfirstlane(__shfl(w, 0, kWave));
        if (w >= b.n_items) return;  // every wavefront ends here once the queue has passed n_items
        // scene s with item_start[s] <= w < item_start[s + 1] (empty scenes own no item)
        int lo = 0, hi = b.n_scenes;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (b.item_start[mid] <= w) lo = mid;
            else hi = mid;
        }
        // The scene's arguments are the same for the whole wavefront (lo is
        // uniform) and the table is never written by the kernel: its fields
        // are read with scalar loads where they are used.
        const TraceArgs& a = scenes[__builtin_amdgcn_readfirstlane(lo)];
        const int64_t base = (int64_t)(w - b.item_start[lo]) * b.rays_per_item;
        for (int k = 0; k < b.rays_per_item; k += kWave) {
            const int64_t i = base + k + lane;
            if (i >= a.n) continue;
            // F16 scenes may differ in brick layout (a.fmt is the same for
            // the whole wavefront)
            if (FMT == kF16 && a.fmt == kF16B2)
                trace_ray<kCombined, kF16B2, false, LDS>(a, i, s_stack + threadIdx.x, kBatchBlock);
            else
                trace_ray<kCombined, FMT, false, LDS>(a, i, s_stack + threadIdx.x, kBatchBlock);
        }
    }
}

__global__ void k_queue_reset(uint32_t* counter) {
    if (threadIdx.x == 0) counter[0] = 0u;
}

__global__ __launch_bounds__(kBatchBlock) void k_count_mismatch(const float* __restrict__ t, const int32_t* __restrict__ prim,
                                                          const float* __restrict__ t_ref,
                                                          const int32_t* __restrict__ prim_ref,
                                                          const float* __restrict__ dx, const float* __restrict__ dy,
                                                          const float* __restrict__ dz, int64_t n, float h,
                                                          unsigned long long* count) {
    __shared__ unsigned int s_sum[kBatchBlock / kWave];
    unsigned int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBatchBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBatchBlock) {
        const bool hit = prim[i] != -1, hit_ref = prim_ref[i] != -1;
        if (hit != hit_ref) {
            ++c;
        } else if (hit) {
            const float len = sqrtf(dx[i] * dx[i] + dy[i] * dy[i] + dz[i] * dz[i]);
            if (fabsf(t[i] - t_ref[i]) * len > h) ++c;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_sum[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int k = 0; k < kBatchBlock / kWave; ++k) s += s_sum[k];
        if (s) atomicAdd(count, s);
    }
}

// The fixed device array of hyb_batch_launch_static: the work counter, the
// item offsets and the descriptor table of up to kStaticItems items, laid out
// at the offsets below (one copy per device, held until the process ends).
constexpr int kStaticItems = HYB_STATIC_BATCH_MAX_ITEMS;
constexpr size_t kStaticQueueOff = 0;
constexpr size_t kStaticStartOff = 256;
constexpr size_t kStaticTableOff = 1536;
constexpr size_t kStaticBytes = kStaticTableOff + sizeof(TraceArgs) * kStaticItems;
static_assert(kStaticStartOff + sizeof(uint32_t) * (kStaticItems + 1) <= kStaticTableOff, "offsets overlap");
static_assert(sizeof(TraceArgs) % sizeof(uint32_t) == 0 && alignof(TraceArgs) <= 256, "table layout");
static_assert(kStaticBytes == 65024, "the array size hyb_batch_launch_static documents");
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Words of host data carried by value in one kernel's arguments (kept under
// the 4 KiB argument limit), written to base[offset ...): how the host fills
// the fixed array without a copy from host memory.
constexpr uint32_t kFillWords = 960;
struct FillChunk {
    uint32_t offset, count;
    uint32_t words[kFillWords];
};

__global__ void k_fill_words(uint32_t* __restrict__ base, FillChunk c) {
    for (uint32_t i = threadIdx.x; i < c.count; i += blockDim.x) base[c.offset + i] = c.words[i];
}

}  // namespace

// Host address of this device's copy of the fixed array (hipGetSymbolAddress
// once per device, with that device current; the array's name is only a
// host-side stand-in), and the device's compute-unit count.
hipError_t static_scratch(int device, void** ptr, int* n_cu) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    static int cus[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        int c = 0;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device);
        if (e != hipSuccess) return e;
        addr[device] = p;
        cus[device] = c;
    }
    *ptr = addr[device];
    *n_cu = cus[device];
    return hipSuccess;
}

// Copies `words` 32-bit words from host memory to dst_words (a word offset
// into the array at base) through k_fill_words launches on `stream`.
hipError_t fill_static(uint32_t* base, uint32_t dst_words, const void* src, size_t words, hipStream_t stream) {
    FillChunk c;
    const uint32_t* w = static_cast<const uint32_t*>(src);
    for (size_t done = 0; done < words; done += kFillWords) {
        c.offset = dst_words + static_cast<uint32_t>(done);
        c.count = static_cast<uint32_t>(std::min<size_t>(kFillWords, words - done));
        std::memcpy(c.words, w + done, sizeof(uint32_t) * c.count);
        hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(256), 0, stream, base, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

const void* batch_kernel(int fmt, int lds_depth) {
#define HYB_BATCH_CASE(F, D) \
    if (fmt == F && lds_depth == D) return reinterpret_cast<const void*>(&k_trace_batch<F, D>);
    HYB_BATCH_CASE(kF32, 8)
    HYB_BATCH_CASE(kF32, 16)
    HYB_BATCH_CASE(kF32, 32)
    HYB_BATCH_CASE(kF16, 8)
    HYB_BATCH_CASE(kF16, 16)
    HYB_BATCH_CASE(kF16, 32)
    HYB_BATCH_CASE(kI8, 8)
    HYB_BATCH_CASE(kI8, 16)
    HYB_BATCH_CASE(kI8, 32)
#undef HYB_BATCH_CASE
    return nullptr;
}

size_t batch_lds_bytes(int lds_depth) { return sizeof(int) * (size_t)lds_depth * kBatchBlock; }

const void* queue_reset_kernel() { return reinterpret_cast<const void*>(&k_queue_reset); }

hipError_t launch_count_mismatch(const float* t, const int32_t* prim, const float* t_ref, const int32_t* prim_ref,
                                 const float* dx, const float* dy, const float* dz, int64_t n, float h,
                                 unsigned long long* count, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBatchBlock - 1) / kBatchBlock, 4096);
    hipLaunchKernelGGL(k_count_mismatch, dim3((unsigned)blocks), dim3(kBatchBlock), 0, stream, t, prim, t_ref, prim_ref, dx,
                       dy, dz, n, h, count);
    return hipGetLastError();
}

}  // namespace hyb

// ---------------------------------------------------------------------------
// batch handle
// ---------------------------------------------------------------------------

using namespace hyb_api;

namespace {

enum ItemKind : uint8_t { kBoth = 0, kTrianglesOnly = 1, kFieldOnly = 2 };

constexpr int32_t kMaxItems = 1 << 16;
constexpr uint32_t kMaxWorkItems = 1u << 31;

}  // namespace

struct hyb_batch_s {
    int device = 0;
    int fmt = hyb::kF32;
    int n_cu = 0;
    std::vector<hyb::TraceArgs> args;  // per item; tau is the item's current threshold
    std::vector<uint8_t> kind;
    std::vector<const hyb_sdf_s*> sdfs;  // per item (null: triangles only)
    std::vector<uint64_t> sdf_version;   // each sdf's version when its fields were copied into args
    std::vector<uint32_t> item_start;  // host copy for the current rays_per_item
    hyb::TraceArgs* d_args = nullptr;
    uint32_t* d_item_start = nullptr;
    uint32_t* d_queue = nullptr;
    hyb_batch_config cfg = {16, 256, 4};
    bool table_dirty = true, graph_dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hyb::BatchArgs kargs = {};
    dim3 grid = dim3(0);
    int32_t graph_lds = 0;
};

namespace {

bool valid_config(const hyb_batch_config& c) {
    return (c.lds_depth == 8 || c.lds_depth == 16 || c.lds_depth == 32) && c.rays_per_item >= 64 &&
           c.rays_per_item <= 65536 && c.rays_per_item % 64 == 0 && c.blocks_per_cu >= 1 && c.blocks_per_cu <= 16;
}

// Validation shared by hyb_batch_create and hyb_batch_launch_static: every
// item as hyb_trace would check it, all sdfs of one storage format (returned
// through *fmt, the batch kernel's format).
hyb_status check_items(const hyb_batch_item* items, int32_t n_items, int* fmt_out) {
    int fmt = -1;
    for (int32_t i = 0; i < n_items; ++i) {
        const hyb_batch_item& it = items[i];
        if (!it.bvh && !it.sdf) return HYB_ERR_INVALID_ARG;
        if (std::isnan(it.threshold) || it.threshold < 0.0f) return HYB_ERR_INVALID_ARG;
        if (!it.bvh && it.threshold != 0.0f) return HYB_ERR_INVALID_ARG;
        if (!it.sdf && !std::isinf(it.threshold)) return HYB_ERR_INVALID_ARG;
        hyb_status rc = check_query(&it.rays, it.n, it.tmax, const_cast<hyb_hits*>(&it.hits));
        if (rc != HYB_OK) return rc;
        if ((it.bvh && !same_device(it.bvh->device)) || (it.sdf && !same_device(it.sdf->device)))
            return HYB_ERR_INVALID_ARG;
        if (it.sdf) {
            if (fmt >= 0 && fmt != static_cast<int>(it.sdf->fmt)) return HYB_ERR_UNSUPPORTED;
            fmt = static_cast<int>(it.sdf->fmt);
        }
    }
    *fmt_out = fmt < 0 ? hyb::kF32 : fmt;
    return HYB_OK;
}

// The arguments of one item's query, as the batch's descriptor table holds them.
void item_args(const hyb_batch_item& it, hyb::TraceArgs& a) {
    fill_trace_args(a, &it.rays, const_cast<hyb_hits*>(&it.hits), it.n, it.tmax, it.threshold);
    fill_scene(a, it.bvh, it.sdf);
    if (!it.sdf) a.h = 1.0f;  // t1 = fma(+inf, h, tmin) must be +inf (then min(., tmax) = tmax), not NaN
}

// Blocks of the persistent launch: as many as the GPU holds at the config's
// blocks per CU (capped by occupancy), never more than the work needs.
hyb_status persistent_grid(int fmt, const hyb_batch_config& cfg, int n_cu, uint64_t work_items, dim3* grid) {
    const void* fn = hyb::batch_kernel(fmt, cfg.lds_depth);
    if (!fn) return HYB_ERR_UNSUPPORTED;
    int occ = 0;
    HYB_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, hyb::kBatchBlock, hyb::batch_lds_bytes(cfg.lds_depth)));
    const int64_t per_cu = std::max(1, std::min(occ, cfg.blocks_per_cu));
    const int64_t waves_needed = (static_cast<int64_t>(work_items) + 3) / 4;  // 4 wavefronts per block
    *grid = dim3(static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(per_cu * n_cu, waves_needed))));
    return HYB_OK;
}

void drop_graph(hyb_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_dirty = true;
}

// A grid replaced in place (hyb_sdf_update) has new step bounds and possibly
// a new certification: copy its fields into the item's arguments again.
void refresh_grids(hyb_batch_s* b) {
    for (size_t i = 0; i < b->sdfs.size(); ++i) {
        const hyb_sdf_s* sdf = b->sdfs[i];
        if (sdf && sdf->version != b->sdf_version[i]) {
            fill_scene(b->args[i], nullptr, sdf);
            b->sdf_version[i] = sdf->version;
            b->table_dirty = true;
        }
    }
}

// Uploads the descriptor table and the item offsets for the current config and
// fixes the launch grid (synchronous on `stream`).
hyb_status sync_table(hyb_batch_s* b, hipStream_t stream) {
    refresh_grids(b);
    if (!b->table_dirty) return HYB_OK;
    const int32_t n_scenes = static_cast<int32_t>(b->args.size());
    uint64_t total = 0;
    for (int32_t s = 0; s < n_scenes; ++s) {
        b->item_start[s] = static_cast<uint32_t>(total);
        total += (static_cast<uint64_t>(b->args[s].n) + b->cfg.rays_per_item - 1) / b->cfg.rays_per_item;
        if (total >= kMaxWorkItems) return HYB_ERR_UNSUPPORTED;
    }
    b->item_start[n_scenes] = static_cast<uint32_t>(total);
    HYB_TRY(hipMemcpyAsync(b->d_args, b->args.data(), sizeof(hyb::TraceArgs) * n_scenes, hipMemcpyHostToDevice, stream));
    HYB_TRY(hipMemcpyAsync(b->d_item_start, b->item_start.data(), sizeof(uint32_t) * (n_scenes + 1),
                           hipMemcpyHostToDevice, stream));
    HYB_TRY(hipStreamSynchronize(stream));

    dim3 grid;
    const hyb_status gs = persistent_grid(b->fmt, b->cfg, b->n_cu, total, &grid);
    if (gs != HYB_OK) return gs;
    const int64_t blocks = grid.x;
    // The graph's kernel nodes hold the launch shape and BatchArgs by value;
    // a change of thresholds alone only rewrites the device table.
    const bool same_shape = b->grid.x == static_cast<unsigned>(blocks) && b->kargs.n_items == total &&
                            b->kargs.rays_per_item == b->cfg.rays_per_item && b->graph_lds == b->cfg.lds_depth;
    b->grid = dim3(static_cast<unsigned>(blocks));
    b->kargs.scenes = b->d_args;
    b->kargs.item_start = b->d_item_start;
    b->kargs.queue = b->d_queue;
    b->kargs.n_scenes = n_scenes;
    b->kargs.n_items = static_cast<uint32_t>(total);
    b->kargs.rays_per_item = b->cfg.rays_per_item;
    b->table_dirty = false;
    if (!same_shape) drop_graph(b);
    b->graph_lds = b->cfg.lds_depth;
    return HYB_OK;
}

hipError_t launch_eager(hyb_batch_s* b, hipStream_t stream) {
    void* reset_args[] = {&b->d_queue};
    hipError_t e = hipLaunchKernel(hyb::queue_reset_kernel(), dim3(1), dim3(64), reset_args, 0, stream);
    if (e != hipSuccess || b->kargs.n_items == 0) return e;
    const hyb::TraceArgs* scenes = b->d_args;
    void* trace_args[] = {&b->kargs, &scenes};
    return hipLaunchKernel(hyb::batch_kernel(b->fmt, b->cfg.lds_depth), b->grid, dim3(hyb::kBatchBlock), trace_args,
                           hyb::batch_lds_bytes(b->cfg.lds_depth), stream);
}

// Two explicit kernel nodes: the queue reset (a fill kernel, so replays of the
// graph never depend on a memset node) and the persistent trace after it.
hipError_t build_graph(hyb_batch_s* b) {
    hipError_t e = hipGraphCreate(&b->graph, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t reset_node = nullptr, trace_node = nullptr;
    void* reset_args[] = {&b->d_queue};
    hipKernelNodeParams p0;
    std::memset(&p0, 0, sizeof(p0));
    p0.func = const_cast<void*>(hyb::queue_reset_kernel());
    p0.gridDim = dim3(1);
    p0.blockDim = dim3(64);
    p0.kernelParams = reset_args;
    e = hipGraphAddKernelNode(&reset_node, b->graph, nullptr, 0, &p0);
    const hyb::TraceArgs* scenes = b->d_args;
    if (e == hipSuccess && b->kargs.n_items > 0) {
        void* trace_args[] = {&b->kargs, &scenes};
        hipKernelNodeParams p1;
        std::memset(&p1, 0, sizeof(p1));
        p1.func = const_cast<void*>(hyb::batch_kernel(b->fmt, b->cfg.lds_depth));
        p1.gridDim = b->grid;
        p1.blockDim = dim3(hyb::kBatchBlock);
        p1.sharedMemBytes = static_cast<unsigned>(hyb::batch_lds_bytes(b->cfg.lds_depth));
        p1.kernelParams = trace_args;
        e = hipGraphAddKernelNode(&trace_node, b->graph, &reset_node, 1, &p1);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return e;
    }
    b->graph_dirty = false;
    return hipSuccess;
}

// Milliseconds of the fastest of `reps` runs of fn (after one warm-up run).
template <class Fn>
hyb_status time_min(Fn&& fn, int reps, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, float* ms) {
    HYB_TRY(fn());
    float best = std::numeric_limits<float>::infinity();
    for (int r = 0; r < reps; ++r) {
        HYB_TRY(hipEventRecord(e0, stream));
        HYB_TRY(fn());
        HYB_TRY(hipEventRecord(e1, stream));
        HYB_TRY(hipEventSynchronize(e1));
        float t = 0.0f;
        HYB_TRY(hipEventElapsedTime(&t, e0, e1));
        best = std::min(best, t);
    }
    *ms = best;
    return HYB_OK;
}

// Threshold of one item: the fastest candidate whose results differ from the
// triangles-only results on at most max_error_rate of the item's rays
// (+inf, the exact triangle query, when none qualifies).
hyb_status tune_item_threshold(hyb_batch_s* b, int32_t item, const std::vector<float>& cands, float max_error_rate,
                               int reps, void* scratch, unsigned long long* d_count, hipStream_t stream,
                               hipEvent_t e0, hipEvent_t e1, float* err_out) {
    hyb::TraceArgs a = b->args[item];
    const int64_t n = a.n;
    hyb::TraceArgs ref = a;
    ref.t = static_cast<float*>(scratch);
    ref.prim = reinterpret_cast<int32_t*>(ref.t + n);
    ref.u = reinterpret_cast<float*>(ref.prim + n);
    ref.v = ref.u + n;
    ref.tau = __builtin_inff();
    HYB_TRY(hyb::launch_trace(hyb::kBvhOnly, false, ref, stream));
    float best_tau = __builtin_inff(), best_ms = std::numeric_limits<float>::infinity(), best_err = 0.0f;
    for (float c : cands) {
        a.tau = c;
        float ms = 0.0f;
        hyb_status rc = time_min([&] { return hyb::launch_trace(hyb::kCombined, false, a, stream); }, reps, stream,
                                 e0, e1, &ms);
        if (rc != HYB_OK) return rc;
        HYB_TRY(hipMemsetAsync(d_count, 0, sizeof(unsigned long long), stream));
        HYB_TRY(hyb::launch_count_mismatch(a.t, a.prim, ref.t, ref.prim, a.dx, a.dy, a.dz, n, a.h, d_count, stream));
        unsigned long long bad = 0;
        HYB_TRY(hipMemcpyAsync(&bad, d_count, sizeof(bad), hipMemcpyDeviceToHost, stream));
        HYB_TRY(hipStreamSynchronize(stream));
        const float err = static_cast<float>(static_cast<double>(bad) / static_cast<double>(n));
        if (err <= max_error_rate && ms < best_ms) {
            best_ms = ms;
            best_tau = c;
            best_err = err;
        }
    }
    b->args[item].tau = best_tau;
    if (err_out) *err_out = best_err;
    return HYB_OK;
}

}  // namespace

extern "C" {

hyb_status hyb_batch_create(const hyb_batch_item* items, int32_t n_items, void* stream, hyb_batch* out) {
    if (!out) return HYB_ERR_INVALID_ARG;
    *out = nullptr;
    if (!items || n_items < 1 || n_items > kMaxItems) return HYB_ERR_INVALID_ARG;
    int fmt = 0;
    const hyb_status checked = check_items(items, n_items, &fmt);
    if (checked != HYB_OK) return checked;
    int dev = 0;
    HYB_TRY(hipGetDevice(&dev));
    hyb_batch_s* b = new (std::nothrow) hyb_batch_s;
    if (!b) return HYB_ERR_OOM;
    b->device = dev;
    b->fmt = fmt;
    b->args.resize(n_items);
    b->kind.resize(n_items);
    b->sdfs.resize(n_items);
    b->sdf_version.resize(n_items);
    b->item_start.resize(n_items + 1);
    for (int32_t i = 0; i < n_items; ++i) {
        const hyb_batch_item& it = items[i];
        item_args(it, b->args[i]);
        b->kind[i] = !it.sdf ? kTrianglesOnly : (!it.bvh ? kFieldOnly : kBoth);
        b->sdfs[i] = it.sdf;
        b->sdf_version[i] = it.sdf ? it.sdf->version : 0;
    }
    hipError_t e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc(&b->d_args, sizeof(hyb::TraceArgs) * n_items);
    if (e == hipSuccess) e = hipMalloc(&b->d_item_start, sizeof(uint32_t) * (n_items + 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_queue, sizeof(uint32_t) * 64);
    hyb_status rc = from_hip(e);
    if (rc == HYB_OK) rc = sync_table(b, static_cast<hipStream_t>(stream));
    if (rc != HYB_OK) {
        hyb_batch_destroy(b);
        return rc;
    }
    *out = b;
    return HYB_OK;
}

hyb_status hyb_batch_set_config(hyb_batch batch, const hyb_batch_config* config) {
    if (!batch || !config || !valid_config(*config)) return HYB_ERR_INVALID_ARG;
    if (std::memcmp(&batch->cfg, config, sizeof(*config)) != 0) {
        batch->cfg = *config;
        batch->table_dirty = true;
    }
    return HYB_OK;
}

hyb_status hyb_batch_get_config(hyb_batch batch, hyb_batch_config* config) {
    if (!batch || !config) return HYB_ERR_INVALID_ARG;
    *config = batch->cfg;
    return HYB_OK;
}

hyb_status hyb_batch_set_threshold(hyb_batch batch, int32_t item, float threshold) {
    if (!batch || item < 0 || item >= static_cast<int32_t>(batch->args.size()) || std::isnan(threshold) ||
        threshold < 0.0f)
        return HYB_ERR_INVALID_ARG;
    const uint8_t k = batch->kind[item];
    if ((k == kTrianglesOnly && !std::isinf(threshold)) || (k == kFieldOnly && threshold != 0.0f))
        return HYB_ERR_INVALID_ARG;
    if (batch->args[item].tau != threshold) {
        batch->args[item].tau = threshold;
        batch->table_dirty = true;
    }
    return HYB_OK;
}

hyb_status hyb_batch_get_threshold(hyb_batch batch, int32_t item, float* threshold) {
    if (!batch || !threshold || item < 0 || item >= static_cast<int32_t>(batch->args.size()))
        return HYB_ERR_INVALID_ARG;
    *threshold = batch->args[item].tau;
    return HYB_OK;
}

hyb_status hyb_batch_launch(hyb_batch batch, void* stream) {
    if (!batch) return HYB_ERR_INVALID_ARG;
    if (!same_device(batch->device)) return HYB_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hyb_status rc = sync_table(batch, st);
    if (rc != HYB_OK) return rc;
    if (batch->graph_dirty) HYB_TRY(build_graph(batch));
    return from_hip(hipGraphLaunch(batch->exec, st));
}

hyb_status hyb_batch_launch_eager(hyb_batch batch, void* stream) {
    if (!batch) return HYB_ERR_INVALID_ARG;
    if (!same_device(batch->device)) return HYB_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hyb_status rc = sync_table(batch, st);
    if (rc != HYB_OK) return rc;
    return from_hip(launch_eager(batch, st));
}

hyb_status hyb_batch_tune(hyb_batch batch, const hyb_batch_tune_opts* opts, float* item_error, float* best_ms,
                          void* stream) {
    if (!batch || !opts || opts->reps < 1 || opts->reps > 100 || (opts->flags & ~3u) || std::isnan(opts->max_error_rate) ||
        opts->max_error_rate < 0.0f || opts->n_thresholds < 0 || (opts->n_thresholds > 0 && !opts->thresholds))
        return HYB_ERR_INVALID_ARG;
    if (!same_device(batch->device)) return HYB_ERR_INVALID_ARG;
    std::vector<float> cands;
    if (opts->n_thresholds > 0) {
        cands.assign(opts->thresholds, opts->thresholds + opts->n_thresholds);
    } else {
        cands = {0.0f, 0.5f, 1.0f, 2.0f, 4.0f, 8.0f, 16.0f, 32.0f, __builtin_inff()};
    }
    for (float c : cands)
        if (std::isnan(c) || c < 0.0f) return HYB_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t n_items = static_cast<int32_t>(batch->args.size());
    refresh_grids(batch);
    if (item_error)
        for (int32_t i = 0; i < n_items; ++i) item_error[i] = 0.0f;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    void* scratch = nullptr;
    unsigned long long* d_count = nullptr;
    hyb_status rc = from_hip(hipEventCreate(&e0));
    if (rc == HYB_OK) rc = from_hip(hipEventCreate(&e1));

    if (rc == HYB_OK && (opts->flags & HYB_TUNE_THRESHOLD)) {
        int64_t max_n = 0;
        for (int32_t i = 0; i < n_items; ++i)
            if (batch->kind[i] == kBoth) max_n = std::max(max_n, batch->args[i].n);
        if (max_n > 0) {
            rc = from_hip(hipMalloc(&scratch, 16 * static_cast<size_t>(max_n)));
            if (rc == HYB_OK) rc = from_hip(hipMalloc(&d_count, sizeof(unsigned long long)));
            for (int32_t i = 0; rc == HYB_OK && i < n_items; ++i) {
                if (batch->kind[i] != kBoth || batch->args[i].n == 0) continue;
                rc = tune_item_threshold(batch, i, cands, opts->max_error_rate, opts->reps, scratch, d_count, st, e0,
                                         e1, item_error ? item_error + i : nullptr);
            }
            batch->table_dirty = true;
        }
    }

    float final_ms = 0.0f;
    if (rc == HYB_OK && (opts->flags & HYB_TUNE_LAUNCH)) {
        hyb_batch_config best = batch->cfg;
        float best_t = std::numeric_limits<float>::infinity();
        for (int32_t lds : {8, 16, 32}) {
            for (int32_t rpi : {64, 256, 1024, 4096}) {
                for (int32_t bpc : {1, 2, 4, 8}) {
                    if (rc != HYB_OK) break;
                    const hyb_batch_config c = {lds, rpi, bpc};
                    batch->cfg = c;
                    batch->table_dirty = true;
                    rc = sync_table(batch, st);
                    float ms = 0.0f;
                    if (rc == HYB_OK)
                        rc = time_min([&] { return launch_eager(batch, st); }, opts->reps, st, e0, e1, &ms);
                    if (rc == HYB_OK && ms < best_t) {
                        best_t = ms;
                        best = c;
                    }
                }
            }
        }
        batch->cfg = best;
        batch->table_dirty = true;
        final_ms = best_t;
    }
    if (rc == HYB_OK) rc = sync_table(batch, st);
    if (rc == HYB_OK && !(opts->flags & HYB_TUNE_LAUNCH))
        rc = time_min([&] { return launch_eager(batch, st); }, opts->reps, st, e0, e1, &final_ms);
    if (rc == HYB_OK && best_ms) *best_ms = final_ms;
    if (scratch) (void)hipFree(scratch);
    if (d_count) (void)hipFree(d_count);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

hyb_status hyb_batch_launch_static(const hyb_batch_item* items, int32_t n_items, const hyb_batch_config* config,
                                   void* stream) {
    if (!items || n_items < 1 || n_items > HYB_STATIC_BATCH_MAX_ITEMS) return HYB_ERR_INVALID_ARG;
    const hyb_batch_config cfg = config ? *config : hyb_batch_config{16, 256, 4};
    if (!valid_config(cfg)) return HYB_ERR_INVALID_ARG;
    int fmt = 0;
    const hyb_status checked = check_items(items, n_items, &fmt);
    if (checked != HYB_OK) return checked;
    int dev = 0;
    HYB_TRY(hipGetDevice(&dev));
    void* ptr = nullptr;
    int n_cu = 0;
    HYB_TRY(hyb::static_scratch(dev, &ptr, &n_cu));
    // offsets and descriptors on the stack: nothing is allocated, on the
    // device or the host
    uint32_t item_start[HYB_STATIC_BATCH_MAX_ITEMS + 1];
    uint64_t total = 0;
    for (int32_t s = 0; s < n_items; ++s) {
        item_start[s] = static_cast<uint32_t>(total);
        total += (static_cast<uint64_t>(items[s].n) + cfg.rays_per_item - 1) / cfg.rays_per_item;
        if (total >= kMaxWorkItems) return HYB_ERR_UNSUPPORTED;
    }
    item_start[n_items] = static_cast<uint32_t>(total);
    dim3 grid;
    const hyb_status gs = persistent_grid(fmt, cfg, n_cu, total, &grid);
    if (gs != HYB_OK) return gs;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* base = static_cast<unsigned char*>(ptr);
    uint32_t* words = reinterpret_cast<uint32_t*>(base);
    HYB_TRY(hyb::fill_static(words, static_cast<uint32_t>(hyb::kStaticStartOff / 4), item_start, n_items + 1, st));
    constexpr size_t kArgWords = sizeof(hyb::TraceArgs) / sizeof(uint32_t);
    for (int32_t s = 0; s < n_items; ++s) {
        hyb::TraceArgs a;
        item_args(items[s], a);
        HYB_TRY(hyb::fill_static(words, static_cast<uint32_t>((hyb::kStaticTableOff + sizeof(a) * s) / 4), &a,
                                 kArgWords, st));
    }
    uint32_t* queue = reinterpret_cast<uint32_t*>(base + hyb::kStaticQueueOff);
    const hyb::TraceArgs* scenes = reinterpret_cast<const hyb::TraceArgs*>(base + hyb::kStaticTableOff);
    void* reset_args[] = {&queue};
    HYB_TRY(hipLaunchKernel(hyb::queue_reset_kernel(), dim3(1), dim3(64), reset_args, 0, st));
    if (total == 0) return HYB_OK;
    hyb::BatchArgs kargs = {};
    kargs.scenes = scenes;
    kargs.item_start = reinterpret_cast<const uint32_t*>(base + hyb::kStaticStartOff);
    kargs.queue = queue;
    kargs.n_scenes = n_items;
    kargs.n_items = static_cast<uint32_t>(total);
    kargs.rays_per_item = cfg.rays_per_item;
    void* trace_args[] = {&kargs, &scenes};
    return from_hip(hipLaunchKernel(hyb::batch_kernel(fmt, cfg.lds_depth), grid, dim3(hyb::kBatchBlock), trace_args,
                                    hyb::batch_lds_bytes(cfg.lds_depth), st));
}

hyb_status hyb_batch_destroy(hyb_batch batch) {
    if (!batch) return HYB_ERR_INVALID_ARG;
    drop_graph(batch);
    if (batch->d_args) (void)hipFree(batch->d_args);
    if (batch->d_item_start) (void)hipFree(batch->d_item_start);
    if (batch->d_queue) (void)hipFree(batch->d_queue);
    delete batch;
    return HYB_OK;
}

}  // extern "C"
