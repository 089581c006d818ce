// Trace kernels: the combined query and the two pure baselines.
//
// One ray per lane.  Rays and hits are SoA arrays, so each of the seven input
// and four output streams is read or written with fully coalesced 256-byte
// wavefront accesses.  The BVH stack lives in LDS ([depth][thread] so the 64
// lanes of a wavefront hit 64 distinct banks), with a small private spill area
// for the rare paths deeper than the LDS part.
#include "hyb_device.hpp"
#include "kernels.hpp"

namespace hyb {

// Wavefronts per SIMD the compiler is held to where that measured faster:
// one-cell F16 bricks, 74 VGPRs left alone, fit seven at 72; the combined I8
// query, which forms its solves again (df_resolve) to fit, seven at 70.
template <int MODE, int FMT, bool COUNT>
constexpr int trace_waves() {
    if (COUNT) return 1;
    if (FMT == kF16 && (MODE == kCombined || MODE == kDfOnly)) return 7;
    if (FMT == kI8 && MODE == kCombined) return 7;
    return 1;
}

template <int MODE, int FMT, bool COUNT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(trace_waves<MODE, FMT, COUNT>())))
void k_trace(TraceArgs a) {
    extern __shared__ int s_stack[];
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x, a.xcd_run) * kBlock + threadIdx.x;
    if (i >= a.n) return;
    trace_ray<MODE, FMT, COUNT>(a, i, s_stack + threadIdx.x, kBlock);
}

template <int MODE, int FMT, bool COUNT>
static hipError_t launch(const TraceArgs& a, hipStream_t stream) {
    const size_t lds = MODE == kDfOnly ? 0 : sizeof(int) * kLdsDepth * kBlock;
    const int64_t blocks = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((k_trace<MODE, FMT, COUNT>), dim3((unsigned)blocks), dim3(kBlock), lds, stream, a);
    return hipGetLastError();
}

template <int MODE, bool COUNT>
static hipError_t launch_fmt(const TraceArgs& a, hipStream_t stream) {
    if constexpr (MODE == kBvhOnly) return launch<MODE, kF32, COUNT>(a, stream);
    switch (a.fmt) {
        case kF32: return launch<MODE, kF32, COUNT>(a, stream);
        case kF16: return launch<MODE, kF16, COUNT>(a, stream);
        case kF16B2: return launch<MODE, kF16B2, COUNT>(a, stream);
        case kI8: return launch<MODE, kI8, COUNT>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_trace(int mode, bool counters, const TraceArgs& args, hipStream_t stream) {
    if (args.n <= 0) return hipSuccess;
    TraceArgs a = args;
    if (a.xcd_run == 0) a.xcd_run = kXcdRun;  // xcd_block needs a run of at least 1
    switch (mode * 2 + (counters ? 1 : 0)) {
        case 0: return launch_fmt<kCombined, false>(a, stream);
        case 1: return launch_fmt<kCombined, true>(a, stream);
        case 2: return launch_fmt<kBvhOnly, false>(a, stream);
        case 3: return launch_fmt<kBvhOnly, true>(a, stream);
        case 4: return launch_fmt<kDfOnly, false>(a, stream);
        case 5: return launch_fmt<kDfOnly, true>(a, stream);
        case 6: return launch_fmt<kShadow, false>(a, stream);
        case 7: return launch_fmt<kShadow, true>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hyb
