// VALU issue rates by instruction class (measurement aid for the roofline of
// the evaluation kernels; not part of the filter).
//
// Each kernel runs eight independent dependency chains per lane of one
// instruction class (so that the chain latency is hidden), over a grid that
// fills the device several times, and the rate is the lane-operations
// completed per second between two HIP events.  The loops compile to exactly
// the named instruction (checked in the AMD assembly of this build; the
// integer one is written as that instruction, since the compiler folds a chain
// of 24-bit multiply-adds), and packed FP32 is disabled here as everywhere in
// the library.

#include "internal.h"
#include "../../include/mcslam.h"

#include <cstdint>

namespace mcs {
namespace {

constexpr int kRateChains = 8;
constexpr int kRateBlock = 256;
constexpr int kRateBlocks = 256 * 8 * 4;   // 8 waves of 4 workgroups per CU, 4 times over
constexpr int kRateUnroll = 4;
constexpr int kRateIters = 512;
constexpr int kRateReps = 3;          // timed launches, after two untimed ones

template <int C>
__global__ __launch_bounds__(kRateBlock) void k_issue_rate(float *out, int iters, float m, float s,
                                                           double md, double sd, uint32_t cm,
                                                           uint32_t cs)
{
    float a[kRateChains];
    double b[kRateChains];
    uint32_t c[kRateChains];
    // Per-lane multiplicands (in VGPRs, so that the FMAs take their two-operand
    // accumulating forms v_fmac_f32 and v_fmac_f64, as most of the evaluation
    // loop's do).
    const float x = m + (float)(threadIdx.x & 1) * s, y = m * s;
    const double xd = md + (double)(threadIdx.x & 1) * sd, yd = md * sd;
    const uint32_t cmv = cm + (threadIdx.x & 1), csv = cs + (threadIdx.x & 2);
    for (int k = 0; k < kRateChains; ++k) {
        a[k] = (float)(threadIdx.x + k) * 1e-3f + 0.5f;
        b[k] = (double)(threadIdx.x + k) * 1e-3 + 0.5;
        c[k] = threadIdx.x + k;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kRateUnroll; ++u) {
#pragma unroll
            for (int k = 0; k < kRateChains; ++k) {
                if (C == MCS_RATE_FP32_FMA) a[k] = fmaf(x, y, a[k]);                  // v_fmac_f32
                if (C == MCS_RATE_FP64_FMA) b[k] = fma(xd, yd, b[k]);                 // v_fmac_f64
                if (C == MCS_RATE_FP64_UNARY) b[k] = __builtin_amdgcn_fract(b[k]);    // v_fract_f64
                if (C == MCS_RATE_INT24)                                               // v_mad_u32_u24
                    asm volatile("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(c[k]) : "v"(c[k]), "v"(cmv), "v"(csv));
                if (C == MCS_RATE_TRANS) a[k] = __builtin_amdgcn_rcpf(a[k]);          // v_rcp_f32
                if (C == MCS_RATE_FP32_FP64) {                                         // alternating
                    a[k] = fmaf(x, y, a[k]);
                    b[k] = fma(xd, yd, b[k]);
                }
            }
        }
    }
    float acc = 0.0f;
    for (int k = 0; k < kRateChains; ++k) acc += a[k] + (float)b[k] + (float)c[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int C>
hipError_t time_class(float *out, hipEvent_t e0, hipEvent_t e1, double *rate)
{
    // Small multiplicands keep every chain finite; the values do not matter.
    const auto launch = [&]() {
        hipLaunchKernelGGL(k_issue_rate<C>, dim3(kRateBlocks), dim3(kRateBlock), 0, nullptr, out,
                           kRateIters, 1e-3f, 1e-3f, 1e-3, 1e-3, 1u, 0u);
    };
    launch();   // warm-up (code load, clocks)
    launch();
    hipError_t e = hipEventRecord(e0, nullptr);
    for (int r = 0; r < kRateReps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return e;
    const double ops = (double)kRateReps * kRateBlocks * kRateBlock * kRateIters * kRateUnroll * kRateChains *
                       (C == MCS_RATE_FP32_FP64 ? 2.0 : 1.0);
    *rate = ms > 0.0f ? ops / (ms * 1e-3) : 0.0;
    return hipSuccess;
}

}  // namespace

hipError_t measure_issue_rates(double *rates)
{
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)kRateBlocks * kRateBlock * sizeof(float));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = time_class<MCS_RATE_FP32_FMA>(out, e0, e1, &rates[MCS_RATE_FP32_FMA]);
    if (e == hipSuccess) e = time_class<MCS_RATE_FP64_FMA>(out, e0, e1, &rates[MCS_RATE_FP64_FMA]);
    if (e == hipSuccess) e = time_class<MCS_RATE_FP64_UNARY>(out, e0, e1, &rates[MCS_RATE_FP64_UNARY]);
    if (e == hipSuccess) e = time_class<MCS_RATE_INT24>(out, e0, e1, &rates[MCS_RATE_INT24]);
    if (e == hipSuccess) e = time_class<MCS_RATE_TRANS>(out, e0, e1, &rates[MCS_RATE_TRANS]);
    if (e == hipSuccess) e = time_class<MCS_RATE_FP32_FP64>(out, e0, e1, &rates[MCS_RATE_FP32_FP64]);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    return e;
}

}  // namespace mcs
