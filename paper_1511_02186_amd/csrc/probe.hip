// Issue-cost probe of libaidw (declared in include/aidw.h): how many SIMD
// cycles a wave64 FP32 FMA, a v_exp_f32 and a VALU instruction with an SGPR
// operand occupy on this device, compiled
// like every kernel here (packed FP32 off).  These costs, not the packed-FMA
// peak, bound the FP32-scaled kernels.
//
// Each thread runs 16 independent chains; a workgroup is 16 waves and two
// workgroups per CU give 8 waves per SIMD.  Kinds:
//   0: FMAs only (8 per chain per iteration);
//   1: one exp2 (after one FMA) per chain per iteration;
//   2: waves (w / 4) even run kind 1, odd run kind 0, so SIMDs hold both;
//   3: subtractions with an SGPR operand only (v_sub_f32 v, s, v);
//   4: those alternating with VGPR-only multiplies.
// Two VALU instructions of different waves can issue in one cycle unless
// both read an SGPR: kinds 3 and 4 show the difference.
#include <algorithm>

#include "handle.h"

using namespace aidw::detail;

namespace {

constexpr int kChains = 16;
constexpr int kFmaPerIter = 8;
constexpr int kThreads = 1024;
constexpr int kBlocksPerCU = 2;

template <int KIND>
__global__ __launch_bounds__(kThreads) void issue_probe(float* __restrict__ out,
                                                        const float* __restrict__ src,
                                                        int iters) {
    float a[kChains], b[kChains];
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        a[j] = threadIdx.x * 1e-3f + j;
        b[j] = 0.5f + j * 1e-3f;
    }
    const bool exp_wave = KIND == 1 || (KIND == 2 && ((wave >> 2) & 1) == 0);
    const float c = 0.999f + threadIdx.x * 1e-9f;  // per lane: a VGPR operand
    for (int i = 0; i < iters; ++i) {
        const float s = src[i & 63];
        if constexpr (KIND >= 3) {
            // s is wave-uniform (a scalar load), so it stays an SGPR operand
#pragma unroll
            for (int f = 0; f < kFmaPerIter; ++f)
#pragma unroll
                for (int j = 0; j < kChains; ++j) {
                    b[j] = s - b[j];
                    if (KIND == 4) a[j] = a[j] * c;
                }
        } else if (exp_wave) {
#pragma unroll
            for (int j = 0; j < kChains; ++j) a[j] = __builtin_amdgcn_exp2f(fmaf(a[j], -1.0f, s));
        } else {
#pragma unroll
            for (int f = 0; f < kFmaPerIter; ++f)
#pragma unroll
                for (int j = 0; j < kChains; ++j) b[j] = fmaf(b[j], 0.999f, s);
        }
    }
    float r = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) r += a[j] + b[j];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = r;
}

template <int KIND>
hipError_t time_probe(hipStream_t s, int blocks, float* out, const float* src, int iters,
                      hipEvent_t e0, hipEvent_t e1, double* ms) {
    hipLaunchKernelGGL(issue_probe<KIND>, dim3(blocks), dim3(kThreads), 0, s, out, src, iters);
    hipError_t e = hipEventRecord(e0, s);
    hipLaunchKernelGGL(issue_probe<KIND>, dim3(blocks), dim3(kThreads), 0, s, out, src, iters);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    *ms = t;
    return e;
}

}  // namespace

extern "C" {

aidw_status aidw_probe_issue_costs(aidw_t h, aidw_issue_costs* out) {
    ErrorScope es(h);
    if (!h || !out) return fail(AIDW_EINVAL, "handle or out is NULL");
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, h->device) != hipSuccess ||
        clock_khz <= 0)
        return fail(AIDW_EDEVICE, "cannot read the device clock");
    const int cus = h->cu_count > 0 ? h->cu_count : 1;
    const int blocks = cus * kBlocksPerCU;
    const size_t bytes = sizeof(float) * ((size_t)blocks * kThreads + 64);
    void* mem = nullptr;
    aidw_status st = device_alloc(h, bytes, &mem);
    if (st != AIDW_OK) return st;
    float* buf = static_cast<float*>(mem);
    float* src = buf + (size_t)blocks * kThreads;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemsetAsync(src, 0, 64 * sizeof(float), h->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double ms[5] = {0, 0, 0, 0, 0};
    const int iters = 8192;
    // a first untimed round brings the clock up
    if (e == hipSuccess) e = time_probe<0>(h->stream, blocks, buf, src, iters, e0, e1, &ms[0]);
    if (e == hipSuccess) e = time_probe<0>(h->stream, blocks, buf, src, iters, e0, e1, &ms[0]);
    if (e == hipSuccess) e = time_probe<1>(h->stream, blocks, buf, src, iters, e0, e1, &ms[1]);
    if (e == hipSuccess) e = time_probe<2>(h->stream, blocks, buf, src, iters, e0, e1, &ms[2]);
    if (e == hipSuccess) e = time_probe<3>(h->stream, blocks, buf, src, iters, e0, e1, &ms[3]);
    if (e == hipSuccess) e = time_probe<4>(h->stream, blocks, buf, src, iters, e0, e1, &ms[4]);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    device_free(h, mem, bytes);
    if (e != hipSuccess) return hip_fail(e, "issue probe");

    // SIMD cycles per wave and iteration: time x clock x SIMDs / waves
    const double hz = clock_khz * 1e3;
    const double waves_per_simd = (double)kThreads / 64.0 * kBlocksPerCU / 4.0;  // 8
    auto per_wave_iter = [&](double t_ms) {
        return t_ms * 1e-3 * hz / (waves_per_simd * (double)iters);
    };
    const double fma = per_wave_iter(ms[0]) / (kChains * kFmaPerIter);
    const double exp_alone = per_wave_iter(ms[1]) / kChains - fma;
    // kind 2: half the waves of each SIMD per kind; what the exp waves add on
    // top of the FMA waves' own cycles, per exp
    const double total = per_wave_iter(ms[2]) * waves_per_simd;
    const double fma_side = waves_per_simd / 2 * kChains * kFmaPerIter * fma;
    const double exp_side_fma = waves_per_simd / 2 * kChains * fma;
    const double exp_beside = (total - fma_side - exp_side_fma) / (waves_per_simd / 2 * kChains);
    const double per_inst = kChains * kFmaPerIter;
    out->sgpr_operand_cycles = per_wave_iter(ms[3]) / per_inst;
    out->sgpr_beside_vgpr_cycles = per_wave_iter(ms[4]) / (2 * per_inst);
    out->fma_cycles = fma;
    out->exp_cycles = exp_alone;
    out->exp_cycles_beside_fma = std::max(0.0, exp_beside);
    out->clock_ghz = hz * 1e-9;
    out->compute_units = cus;
    return AIDW_OK;
}

}  // extern "C"
