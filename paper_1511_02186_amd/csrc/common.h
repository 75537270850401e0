// Internal declarations shared by the libaidw host code and its kernel
// translation units.  Not part of the public C ABI (see include/aidw.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aidw {

constexpr int kWaveSize = 64;
constexpr int kWavesPerGroup = 4;
constexpr int kGroupSize = kWaveSize * kWavesPerGroup;

// Largest k handled in registers (matches AIDW_KMAX).
constexpr int kKMax = 32;

// Per-problem constants of the alpha determination (Sec. 2.2, Eq. 2-6).
struct AlphaParams {
    double levels[5];  // alpha_1..alpha_5
    double R_min, R_max;
    double r_exp;      // Eq. 2, computed once per problem on the host
    int k;
};

// One FP32-scaled problem: planar device arrays, optional diagnostics.
struct ProblemF32 {
    const float* dx;
    const float* dy;
    const float* dz;
    const float* qx;
    const float* qy;
    float* out;
    double* r_obs;     // optional
    double* alpha;     // optional
    int32_t* knn;      // optional [n][k]
    int m;
    int n;
    AlphaParams ap;
};

struct ProblemF64 {
    const double* dx;
    const double* dy;
    const double* dz;
    const double* qx;
    const double* qy;
    double* out;
    double* r_obs;
    double* alpha;
    int32_t* knn;
    int m;
    int n;
    AlphaParams ap;
};

// Register bucket used for a given k: the top-k list holds K >= k entries,
// the first K - k of which are fixed at -infinity.
int k_bucket(int k);

// Launch configuration of the FP32-scaled fused kernel.
struct LaunchF32 {
    int q_per_lane;  // queries owned by each lane: 1, 2 or 4
};

hipError_t launch_aidw_f32(const ProblemF32& p, const LaunchF32& cfg, hipStream_t stream);
hipError_t launch_aidw_f64(const ProblemF64& p, hipStream_t stream);

}  // namespace aidw
