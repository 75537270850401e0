// Device-side pieces of the alpha determination (Sec. 2.2) and the
// register-resident k-nearest list (Sec. 3.1.2), shared by the FP32-scaled
// and the FP64 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace aidw {

// Eq. 5: mu_R in [0, 1]; the argument of the cosine is (pi / R_max)(R - R_min)
// and the first case whose interval contains R is taken.
__device__ __forceinline__ double eq5_mu(double R, double R_min, double R_max) {
    if (R <= R_min) return 0.0;
    if (R <= R_max) return 0.5 - 0.5 * cos((M_PI / R_max) * (R - R_min));
    return 1.0;
}

// Eq. 6: triangular membership over the five levels, knots at
// mu = 0.1, 0.3, 0.5, 0.7, 0.9, flat outside; first matching case taken.
__device__ __forceinline__ double eq6_alpha(double mu, const double* lv) {
    if (mu <= 0.1) return lv[0];
    if (mu <= 0.3) return lv[0] * (1.0 - 5.0 * (mu - 0.1)) + 5.0 * lv[1] * (mu - 0.1);
    if (mu <= 0.5) return 5.0 * lv[2] * (mu - 0.3) + lv[1] * (1.0 - 5.0 * (mu - 0.3));
    if (mu <= 0.7) return lv[2] * (1.0 - 5.0 * (mu - 0.5)) + 5.0 * lv[3] * (mu - 0.5);
    if (mu <= 0.9) return 5.0 * lv[4] * (mu - 0.7) + lv[3] * (1.0 - 5.0 * (mu - 0.7));
    return lv[4];
}

// Eq. 3-6 for one query from its sorted list of squared distances t[0..K-1]
// whose first K - k entries are -infinity.  Returns alpha; r_obs through
// the reference.  Summed in ascending order in FP64.
template <int K, typename T>
__device__ __forceinline__ double alpha_from_list(const T (&t)[K], const AlphaParams& ap,
                                                  double& r_obs) {
    // The K - k padding entries are -inf and every real entry is >= 0 (or
    // +inf): testing the value instead of the index keeps the test per lane,
    // so no uniform masks of the padding stay live in SGPRs through the scan.
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (t[i] > (T)-INFINITY) s += sqrt((double)t[i]);
    r_obs = s / (double)ap.k;
    const double R = r_obs / ap.r_exp;
    return eq6_alpha(eq5_mu(R, ap.R_min, ap.R_max), ap.levels);
}

// The smallest real entry (index K - k: the first that is not -inf padding),
// read with static indices only.
template <int K, typename T>
__device__ __forceinline__ T list_min(const T (&t)[K], int) {
    T v = t[K - 1];
#pragma unroll
    for (int i = K - 1; i >= 0; --i) v = t[i] > (T)-INFINITY ? t[i] : v;
    return v;
}

// Insert v into the ascending list t, dropping the largest entry: entry i
// becomes the median of (t[i-1], v, t[i]).  Equal values do not move, so
// a later-scanned point never displaces an earlier one at equal distance.
template <int K>
__device__ __forceinline__ void list_insert(float (&t)[K], float v) {
#pragma unroll
    for (int i = K - 1; i > 0; --i) t[i] = __builtin_amdgcn_fmed3f(t[i - 1], v, t[i]);
    t[0] = fminf(t[0], v);
}

// Same insertion carrying the data index; strict comparisons keep the
// earlier (smaller) index first among equal distances.
template <int K, typename T>
__device__ __forceinline__ void list_insert_idx(T (&t)[K], int (&ti)[K], T v, int vi) {
#pragma unroll
    for (int i = K - 1; i > 0; --i) {
        const bool before_prev = v < t[i - 1];
        const bool before_cur = v < t[i];
        const T nt = before_prev ? t[i - 1] : (before_cur ? v : t[i]);
        const int ni = before_prev ? ti[i - 1] : (before_cur ? vi : ti[i]);
        t[i] = nt;
        ti[i] = ni;
    }
    if (v < t[0]) {
        t[0] = v;
        ti[0] = vi;
    }
}

// Squared distance in FP32, the one formula every FP32 kernel uses so that
// their k-nearest lists agree bit for bit.
__device__ __forceinline__ float sqdist(float qx, float qy, float px, float py) {
    const float ex = qx - px;
    const float ey = qy - py;
    return fmaf(ey, ey, ex * ex);
}

// Per-query terms of pass 2 from the k-nearest list: alpha (Eq. 3-6), and for
// w = exp2(na * log2 d^2 + aL0) = (d_min^2 / d^2)^(alpha/2), na = -alpha/2 and
// aL0 = (alpha/2) log2 d_min^2.
template <int K>
__device__ __forceinline__ void query_power(const float (&top)[K], const AlphaParams& ap,
                                            double& r_obs, double& al, float& na, float& aL0,
                                            float& d2min) {
    al = alpha_from_list<K, float>(top, ap, r_obs);
    const float a = (float)(0.5 * al);
    d2min = list_min<K, float>(top, ap.k);
    const float L0 = __builtin_amdgcn_logf(d2min);
    na = -a;
    aL0 = a * L0;
}

// alpha as a small whole power (1..8) when the weights can be formed as
// (d_min / d)^alpha with one reciprocal square root per pair; 0 otherwise.
__device__ __forceinline__ int integer_power(double alpha, float d2min) {
    const bool whole = alpha >= 1.0 && alpha <= 8.0 && alpha == (double)(int)alpha;
    return (whole && d2min >= 1.17549435e-38f) ? (int)alpha : 0;
}

}  // namespace aidw
