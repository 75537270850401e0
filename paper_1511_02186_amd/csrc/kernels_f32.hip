// FP32-scaled fused AIDW kernel for gfx950.
//
// One launch runs both of the paper's full passes over the m data points
// for every query (Sec. 3.2): pass 1 finds the k nearest data points
// (Sec. 3.1.2) and from them alpha (Eq. 2-6); pass 2 forms the weighted
// average of Eq. 1.
//
// Mapping to CDNA4:
//  * Each lane owns Q queries (query = wave*64*Q + slot*64 + lane), so query
//    loads and output stores are coalesced per slot.
//  * All lanes of a wave walk the data points in the same order, so a data
//    point is wave-uniform: its coordinates are fetched with scalar loads
//    into SGPRs (B points per batch) and broadcast to every lane as an
//    instruction operand.  This replaces the paper's shared-memory tiles: no
//    LDS traffic, no barriers, and one scalar fetch serves 64*Q pair
//    evaluations.
//  * The k-nearest list lives in registers as squared distances; a batch of
//    B candidates is first reduced to its minimum (v_min3) and compared with
//    the k-th entry, so insertion code runs only when some lane improves.
//    Insertion is a chain of v_med3.
//  * Pass-2 weights are rescaled per query so that none exceeds 1:
//    w = (d_min^2 / d^2)^(alpha/2) = exp2(-(alpha/2) log2 d^2 + (alpha/2) log2 d_min^2),
//    i.e. one v_log_f32, one FMA and one v_exp_f32 per pair.  The common
//    factor d_min^(-alpha) cancels in the ratio of Eq. 1.
//  * Sum w and sum w*z are accumulated in FP32 over each batch of B points
//    and folded into FP64 accumulators after every batch; the final ratio is
//    taken in FP64.
//  * Queries that coincide with a data point (d_min == 0) use a variant of
//    the pass-2 loop, selected wave-uniformly, that clamps the exponent at 0:
//    log2(0) = -inf turns the exponent into NaN exactly for the coincident
//    points, the clamp maps it to 0 (weight 1), and every other point gets
//    weight exp2(-inf) = 0, so the result is the mean z of the coincident
//    points.
#include "common.h"
#include "device_math.h"

namespace aidw {
namespace {

constexpr int kBatch = 16;

__device__ __forceinline__ float sqdist(float qx, float qy, float px, float py) {
    const float ex = qx - px;
    const float ey = qy - py;
    return fmaf(ey, ey, ex * ex);
}

template <int Q, bool SAFE>
__device__ __forceinline__ void pass2(const float* __restrict__ X, const float* __restrict__ Y,
                                      const float* __restrict__ Z, int m, const float (&qx)[Q],
                                      const float (&qy)[Q], const float (&na)[Q],
                                      const float (&aL0)[Q], double (&Sw)[Q], double (&Swz)[Q]) {
    const int mb = m - m % kBatch;
    int j = 0;
    for (; j < mb; j += kBatch) {
        float px[kBatch], py[kBatch], pz[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            px[u] = X[j + u];
            py[u] = Y[j + u];
            pz[u] = Z[j + u];
        }
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            float sw = 0.0f, swz = 0.0f;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const float d2 = sqdist(qx[s], qy[s], px[u], py[u]);
                float t = fmaf(na[s], __builtin_amdgcn_logf(d2), aL0[s]);
                if (SAFE) t = fminf(t, 0.0f);
                const float w = __builtin_amdgcn_exp2f(t);
                sw += w;
                swz = fmaf(w, pz[u], swz);
            }
            Sw[s] += (double)sw;
            Swz[s] += (double)swz;
        }
    }
    for (; j < m; ++j) {
        const float px = X[j], py = Y[j], pz = Z[j];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const float d2 = sqdist(qx[s], qy[s], px, py);
            float t = fmaf(na[s], __builtin_amdgcn_logf(d2), aL0[s]);
            if (SAFE) t = fminf(t, 0.0f);
            const float w = __builtin_amdgcn_exp2f(t);
            Sw[s] += (double)w;
            Swz[s] += (double)(w * pz);
        }
    }
}

template <int K, int Q, bool TRACK>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_fused(ProblemF32 p) {
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
    const int m = p.m;
    const float* __restrict__ X = p.dx;
    const float* __restrict__ Y = p.dy;
    const float* __restrict__ Z = p.dz;

    int qi[Q];
    float qx[Q], qy[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        qi[s] = (wave * Q + s) * kWaveSize + lane;
        const int c = qi[s] < p.n ? qi[s] : p.n - 1;
        qx[s] = p.qx[c];
        qy[s] = p.qy[c];
    }

    // ---- pass 1: k nearest data points by squared distance -----------------
    const int pad = K - p.ap.k;
    float top[Q][K];
    int tix[TRACK ? Q : 1][TRACK ? K : 1];
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
        for (int i = 0; i < K; ++i) {
            top[s][i] = i < pad ? -INFINITY : INFINITY;
            if constexpr (TRACK) tix[s][i] = -1;
        }

    const int mb = m - m % kBatch;
    int j = 0;
    for (; j < mb; j += kBatch) {
        float px[kBatch], py[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            px[u] = X[j + u];
            py[u] = Y[j + u];
        }
        float d2[Q][kBatch];
        float mn[Q];
        bool hit = false;
#pragma unroll
        for (int s = 0; s < Q; ++s) {
#pragma unroll
            for (int u = 0; u < kBatch; ++u) d2[s][u] = sqdist(qx[s], qy[s], px[u], py[u]);
            mn[s] = d2[s][0];
#pragma unroll
            for (int u = 1; u < kBatch; ++u) mn[s] = fminf(mn[s], d2[s][u]);
            hit |= mn[s] < top[s][K - 1];
        }
        if (hit) {
#pragma unroll
            for (int s = 0; s < Q; ++s) {
                if (mn[s] < top[s][K - 1]) {
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        if (d2[s][u] < top[s][K - 1]) {
                            if constexpr (TRACK)
                                list_insert_idx<K, float>(top[s], tix[s], d2[s][u], j + u);
                            else
                                list_insert<K>(top[s], d2[s][u]);
                        }
                    }
                }
            }
        }
    }
    for (; j < m; ++j) {
        const float px = X[j], py = Y[j];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const float d2 = sqdist(qx[s], qy[s], px, py);
            if (d2 < top[s][K - 1]) {
                if constexpr (TRACK)
                    list_insert_idx<K, float>(top[s], tix[s], d2, j);
                else
                    list_insert<K>(top[s], d2);
            }
        }
    }

    // ---- alpha per query (Eq. 2-6) in FP64 ---------------------------------
    float na[Q], aL0[Q];
    bool coincident = false;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        double r_obs;
        const double al = alpha_from_list<K, float>(top[s], p.ap, r_obs);
        const float a = (float)(0.5 * al);
        const float L0 = __builtin_amdgcn_logf(list_min<K, float>(top[s], p.ap.k));
        na[s] = -a;
        aL0[s] = a * L0;
        coincident |= (L0 == -INFINITY);
        if (qi[s] < p.n) {
            if (p.r_obs) p.r_obs[qi[s]] = r_obs;
            if (p.alpha) p.alpha[qi[s]] = al;
            if constexpr (TRACK) {
#pragma unroll
                for (int i = 0; i < K; ++i)
                    if (i >= pad) p.knn[(int64_t)qi[s] * p.ap.k + (i - pad)] = tix[s][i];
            }
        }
    }

    // ---- pass 2: weighted average of Eq. 1 with rescaled weights ------------
    double Sw[Q], Swz[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) Sw[s] = Swz[s] = 0.0;
    if (__any(coincident))
        pass2<Q, true>(X, Y, Z, m, qx, qy, na, aL0, Sw, Swz);
    else
        pass2<Q, false>(X, Y, Z, m, qx, qy, na, aL0, Sw, Swz);

#pragma unroll
    for (int s = 0; s < Q; ++s)
        if (qi[s] < p.n) p.out[qi[s]] = (float)(Swz[s] / Sw[s]);
}

template <int K, int Q, bool TRACK>
hipError_t launch_kq(const ProblemF32& p, hipStream_t stream) {
    const int64_t per_group = (int64_t)kGroupSize * Q;
    const int64_t groups = (p.n + per_group - 1) / per_group;
    hipLaunchKernelGGL((aidw_f32_fused<K, Q, TRACK>), dim3((unsigned)groups), dim3(kGroupSize),
                       0, stream, p);
    return hipGetLastError();
}

template <int K>
hipError_t launch_k(const ProblemF32& p, const LaunchF32& cfg, hipStream_t stream) {
    if (p.knn) return launch_kq<K, 1, true>(p, stream);
    switch (cfg.q_per_lane) {
        case 1: return launch_kq<K, 1, false>(p, stream);
        case 2: return launch_kq<K, 2, false>(p, stream);
        case 4: return launch_kq<K, 4, false>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_aidw_f32(const ProblemF32& p, const LaunchF32& cfg, hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
    switch (k_bucket(p.ap.k)) {
        case 4: return launch_k<4>(p, cfg, stream);
        case 8: return launch_k<8>(p, cfg, stream);
        case 10: return launch_k<10>(p, cfg, stream);
        case 12: return launch_k<12>(p, cfg, stream);
        case 16: return launch_k<16>(p, cfg, stream);
        case 20: return launch_k<20>(p, cfg, stream);
        case 24: return launch_k<24>(p, cfg, stream);
        case 32: return launch_k<32>(p, cfg, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace aidw
