// Plain FP64 AIDW kernel for gfx950: the straightforward two-pass method of
// Sec. 3.2 in double precision, one query per lane.
//
//  * pass 1: squared distances d^2 = dx*dx + dy*dy with no FMA contraction,
//    so they are bit-identical to a plain C evaluation; the k nearest are
//    kept in a register list ordered by (d^2, data index) (Sec. 3.1.2);
//  * alpha from Eq. 2-6;
//  * pass 2: w = d^-alpha evaluated as pow(d^2, -alpha/2), unscaled, with
//    both sums of Eq. 1 Neumaier-compensated.  A query that coincides with
//    data points (d = 0, alpha > 0) returns the mean z of those points.
//
// Data points are wave-uniform and are read with scalar loads, as in the
// FP32-scaled kernel.  This kernel is the precision reference and the
// speed baseline of the FP32-scaled path.
#include "common.h"
#include "device_math.h"

namespace aidw {
namespace {

constexpr int kBatch = 8;

#pragma clang fp contract(off)
__device__ __forceinline__ double sqdist64(double qx, double qy, double px, double py) {
    const double ex = qx - px;
    const double ey = qy - py;
    const double xx = ex * ex;
    const double yy = ey * ey;
    return xx + yy;
}

struct Neumaier {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x) {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

// Data are read through the constant address space: at wave-uniform
// addresses such loads are scalar, also when the problem itself was loaded
// from memory (a serving job descriptor).
typedef const __attribute__((address_space(4))) double* cptr64;

// One query (index qi; lanes with qi >= n compute a clamped copy and store
// nothing): both passes over all m points.
template <int K, bool TRACK>
__device__ __forceinline__ void f64_query(const ProblemF64& p, int qi) {
    const int c = qi < p.n ? qi : p.n - 1;
    const double qx = p.qx[c], qy = p.qy[c];
    const int m = p.m;
    const cptr64 X = (cptr64)p.dx;
    const cptr64 Y = (cptr64)p.dy;
    const cptr64 Z = (cptr64)p.dz;

    const int pad = K - p.ap.k;
    double top[K];
    int tix[TRACK ? K : 1];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        top[i] = i < pad ? -INFINITY : INFINITY;
        if constexpr (TRACK) tix[i] = -1;
    }

    // ---- pass 1 -------------------------------------------------------------
    const int mb = m - m % kBatch;
    int j = 0;
    for (; j < mb; j += kBatch) {
        double d2[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) d2[u] = sqdist64(qx, qy, X[j + u], Y[j + u]);
        double mn = d2[0];
#pragma unroll
        for (int u = 1; u < kBatch; ++u) mn = fmin(mn, d2[u]);
        if (mn < top[K - 1]) {
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (d2[u] < top[K - 1]) {
                    if constexpr (TRACK) {
                        list_insert_idx<K, double>(top, tix, d2[u], j + u);
                    } else {
                        int dummy[K];
                        list_insert_idx<K, double>(top, dummy, d2[u], j + u);
                    }
                }
            }
        }
    }
    for (; j < m; ++j) {
        const double d2 = sqdist64(qx, qy, X[j], Y[j]);
        if (d2 < top[K - 1]) {
            if constexpr (TRACK) {
                list_insert_idx<K, double>(top, tix, d2, j);
            } else {
                int dummy[K];
                list_insert_idx<K, double>(top, dummy, d2, j);
            }
        }
    }

    // ---- alpha (Eq. 2-6) ------------------------------------------------------
    double r_obs;
    const double al = alpha_from_list<K, double>(top, p.ap, r_obs);
    const double d2min = list_min<K, double>(top, p.ap.k);
    const bool coincident = (d2min == 0.0) && (al > 0.0);
    const double e = -0.5 * al;

    // ---- pass 2 (Eq. 1) -----------------------------------------------------
    Neumaier num, den;
    for (j = 0; j < m; ++j) {
        const double d2 = sqdist64(qx, qy, X[j], Y[j]);
        const double w = coincident ? (d2 == 0.0 ? 1.0 : 0.0) : pow(d2, e);
        num.add(w * Z[j]);
        den.add(w);
    }

    if (qi < p.n) {
        p.out[qi] = num.value() / den.value();
        if (p.r_obs) p.r_obs[qi] = r_obs;
        if (p.alpha) p.alpha[qi] = al;
        if constexpr (TRACK) {
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i >= pad) p.knn[(int64_t)qi * p.ap.k + (i - pad)] = tix[i];
        }
    }
}

template <int K, bool TRACK>
__global__ __launch_bounds__(kGroupSize) void aidw_f64_plain(ProblemF64 p) {
    f64_query<K, TRACK>(p, (int)(blockIdx.x * kGroupSize + threadIdx.x));
}

// Serving: one wave per (job, 64-query tile) item.
template <int K, bool TRACK>
__global__ __launch_bounds__(kGroupSize) void aidw_f64_serve(const ProblemF64* __restrict__ jobs,
                                                             const ServeItem* __restrict__ items,
                                                             int n_items) {
    const int it = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6));
    if (it >= n_items) return;
    const ServeItem w = items[it];
    f64_query<K, TRACK>(jobs[w.job], w.tile * kWaveSize + (int)(threadIdx.x & (kWaveSize - 1)));
}

template <int K>
hipError_t launch_k(const ProblemF64& p, hipStream_t stream) {
    const int64_t groups = (p.n + kGroupSize - 1) / kGroupSize;
    if (p.knn)
        hipLaunchKernelGGL((aidw_f64_plain<K, true>), dim3((unsigned)groups), dim3(kGroupSize), 0,
                           stream, p);
    else
        hipLaunchKernelGGL((aidw_f64_plain<K, false>), dim3((unsigned)groups), dim3(kGroupSize), 0,
                           stream, p);
    return hipGetLastError();
}

template <int K>
hipError_t launch_serve_k(const ProblemF64* jobs, const ServeItem* items, int n_items, bool track,
                          hipStream_t stream) {
    const unsigned groups = (unsigned)((n_items + kWavesPerGroup - 1) / kWavesPerGroup);
    if (track)
        hipLaunchKernelGGL((aidw_f64_serve<K, true>), dim3(groups), dim3(kGroupSize), 0, stream,
                           jobs, items, n_items);
    else
        hipLaunchKernelGGL((aidw_f64_serve<K, false>), dim3(groups), dim3(kGroupSize), 0, stream,
                           jobs, items, n_items);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_aidw_f64_serve(const ProblemF64* jobs, const ServeItem* items, int n_items,
                                 int K, bool track, hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
    switch (K) {
        case 4: return launch_serve_k<4>(jobs, items, n_items, track, stream);
        case 8: return launch_serve_k<8>(jobs, items, n_items, track, stream);
        case 10: return launch_serve_k<10>(jobs, items, n_items, track, stream);
        case 12: return launch_serve_k<12>(jobs, items, n_items, track, stream);
        case 16: return launch_serve_k<16>(jobs, items, n_items, track, stream);
        case 20: return launch_serve_k<20>(jobs, items, n_items, track, stream);
        case 24: return launch_serve_k<24>(jobs, items, n_items, track, stream);
        case 32: return launch_serve_k<32>(jobs, items, n_items, track, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aidw_f64(const ProblemF64& p, hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
    switch (k_bucket(p.ap.k)) {
        case 4: return launch_k<4>(p, stream);
        case 8: return launch_k<8>(p, stream);
        case 10: return launch_k<10>(p, stream);
        case 12: return launch_k<12>(p, stream);
        case 16: return launch_k<16>(p, stream);
        case 20: return launch_k<20>(p, stream);
        case 24: return launch_k<24>(p, stream);
        case 32: return launch_k<32>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace aidw
