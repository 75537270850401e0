// Plain FP64 AIDW kernel for gfx950: the straightforward two-pass method of
// Sec. 3.2 in double precision, one query per lane.
//
//  * pass 1: squared distances d^2 = dx*dx + dy*dy with no FMA contraction,
//    so they are bit-identical to a plain C evaluation; the k nearest are
//    kept in a register list ordered by (d^2, data index) (Sec. 3.1.2);
//  * alpha from Eq. 2-6;
//  * pass 2: w = d^-alpha, unscaled, with both sums of Eq. 1
//    Neumaier-compensated: in a wave whose 64 queries share one whole alpha A
//    in [1, 8] (alpha_5 of the paper's levels, most tiles of uniform data)
//    as 1 / (d2^(A div 2) sqrt(d2)^(A mod 2)) with IEEE-rounded products,
//    square root and division, within a few ulp of pow; otherwise
//    pow(d^2, -alpha/2) (a per-lane choice would run both in mixed waves).
//    A query that coincides with data points (d = 0, alpha > 0) returns the
//    mean z of those points.
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

// A whole alpha in [1, 8], else 0.
__device__ __forceinline__ int whole_alpha(double al) {
    return (al >= 1.0 && al <= 8.0 && al == floor(al)) ? (int)al : 0;
}

// d^-A from d^2 for a whole A in [1, 8]: d2 multiplied in A div 2 times,
// times sqrt(d2) for odd A, then one division (about A/2 + 2 roundings in
// all, against pow's one; FP64 keeps that far below the 1e-12 bar).
template <int A>
__device__ __forceinline__ double whole_weight(double d2) {
    double q = 1.0;
#pragma unroll
    for (int i = 0; i < A / 2; ++i) q *= d2;
    if constexpr (A % 2 == 1) q *= sqrt(d2);
    return 1.0 / q;
}

// The same for a run-time A, operation for operation (a multiply by 1.0 is
// exact), for kernels that cannot dispatch on A.
__device__ __forceinline__ double whole_weight_rt(double d2, int A) {
    const int h = A >> 1;
    double q = 1.0;
    q = h >= 1 ? q * d2 : q;
    q = h >= 2 ? q * d2 : q;
    q = h >= 3 ? q * d2 : q;
    q = h >= 4 ? q * d2 : q;
    q *= (A & 1) ? sqrt(d2) : 1.0;
    return 1.0 / q;
}

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
    const int A = coincident ? 0 : whole_alpha(al);

    // ---- pass 2 (Eq. 1) -----------------------------------------------------
    Neumaier num, den;
    const int a0 = __builtin_amdgcn_readfirstlane(A);
    bool done = false;
    if (a0 != 0 && __all(A == a0)) {  // one whole power in every lane
        auto scan = [&](auto weight) {
            for (int jj = 0; jj < m; ++jj) {
                const double w = weight(sqdist64(qx, qy, X[jj], Y[jj]));
                num.add(w * Z[jj]);
                den.add(w);
            }
        };
        done = true;
        switch (a0) {
#define AIDW_F64_WHOLE(AA) \
    case AA: scan([](double d2) { return whole_weight<AA>(d2); }); break;
            AIDW_F64_WHOLE(1) AIDW_F64_WHOLE(2) AIDW_F64_WHOLE(3) AIDW_F64_WHOLE(4)
            AIDW_F64_WHOLE(5) AIDW_F64_WHOLE(6) AIDW_F64_WHOLE(7) AIDW_F64_WHOLE(8)
#undef AIDW_F64_WHOLE
            default: done = false; break;
        }
    }
    if (!done) {
        for (j = 0; j < m; ++j) {
            const double d2 = sqdist64(qx, qy, X[j], Y[j]);
            const double w = coincident ? (d2 == 0.0 ? 1.0 : 0.0) : pow(d2, e);
            num.add(w * Z[j]);
            den.add(w);
        }
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

// ---- data-access variants (the paper's naive and tiled versions in FP64) ------
// The arithmetic of f64_query point by point in the same order -- the k
// nearest by (d^2, index), pass 2 Neumaier-summed in data order -- so every
// variant equals the plain kernel bit for bit; only the way a data point
// reaches the lanes differs: access 0 scalar loads (as the plain kernel),
// 1 LDS tiles of kTile64 points staged by the workgroup with coalesced loads,
// 2 one vector load per lane and point (the address is lane-dependent in
// form: vary = 0 at run time but unknown to the compiler).  Layout 0 reads
// x[], y[], z[]; layout 1 one 32-byte {x, y, z, pad} per point, packed by
// the library.
constexpr int kTile64 = kGroupSize;

struct D4 {
    double x, y, z, w;
};

template <int ACCESS, int LAYOUT>
__device__ __forceinline__ D4 fetch64(const ProblemF64& p, const double4* __restrict__ aos, int j,
                                      int vary) {
    if constexpr (ACCESS == 0) {
        if constexpr (LAYOUT == 1) {
            const cptr64 a = (cptr64)aos + 4 * (int64_t)j;
            return D4{a[0], a[1], a[2], 0.0};
        } else {
            return D4{((cptr64)p.dx)[j], ((cptr64)p.dy)[j], ((cptr64)p.dz)[j], 0.0};
        }
    } else {
        const int i = ACCESS == 2 ? j + ((int)threadIdx.x & vary) : j;
        if constexpr (LAYOUT == 1) {
            const double4 v = aos[i];
            return D4{v.x, v.y, v.z, 0.0};
        } else {
            return D4{p.dx[i], p.dy[i], p.dz[i], 0.0};
        }
    }
}

template <int K, int ACCESS, int LAYOUT, bool TRACK>
__global__ __launch_bounds__(kGroupSize) void aidw_f64_variant(ProblemF64 p,
                                                               const double4* __restrict__ aos,
                                                               int vary) {
    __shared__ D4 tile[kTile64];
    const int qi = blockIdx.x * kGroupSize + threadIdx.x;
    const int c = qi < p.n ? qi : p.n - 1;
    const double qx = p.qx[c], qy = p.qy[c];
    const int m = p.m;
    const int pad = K - p.ap.k;
    double top[K];
    int tix[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        top[i] = i < pad ? -INFINITY : INFINITY;
        tix[i] = -1;
    }
    // the whole workgroup walks the data in tiles (ACCESS 1) or each lane on
    // its own (ACCESS 0, 2); `visit` sees every point once, in data order
    auto walk = [&](auto&& visit) {
        if constexpr (ACCESS == 1) {
            for (int base = 0; base < m; base += kTile64) {
                const int cnt = min(kTile64, m - base);
                if ((int)threadIdx.x < cnt)
                    tile[threadIdx.x] = fetch64<1, LAYOUT>(p, aos, base + threadIdx.x, 0);
                __syncthreads();
                for (int j = 0; j < cnt; ++j) visit(tile[j], base + j);
                __syncthreads();
            }
        } else {
            for (int j = 0; j < m; ++j) visit(fetch64<ACCESS, LAYOUT>(p, aos, j, vary), j);
        }
    };
    walk([&](const D4& pt, int j) {
        const double d2 = sqdist64(qx, qy, pt.x, pt.y);
        if (d2 < top[K - 1]) list_insert_idx<K, double>(top, tix, d2, j);
    });
    double r_obs;
    const double al = alpha_from_list<K, double>(top, p.ap, r_obs);
    const double d2min = list_min<K, double>(top, p.ap.k);
    const bool coincident = (d2min == 0.0) && (al > 0.0);
    const double e = -0.5 * al;
    const int A = coincident ? 0 : whole_alpha(al);
    // the plain kernel's choice, made per wave of 64 consecutive queries
    const int a0 = __builtin_amdgcn_readfirstlane(A);
    const bool whole = a0 != 0 && __all(A == a0);
    Neumaier num, den;
    walk([&](const D4& pt, int) {
        const double d2 = sqdist64(qx, qy, pt.x, pt.y);
        const double w = coincident ? (d2 == 0.0 ? 1.0 : 0.0)
                                    : (whole ? whole_weight_rt(d2, a0) : pow(d2, e));
        num.add(w * pt.z);
        den.add(w);
    });
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

__global__ void pack_aoas64(const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, int m, double4* __restrict__ aos) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) aos[i] = make_double4(x[i], y[i], z[i], 0.0);
}

template <int K, int ACCESS, int LAYOUT>
hipError_t launch_v64(const ProblemF64& p, const double4* aos, hipStream_t s) {
    const unsigned groups = (unsigned)((p.n + kGroupSize - 1) / kGroupSize);
    if (p.knn)
        hipLaunchKernelGGL((aidw_f64_variant<K, ACCESS, LAYOUT, true>), dim3(groups),
                           dim3(kGroupSize), 0, s, p, aos, 0);
    else
        hipLaunchKernelGGL((aidw_f64_variant<K, ACCESS, LAYOUT, false>), dim3(groups),
                           dim3(kGroupSize), 0, s, p, aos, 0);
    return hipGetLastError();
}

template <int K>
hipError_t launch_vk64(const ProblemF64& p, int access, int layout, const double4* aos,
                       hipStream_t s) {
    switch (access * 2 + layout) {
        case 0: return launch_k<K>(p, s);  // the plain kernel itself
        case 1: return launch_v64<K, 0, 1>(p, aos, s);
        case 2: return launch_v64<K, 1, 0>(p, aos, s);
        case 3: return launch_v64<K, 1, 1>(p, aos, s);
        case 4: return launch_v64<K, 2, 0>(p, aos, s);
        case 5: return launch_v64<K, 2, 1>(p, aos, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_aidw_f64_variant(const ProblemF64& p, int access, int layout, double4* aos,
                                   hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
    if (layout == 1) {
        hipLaunchKernelGGL(pack_aoas64, dim3((unsigned)((p.m + 255) / 256)), dim3(256), 0, stream,
                           p.dx, p.dy, p.dz, p.m, aos);
    }
    switch (k_bucket(p.ap.k)) {
        case 4: return launch_vk64<4>(p, access, layout, aos, stream);
        case 8: return launch_vk64<8>(p, access, layout, aos, stream);
        case 10: return launch_vk64<10>(p, access, layout, aos, stream);
        case 12: return launch_vk64<12>(p, access, layout, aos, stream);
        case 16: return launch_vk64<16>(p, access, layout, aos, stream);
        case 20: return launch_vk64<20>(p, access, layout, aos, stream);
        case 24: return launch_vk64<24>(p, access, layout, aos, stream);
        case 32: return launch_vk64<32>(p, access, layout, aos, stream);
        default: return hipErrorInvalidValue;
    }
}

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
