// Data-access variants of the FP32-scaled AIDW kernel, for measuring the
// paper's design axes on gfx950 (Sec. 3.1.3 data layouts, Sec. 3.2 naive and
// tiled versions; Sec. 4-5 compare them).  All variants do the same
// arithmetic as the production kernel -- register k-nearest list, alpha in
// FP64, rescaled exp2/log2 weights, FP32 partial sums folded into FP64 --
// and differ only in how a data point reaches the lanes:
//
//   access 0, scalar:  wave-uniform scalar loads into SGPRs (production);
//   access 1, tiled:   a workgroup stages 256 points in LDS with coalesced
//                      loads, barrier, every lane reads each point from LDS
//                      (the paper's tiled version);
//   access 2, naive:   every lane issues its own global load of each point
//                      (the paper's naive version: no shared memory; the
//                      load address is made lane-dependent in form so that it
//                      stays a vector load);
//
// and layout 0 = SoA (x[], y[], z[]), layout 1 = AoaS (one 16-byte aligned
// {x, y, z, pad} per point, built by the library in its workspace).
#include "common.h"
#include "device_math.h"

namespace aidw {
namespace {

constexpr int kTile = kGroupSize;  // points per LDS tile: one per thread

struct P4 {
    float x, y, z, w;
};

typedef const __attribute__((address_space(4))) float* cptr;

// Point j of the data set, by access scheme and layout.  Scalar access reads
// through the constant address space (wave-uniform scalar loads).  Naive
// access offsets the index by (threadIdx.x & vary), with vary = 0 at run time
// but unknown to the compiler, so every lane issues its own vector load.
template <int ACCESS, int LAYOUT>
__device__ __forceinline__ P4 fetch(const ProblemF32& p, const float4* __restrict__ aos, int j,
                                    int vary) {
    if constexpr (ACCESS == 0) {
        if constexpr (LAYOUT == 1) {
            const cptr a = (cptr)aos + 4 * (int64_t)j;
            return P4{a[0], a[1], a[2], 0.0f};
        } else {
            return P4{((cptr)p.dx)[j], ((cptr)p.dy)[j], ((cptr)p.dz)[j], 0.0f};
        }
    } else {
        const int i = ACCESS == 2 ? j + ((int)threadIdx.x & vary) : j;
        if constexpr (LAYOUT == 1) {
            const float4 v = aos[i];
            return P4{v.x, v.y, v.z, 0.0f};
        } else {
            return P4{p.dx[i], p.dy[i], p.dz[i], 0.0f};
        }
    }
}

template <int K>
__device__ __forceinline__ void knn_one(float qx, float qy, const P4& pt, float (&top)[K]) {
    const float d2 = sqdist(qx, qy, pt.x, pt.y);
    if (d2 < top[K - 1]) list_insert<K>(top, d2);
}

__device__ __forceinline__ float weight(float qx, float qy, const P4& pt, float na, float aL0,
                                        bool safe) {
    const float d2 = sqdist(qx, qy, pt.x, pt.y);
    float t = fmaf(na, __builtin_amdgcn_logf(d2), aL0);
    if (safe) t = fminf(t, 0.0f);
    return __builtin_amdgcn_exp2f(t);
}

template <int K, int ACCESS, int LAYOUT>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_variant(ProblemF32 p,
                                                               const float4* __restrict__ aos,
                                                               int vary) {
    __shared__ P4 tile[kTile];
    const int q = blockIdx.x * kGroupSize + threadIdx.x;
    const int c = q < p.n ? q : p.n - 1;
    const float qx = p.qx[c], qy = p.qy[c];
    const int m = p.m;
    const int pad = K - p.ap.k;
    float top[K];
#pragma unroll
    for (int i = 0; i < K; ++i) top[i] = i < pad ? -INFINITY : INFINITY;

    // ---- pass 1 ----
    if constexpr (ACCESS == 1) {
        for (int base = 0; base < m; base += kTile) {
            const int cnt = min(kTile, m - base);
            if ((int)threadIdx.x < cnt)
                tile[threadIdx.x] = fetch<1, LAYOUT>(p, aos, base + threadIdx.x, 0);
            __syncthreads();
            for (int j = 0; j < cnt; ++j) knn_one<K>(qx, qy, tile[j], top);
            __syncthreads();
        }
    } else {
        for (int j = 0; j < m; ++j) knn_one<K>(qx, qy, fetch<ACCESS, LAYOUT>(p, aos, j, vary), top);
    }

    double r_obs;
    const double al = alpha_from_list<K, float>(top, p.ap, r_obs);
    const float a = (float)(0.5 * al);
    const float L0 = __builtin_amdgcn_logf(list_min<K, float>(top, p.ap.k));
    const float na = -a, aL0 = a * L0;
    const bool safe = __any(!(aL0 > -INFINITY));

    // ---- pass 2: FP32 sums over 16 points, folded into FP64 ----
    double Sw = 0.0, Swz = 0.0;
    float sw = 0.0f, swz = 0.0f;
    int in_batch = 0;
    auto add = [&](const P4& pt) {
        const float w = weight(qx, qy, pt, na, aL0, safe);
        sw += w;
        swz = fmaf(w, pt.z, swz);
        if (++in_batch == 16) {
            Sw += (double)sw;
            Swz += (double)swz;
            sw = swz = 0.0f;
            in_batch = 0;
        }
    };
    if constexpr (ACCESS == 1) {
        for (int base = 0; base < m; base += kTile) {
            const int cnt = min(kTile, m - base);
            if ((int)threadIdx.x < cnt)
                tile[threadIdx.x] = fetch<1, LAYOUT>(p, aos, base + threadIdx.x, 0);
            __syncthreads();
            for (int j = 0; j < cnt; ++j) add(tile[j]);
            __syncthreads();
        }
    } else {
        for (int j = 0; j < m; ++j) add(fetch<ACCESS, LAYOUT>(p, aos, j, vary));
    }
    Sw += (double)sw;
    Swz += (double)swz;
    if (q < p.n) {
        p.out[q] = (float)(Swz / Sw);
        if (p.r_obs) p.r_obs[q] = r_obs;
        if (p.alpha) p.alpha[q] = al;
    }
}

__global__ void pack_aoas(const float* __restrict__ x, const float* __restrict__ y,
                          const float* __restrict__ z, int m, float4* __restrict__ aos) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) aos[i] = make_float4(x[i], y[i], z[i], 0.0f);
}

template <int K, int ACCESS, int LAYOUT>
hipError_t launch_v(const ProblemF32& p, const float4* aos, hipStream_t s) {
    const unsigned groups = (unsigned)((p.n + kGroupSize - 1) / kGroupSize);
    hipLaunchKernelGGL((aidw_f32_variant<K, ACCESS, LAYOUT>), dim3(groups), dim3(kGroupSize), 0, s,
                       p, aos, 0);
    return hipGetLastError();
}

template <int K>
hipError_t launch_vk(const ProblemF32& p, int access, int layout, const float4* aos,
                     hipStream_t s) {
    switch (access * 2 + layout) {
        case 0: return launch_v<K, 0, 0>(p, aos, s);
        case 1: return launch_v<K, 0, 1>(p, aos, s);
        case 2: return launch_v<K, 1, 0>(p, aos, s);
        case 3: return launch_v<K, 1, 1>(p, aos, s);
        case 4: return launch_v<K, 2, 0>(p, aos, s);
        case 5: return launch_v<K, 2, 1>(p, aos, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_aidw_f32_variant(const ProblemF32& p, int access, int layout, float4* aos,
                                   hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
    if (layout == 1) {
        hipLaunchKernelGGL(pack_aoas, dim3((unsigned)((p.m + 255) / 256)), dim3(256), 0, stream,
                           p.dx, p.dy, p.dz, p.m, aos);
    }
    switch (k_bucket(p.ap.k)) {
        case 4: return launch_vk<4>(p, access, layout, aos, stream);
        case 8: return launch_vk<8>(p, access, layout, aos, stream);
        case 10: return launch_vk<10>(p, access, layout, aos, stream);
        case 12: return launch_vk<12>(p, access, layout, aos, stream);
        case 16: return launch_vk<16>(p, access, layout, aos, stream);
        case 20: return launch_vk<20>(p, access, layout, aos, stream);
        case 24: return launch_vk<24>(p, access, layout, aos, stream);
        case 32: return launch_vk<32>(p, access, layout, aos, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace aidw
