// FP32-scaled AIDW kernels for gfx950.
//
// Every query gets the paper's two full passes over the m data points
// (Sec. 3.2): pass 1 finds the k nearest data points (Sec. 3.1.2) and from
// them alpha (Eq. 2-6); pass 2 forms the weighted average of Eq. 1.
//
// Mapping to CDNA4:
//  * A wave owns a tile of 64*Q queries; lane l, slot s holds query
//    base + s*64 + l, so query loads and output stores are coalesced.
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
//    factor d_min^(-alpha) cancels in the ratio of Eq. 1.  Waves whose
//    queries share one whole alpha A in [1, 8] use w = rsq(d^2)^A instead
//    (one transcendental), unscaled when max|z| and d_min allow it.
//  * Pass 2 with one query per lane is software-pipelined by one batch: the
//    transcendentals of batch b+1 are issued back to back, as a burst, after
//    the weights of batch b are summed.  On gfx950 a transcendental keeps the
//    SIMD from pairing two VALU instructions of different waves in one
//    issue cycle; spread one per weight, with the weight's next multiply
//    waiting on it, it cost about 14 cycles of issue per wave instead of the
//    8 it costs inside a burst.
//  * Sum w and sum w*z are accumulated in FP32 over each batch of B points
//    and folded into FP64 accumulators after every batch; the final ratio is
//    taken in FP64.
//  * Queries that coincide with a data point (d_min == 0) use a variant of
//    the pass-2 loop, selected wave-uniformly, that clamps the exponent at 0:
//    log2(0) = -inf turns the exponent into NaN exactly for the coincident
//    points, the clamp maps it to 0 (weight 1), and every other point gets
//    weight exp2(-inf) = 0, so the result is the mean z of the coincident
//    points.
//
// Drivers sharing these building blocks:
//  * aidw_f32_fused: one wave per tile, both passes over all m points;
//  * aidw_f32_batch: one wave per (problem, tile) item of a longest-first
//    work list, so one launch (capturable in a hipGraph) serves many
//    problems of uneven size;
//  * split-m: when n is too small to fill the device, the m points are cut
//    into S segments; one launch computes per-segment k-nearest lists, a
//    merge kernel turns them into alpha, a third launch computes
//    per-segment weighted sums and a last kernel adds the segments in order;
//  * aidw_f32_serve: fused and split items of many jobs in one launch per
//    scheduling tick.
#include "common.h"
#include "device_math.h"

namespace aidw {
namespace {

// Data points per scalar-load batch.  Pass 1 loads x and y (2 SGPRs per
// point), pass 2 also z (3 SGPRs per point); the batch is sized so that the
// SGPR file holds it without spills.  Lanes that own several queries use
// smaller batches to leave SGPRs for their extra state.  Pass 1 keeps B
// squared distances in VGPRs until the batch minimum is known: 16 keeps the
// k <= 16 kernels at 64 VGPRs or fewer (8 waves per SIMD), where 32 points
// took 69 VGPRs (7 waves).
#ifndef AIDW_F32_B1
#define AIDW_F32_B1 16
#endif
#ifndef AIDW_F32_B2
#define AIDW_F32_B2 16
#endif
template <int Q>
constexpr int batch1_for() { return Q == 1 ? AIDW_F32_B1 : 16; }
template <int Q>
constexpr int batch2_for() { return Q == 1 ? AIDW_F32_B2 : 16; }


__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWaveSize - 1); }

// Global wave index, made visibly wave-uniform (an SGPR) so that everything
// derived from it -- data ranges in particular -- stays scalar.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6));
}

// Data points are read through the constant address space: the kernels never
// write them, and loads from that space at wave-uniform addresses are always
// lowered to scalar loads, also when the array's address itself was loaded
// from memory (a batch descriptor).
typedef const __attribute__((address_space(4))) float* cptr;
__device__ __forceinline__ cptr as_const(const float* p) { return (cptr)p; }

// ---- pass 1: fold data points [j0, j1) into the k-nearest lists ------------
template <int K, int Q, bool TRACK>
__device__ __forceinline__ void scan_knn(cptr X, cptr Y, int j0, int j1, const float (&qx)[Q],
                                         const float (&qy)[Q], float (&top)[Q][K],
                                         int (&tix)[TRACK ? Q : 1][TRACK ? K : 1]) {
    constexpr int B = batch1_for<Q>();
    int j = j0;
    for (; j + B <= j1; j += B) {
        float px[B], py[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            px[u] = X[j + u];
            py[u] = Y[j + u];
        }
        float d2[Q][B];
        float mn[Q];
        bool hit = false;
#pragma unroll
        for (int s = 0; s < Q; ++s) {
#pragma unroll
            for (int u = 0; u < B; ++u) d2[s][u] = sqdist(qx[s], qy[s], px[u], py[u]);
            mn[s] = d2[s][0];
#pragma unroll
            for (int u = 1; u < B; ++u) mn[s] = fminf(mn[s], d2[s][u]);
            hit |= mn[s] < top[s][K - 1];
        }
        if (hit) {
#pragma unroll
            for (int s = 0; s < Q; ++s) {
                if (mn[s] < top[s][K - 1]) {
#pragma unroll
                    for (int u = 0; u < B; ++u) {
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
    for (; j < j1; ++j) {
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
}

template <int K, int Q, bool TRACK>
__device__ __forceinline__ void init_lists(float (&top)[Q][K],
                                           int (&tix)[TRACK ? Q : 1][TRACK ? K : 1], int k) {
    const int pad = K - k;
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
        for (int i = 0; i < K; ++i) {
            top[s][i] = i < pad ? -INFINITY : INFINITY;
            if constexpr (TRACK) tix[s][i] = -1;
        }
}

// True when the query coincides with a data point: log2(d_min^2) = -inf makes
// aL0 -inf (alpha > 0) or NaN (alpha = 0).
__device__ __forceinline__ bool coincident(float aL0) { return !(aL0 > -INFINITY); }

// ---- pass 2: weighted sums over data points [j0, j1) -----------------------
// Pass 2 with one query per lane and a general alpha: w = exp2(na log2(d^2)
// + aL0).  Software-pipelined by one batch like the whole-power loop: the
// log2 and exp2 of batch b+1 go out as two bursts after batch b is summed.
template <bool SAFE>
__device__ __forceinline__ void scan_wsum1(cptr X, cptr Y, cptr Z, int j0, int j1, float qx,
                                           float qy, float na, float aL0, double& Sw,
                                           double& Swz) {
    constexpr int B = batch2_for<1>();
    auto from_d2 = [&](const float (&d2)[B], float (&w)[B]) {
        float t[B];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = __builtin_amdgcn_logf(d2[u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            t[u] = fmaf(na, t[u], aL0);
            if (SAFE) t[u] = fminf(t[u], 0.0f);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < B; ++u) w[u] = __builtin_amdgcn_exp2f(t[u]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto weights = [&](const float (&px)[B], const float (&py)[B], float (&w)[B]) {
        float d2[B];
#pragma unroll
        for (int u = 0; u < B; ++u) d2[u] = sqdist(qx, qy, px[u], py[u]);
        from_d2(d2, w);
    };
    auto sum = [&](const float (&w)[B], const float (&pz)[B]) {
        float sw = 0.0f, swz = 0.0f;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            sw += w[u];
            swz = fmaf(w[u], pz[u], swz);
        }
        Sw += (double)sw;
        Swz += (double)swz;
    };
    int j = j0;
    if (j + 2 * B <= j1) {
        float w[B];
        {
            float px[B], py[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                px[u] = X[j + u];
                py[u] = Y[j + u];
            }
            weights(px, py, w);
        }
        for (; j + 2 * B <= j1; j += B) {
            float pz[B], nx[B], ny[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                pz[u] = Z[j + u];
                nx[u] = X[j + B + u];
                ny[u] = Y[j + B + u];
            }
            // point by point, as in the whole-power loop: next batch's
            // distance beside this batch's sums
            float d2[B], sw = 0.0f, swz = 0.0f;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < B; ++u) {
                d2[u] = sqdist(qx, qy, nx[u], ny[u]);
                sw += w[u];
                swz = fmaf(w[u], pz[u], swz);
                __builtin_amdgcn_sched_barrier(0);
            }
            Sw += (double)sw;
            Swz += (double)swz;
            from_d2(d2, w);
        }
        float pz[B];
#pragma unroll
        for (int u = 0; u < B; ++u) pz[u] = Z[j + u];
        sum(w, pz);
        j += B;
    }
    for (; j + B <= j1; j += B) {
        float px[B], py[B], pz[B], w[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            px[u] = X[j + u];
            py[u] = Y[j + u];
            pz[u] = Z[j + u];
        }
        weights(px, py, w);
        sum(w, pz);
    }
    for (; j < j1; ++j) {
        const float d2 = sqdist(qx, qy, X[j], Y[j]);
        float t = fmaf(na, __builtin_amdgcn_logf(d2), aL0);
        if (SAFE) t = fminf(t, 0.0f);
        const float w = __builtin_amdgcn_exp2f(t);
        Sw += (double)w;
        Swz += (double)(w * Z[j]);
    }
}

// The same for Q queries per lane (the kernels for few query tiles), without
// the pipelining: their registers are already spent on the Q lists.
template <int Q, bool SAFE>
__device__ __forceinline__ void scan_wsum(cptr X, cptr Y, cptr Z, int j0, int j1,
                                          const float (&qx)[Q], const float (&qy)[Q],
                                          const float (&na)[Q], const float (&aL0)[Q],
                                          double (&Sw)[Q], double (&Swz)[Q]) {
    constexpr int B = batch2_for<Q>();
    int j = j0;
    for (; j + B <= j1; j += B) {
        float px[B], py[B], pz[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            px[u] = X[j + u];
            py[u] = Y[j + u];
            pz[u] = Z[j + u];
        }
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            float sw = 0.0f, swz = 0.0f;
#pragma unroll
            for (int u = 0; u < B; ++u) {
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
    for (; j < j1; ++j) {
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

// s^A for a compile-time integer A, by repeated squaring.
template <int A>
__device__ __forceinline__ float ipow(float s) {
    if constexpr (A == 1) return s;
    else if constexpr (A % 2 == 0) {
        const float h = ipow<A / 2>(s);
        return h * h;
    } else {
        return ipow<A - 1>(s) * s;
    }
}

// One batch of whole-power weights from r = rsq(d^2): w = (d_min r)^A, or
// r^A without SCALED; Σw and Σwz summed in point order in FP32, then added
// to the FP64 sums.  No fusing of w's last product into sw += w: Σw and Σwz
// then round alike (a constant field comes out exact).  The explicit fmaf
// calls stay.
template <int A, bool SCALED, int B>
__device__ __forceinline__ void int_batch(const float (&r)[B], const float (&pz)[B], float dmin,
                                          double& Sw, double& Swz) {
#pragma clang fp contract(off)
    auto power = [&](float x) { return ipow<A>(SCALED ? dmin * x : x); };
    const float w0 = power(r[0]);
    float sw = w0, swz = w0 * pz[0];
#pragma unroll
    for (int u = 1; u < B; ++u) {
        const float w = power(r[u]);
        sw += w;
        swz = fmaf(w, pz[u], swz);
    }
    Sw += (double)sw;
    Swz += (double)swz;
}

// Pass 2 for a wave whose queries all have the same integer power A and a
// normal, nonzero d_min: w = (d_min / d)^A = (d_min * rsq(d^2))^A, one
// transcendental instead of two.  Without SCALED the common factor d_min^-A
// is left in (w = rsq(d^2)^A, one multiply less per pair); the caller allows
// that only where every weight and every w*z stays inside the FP32 range.
//
// Software-pipelined by one batch: the rsq of batch b+1 go out as one burst
// after the weights of batch b are summed (15 % less time for this loop at
// m = n = 2^20 than one rsq beside each weight).
template <int A, bool SCALED>
__device__ __forceinline__ void scan_wsum_int(cptr X, cptr Y, cptr Z, int j0, int j1, float qx,
                                              float qy, float dmin, double& Sw, double& Swz) {
#pragma clang fp contract(off)
    constexpr int B = batch2_for<1>();
    int j = j0;
    if (j + 2 * B <= j1) {
        float r[B];
#pragma unroll
        for (int u = 0; u < B; ++u) r[u] = __builtin_amdgcn_rsqf(sqdist(qx, qy, X[j + u], Y[j + u]));
        for (; j + 2 * B <= j1; j += B) {
            float pz[B], nx[B], ny[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                pz[u] = Z[j + u];
                nx[u] = X[j + B + u];
                ny[u] = Y[j + B + u];
            }
            // point by point: the distance of the next batch's point beside
            // this batch's weight, so that scalar-operand subtractions sit
            // between plain multiplies (two VALU instructions of different
            // waves pair in one issue cycle only if at most one reads an
            // SGPR); the scheduling barriers keep that order
            float d2[B], sw, swz;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < B; ++u) {
                d2[u] = sqdist(qx, qy, nx[u], ny[u]);
                const float w = ipow<A>(SCALED ? dmin * r[u] : r[u]);
                if (u == 0) {
                    sw = w;
                    swz = w * pz[0];
                } else {
                    sw += w;
                    swz = fmaf(w, pz[u], swz);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            Sw += (double)sw;
            Swz += (double)swz;
#pragma unroll
            for (int u = 0; u < B; ++u) r[u] = __builtin_amdgcn_rsqf(d2[u]);
        }
        float pz[B];
#pragma unroll
        for (int u = 0; u < B; ++u) pz[u] = Z[j + u];
        int_batch<A, SCALED>(r, pz, dmin, Sw, Swz);
        j += B;
    }
    // fewer than 2B points in all: at most one whole batch, then the rest
    for (; j + B <= j1; j += B) {
        float r[B], pz[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            r[u] = __builtin_amdgcn_rsqf(sqdist(qx, qy, X[j + u], Y[j + u]));
            pz[u] = Z[j + u];
        }
        int_batch<A, SCALED>(r, pz, dmin, Sw, Swz);
    }
    for (; j < j1; ++j) {
        const float r = __builtin_amdgcn_rsqf(sqdist(qx, qy, X[j], Y[j]));
        const float w = ipow<A>(SCALED ? dmin * r : r);
        Sw += (double)w;
        Swz += (double)(w * Z[j]);
    }
}

// True when the weights rsq(d^2)^A = d^-A of a query can be summed unscaled:
// L = A log2(d_min) (= aL0) bounds every weight by 2^-L.  Needs L <= 60 (the
// nearest weight stays >= 2^-60, so far weights lost to underflow are
// negligible) and 16 * 2^-L * max|z| < 2^124 (no FP32 batch sum overflows).
__device__ __forceinline__ bool unscaled_ok(float aL0, const float* zmax) {
    if (!zmax) return false;
    const float zm = *zmax;
    const float lim = fminf(100.0f, 120.0f - __builtin_amdgcn_logf(zm));  // inf when zm = 0
    return aL0 <= 60.0f && -aL0 <= lim;
}

// ---- speculative single pass -------------------------------------------------
// Pass 1 together with the pass-2 sums of one whole power A, from the same
// squared distances.  When alpha_5 is a whole number A in [1, 8], alpha is A
// for every query whose R reaches R_max (Eq. 5 gives mu_R = 1 and Eq. 6
// alpha_5); on uniform data that is nearly every query, because the mean of
// k neighbour distances exceeds the expected first-neighbour distance of
// Eq. 2 several times.  A query that ends at alpha = A, with unscaled
// weights allowed, has then finished both passes in one scan; the others
// run pass 2 afterwards.  The sums are those of pass 2's unscaled
// whole-power loop bit for bit (the loop a wave of such queries takes): the
// same batches aligned at j0, the same order and the same rounding
// (scan_wsum_int<A, false>).  The k-nearest list comes out as pass 1's: the
// multiset of the k smallest squared distances does not depend on the
// batching.
template <int K, int A>
__device__ __forceinline__ void scan_knn_wsum_int(cptr X, cptr Y, cptr Z, int j0, int j1, float qx,
                                                  float qy, float (&top)[K], double& Sw,
                                                  double& Swz) {
#pragma clang fp contract(off)
    constexpr int B = batch2_for<1>();
    // One batch: B squared distances, the list screen and insertion, then
    // the B rsq in one burst (the first result is ready before the burst
    // ends, so the weights wait on nothing) and the weights and sums.  The
    // distances turn into their rsq in place: a batch needs B registers.
    // The z of a batch are loaded after its distances (so x, y and z are
    // never in SGPRs together) and arrive during the rsq burst.
    int j = j0;
    for (; j + B <= j1; j += B) {
        float v[B];
        {
            float px[B], py[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                px[u] = X[j + u];
                py[u] = Y[j + u];
            }
#pragma unroll
            for (int u = 0; u < B; ++u) v[u] = sqdist(qx, qy, px[u], py[u]);
        }
        __builtin_amdgcn_sched_barrier(0);
        float pz[B];
#pragma unroll
        for (int u = 0; u < B; ++u) pz[u] = Z[j + u];
        __builtin_amdgcn_sched_barrier(0);
        float mn = v[0];
#pragma unroll
        for (int u = 1; u < B; ++u) mn = fminf(mn, v[u]);
        if (mn < top[K - 1]) {
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (v[u] < top[K - 1]) list_insert<K>(top, v[u]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = __builtin_amdgcn_rsqf(v[u]);
        __builtin_amdgcn_sched_barrier(0);
        int_batch<A, false>(v, pz, 0.0f, Sw, Swz);
    }
    for (; j < j1; ++j) {
        const float d2 = sqdist(qx, qy, X[j], Y[j]);
        if (d2 < top[K - 1]) list_insert<K>(top, d2);
        const float w = ipow<A>(__builtin_amdgcn_rsqf(d2));
        Sw += (double)w;
        Swz += (double)(w * Z[j]);
    }
}

// Pass 1 over [j0, j1) with speculative sums for power A.  Early in the
// range (see kSpecCheckAt) the wave predicts each lane's final R: in a random
// order of the data the k-th distances shrink with the square root of the
// points seen, so the sum of the k distances found so far, times
// sqrt(seen / m), estimates the final sum.  If in some lane that estimate is
// below kSpecKeep times p.spec_dist_sum (the sum at which Eq. 5 reaches
// mu_R = 0.9, below which Eq. 6 leaves alpha_5), the speculation stops there
// and the scan goes on as plain pass 1.  The bias towards going on reflects
// the costs: a tile that gives up in vain needs a second scan later, one that
// goes on in vain has formed sums for nothing.
// Returns the first point that pass 1 has not seen: j1 when the sums in Sw,
// Swz cover the whole range, else where the plain scan must continue.
constexpr float kSpecKeep = 0.75f;
// The check comes after 1/kSpecCheckAt of the range, but after at least
// kSpecCheckMin points (a sample the k-th distance can be read from).
constexpr int kSpecCheckAt = 32;
constexpr int kSpecCheckMin = 512;

template <int K, int A>
__device__ __forceinline__ int knn_speculative(const ProblemF32& p, int j0, int j1, float qx,
                                               float qy, float (&top)[K], double& Sw, double& Swz) {
    cptr X = as_const(p.dx), Y = as_const(p.dy), Z = as_const(p.dz);
    const int jc = j0 + ((max((j1 - j0) / kSpecCheckAt, min(j1 - j0, kSpecCheckMin))) &
                         ~(batch2_for<1>() - 1));
    scan_knn_wsum_int<K, A>(X, Y, Z, j0, jc, qx, qy, top, Sw, Swz);
    if (jc > j0) {
        float s = 0.0f;  // -inf padding entries add nothing
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (top[i] > -INFINITY) s += __builtin_sqrtf(top[i]);
        const float predicted = s * __builtin_sqrtf((float)(jc - j0) / (float)p.m);
        if (!__all(predicted >= kSpecKeep * p.spec_dist_sum)) return jc;
    }
    scan_knn_wsum_int<K, A>(X, Y, Z, jc, j1, qx, qy, top, Sw, Swz);
    return j1;
}

// Pass 1 of one lane's query over [j0, j1), with the speculative sums of
// p.spec_power when that is set.  Returns true when Sw, Swz hold those sums
// for the whole range.
template <int K>
__device__ __forceinline__ bool knn_maybe_speculative(const ProblemF32& p, int j0, int j1, float qx,
                                                      float qy, float (&top)[K], double& Sw,
                                                      double& Swz) {
    int jscan = j0;
    switch (p.spec_power) {
#define AIDW_SPEC_CASE(A)                                                   \
    case A:                                                                 \
        jscan = knn_speculative<K, A>(p, j0, j1, qx, qy, top, Sw, Swz);      \
        break;
        AIDW_SPEC_CASE(1) AIDW_SPEC_CASE(2) AIDW_SPEC_CASE(3) AIDW_SPEC_CASE(4)
        AIDW_SPEC_CASE(5) AIDW_SPEC_CASE(6) AIDW_SPEC_CASE(7) AIDW_SPEC_CASE(8)
#undef AIDW_SPEC_CASE
        default:
            break;
    }
    float qxa[1] = {qx}, qya[1] = {qy};
    float topa[1][K];
#pragma unroll
    for (int i = 0; i < K; ++i) topa[0][i] = top[i];
    int tix[1][1];
    scan_knn<K, 1, false>(as_const(p.dx), as_const(p.dy), jscan, j1, qxa, qya, topa, tix);
#pragma unroll
    for (int i = 0; i < K; ++i) top[i] = topa[0][i];
    return p.spec_power != 0 && jscan == j1;
}

template <int A>
__device__ __forceinline__ void scan_wsum_int_any(cptr X, cptr Y, cptr Z, int j0, int j1,
                                                  float qx, float qy, float dmin, bool unscaled,
                                                  double& Sw, double& Swz) {
    if (__all(unscaled))
        scan_wsum_int<A, false>(X, Y, Z, j0, j1, qx, qy, dmin, Sw, Swz);
    else
        scan_wsum_int<A, true>(X, Y, Z, j0, j1, qx, qy, dmin, Sw, Swz);
}

// Pass 2 for one lane's queries: the whole-power loop when every lane of the
// wave has the same integer power (see integer_power), else the exp2/log2 one.
template <int Q>
__device__ __forceinline__ void scan_wsum_any(cptr X, cptr Y, cptr Z, int j0, int j1,
                                              const float (&qx)[Q], const float (&qy)[Q],
                                              const float (&na)[Q], const float (&aL0)[Q],
                                              double (&Sw)[Q], double (&Swz)[Q],
                                              int ipw = 0, float dmin = 0.0f,
                                              const float* zmax = nullptr) {
    if constexpr (Q == 1) {
        // same whole power in every lane: the one-transcendental loop
        const int a0 = __builtin_amdgcn_readfirstlane(ipw);
        if (a0 != 0 && __all(ipw == a0)) {
            const bool un = unscaled_ok(aL0[0], zmax);
            switch (a0) {
#define AIDW_INT_CASE(A) \
    case A: return scan_wsum_int_any<A>(X, Y, Z, j0, j1, qx[0], qy[0], dmin, un, Sw[0], Swz[0]);
                AIDW_INT_CASE(1) AIDW_INT_CASE(2) AIDW_INT_CASE(3) AIDW_INT_CASE(4)
                AIDW_INT_CASE(5) AIDW_INT_CASE(6) AIDW_INT_CASE(7) AIDW_INT_CASE(8)
#undef AIDW_INT_CASE
                default: break;
            }
        }
    }
    bool any_coincident = false;
#pragma unroll
    for (int s = 0; s < Q; ++s) any_coincident |= coincident(aL0[s]);
    if constexpr (Q == 1) {
        if (__any(any_coincident))
            scan_wsum1<true>(X, Y, Z, j0, j1, qx[0], qy[0], na[0], aL0[0], Sw[0], Swz[0]);
        else
            scan_wsum1<false>(X, Y, Z, j0, j1, qx[0], qy[0], na[0], aL0[0], Sw[0], Swz[0]);
    } else {
        if (__any(any_coincident))
            scan_wsum<Q, true>(X, Y, Z, j0, j1, qx, qy, na, aL0, Sw, Swz);
        else
            scan_wsum<Q, false>(X, Y, Z, j0, j1, qx, qy, na, aL0, Sw, Swz);
    }
}

// The query at tile position `pos` (< p.n) of a problem.
__device__ __forceinline__ int query_at(const ProblemF32& p, int pos) {
    return p.order ? p.order[pos] : pos;
}

// A lane's queries of the tile starting at position `base`: positions qi
// (lanes past the end load the last query and write nothing), the queries'
// own indices qs (where their results go) and coordinates.
template <int Q>
__device__ __forceinline__ void load_queries(const ProblemF32& p, int base, int (&qi)[Q],
                                             int (&qs)[Q], float (&qx)[Q], float (&qy)[Q]) {
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        qi[s] = base + s * kWaveSize + lane;
        qs[s] = query_at(p, qi[s] < p.n ? qi[s] : p.n - 1);
        qx[s] = p.qx[qs[s]];
        qy[s] = p.qy[qs[s]];
    }
}

// ---- one tile of 64*Q queries, both passes over all m points ---------------
// A problem's fields that are needed only after a scan (the alpha
// parameters, the output pointers) are read through a pointer to the
// problem in the kernarg segment (or in the batch's table), laundered by an
// empty asm at the point of use: loads of kernel arguments otherwise all go
// to the kernel's entry, and their SGPRs stay live through the scans, which
// costs resident waves (on gfx950 8 per SIMD up to 80 SGPRs, 7 up to about
// 88, 6 beyond).
typedef const __attribute__((address_space(4))) ProblemF32* prob_ptr;
typedef const __attribute__((address_space(4))) AlphaParams* alpha_ptr;

template <typename T>
__device__ __forceinline__ T launder(T ptr) {
    asm volatile("" : "+s"(ptr));
    return ptr;
}

__device__ __forceinline__ AlphaParams load_alpha(alpha_ptr a) {
    AlphaParams ap;
#pragma unroll
    for (int j = 0; j < 5; ++j) ap.levels[j] = a->levels[j];
    ap.R_min = a->R_min;
    ap.R_max = a->R_max;
    ap.r_exp = a->r_exp;
    ap.k = a->k;
    return ap;
}

// Pass-1 result of one lane's queries: the pass-2 terms (Eq. 2-6) and the
// diagnostic outputs (lp: the problem, read late).
template <int K, int Q, bool TRACK>
__device__ __forceinline__ void tile_powers(prob_ptr lp, const int (&qi)[Q], const int (&qs)[Q],
                                            const float (&top)[Q][K],
                                            const int (&tix)[TRACK ? Q : 1][TRACK ? K : 1],
                                            float (&na)[Q], float (&aL0)[Q], float (&d2min)[Q],
                                            int& ipw) {
    const prob_ptr L = launder(lp);
    const AlphaParams ap = load_alpha(&L->ap);
    const int n = L->n;
    double* const r_obs_out = L->r_obs;
    double* const alpha_out = L->alpha;
    const int pad = K - ap.k;
    ipw = 0;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        double r_obs, al;
        query_power<K>(top[s], ap, r_obs, al, na[s], aL0[s], d2min[s]);
        if (Q == 1) ipw = integer_power(al, d2min[s]);
        if (qi[s] < n) {
            if (r_obs_out) r_obs_out[qs[s]] = r_obs;
            if (alpha_out) alpha_out[qs[s]] = al;
            if constexpr (TRACK) {
                int32_t* const knn = L->knn;
#pragma unroll
                for (int i = 0; i < K; ++i)
                    if (i >= pad) knn[(int64_t)qs[s] * ap.k + (i - pad)] = tix[s][i];
            }
        }
    }
}

template <int K, int Q, bool TRACK>
__device__ __forceinline__ void fused_tile(const ProblemF32& p, prob_ptr lp, int base) {
    int qi[Q], qs[Q];
    float qx[Q], qy[Q];
    load_queries<Q>(p, base, qi, qs, qx, qy);

    float top[Q][K];
    int tix[TRACK ? Q : 1][TRACK ? K : 1];
    init_lists<K, Q, TRACK>(top, tix, p.ap.k);
    scan_knn<K, Q, TRACK>(as_const(p.dx), as_const(p.dy), 0, p.m, qx, qy, top, tix);

    float na[Q], aL0[Q], d2min[Q];
    int ipw;
    tile_powers<K, Q, TRACK>(lp, qi, qs, top, tix, na, aL0, d2min, ipw);

    double Sw[Q], Swz[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) Sw[s] = Swz[s] = 0.0;
    scan_wsum_any<Q>(as_const(p.dx), as_const(p.dy), as_const(p.dz), 0, p.m, qx, qy, na, aL0, Sw,
                     Swz, ipw, sqrtf(d2min[0]), p.zmax);

    const prob_ptr L = launder(lp);
    float* const out = L->out;
    const int n = L->n;
#pragma unroll
    for (int s = 0; s < Q; ++s)
        if (qi[s] < n) out[qs[s]] = (float)(Swz[s] / Sw[s]);
}

// Arguments of the speculative launch, one struct so that the kernel finds
// the workspace at a known place in its kernarg segment.
struct SpecArgs {
    ProblemF32 p;
    DeferWorkspace ws;
};
typedef const __attribute__((address_space(4))) SpecArgs* spec_args_ptr;

// One tile of the speculative launch: pass 1 with the sums of p.spec_power
// (knn_speculative), and the output of every lane whose sums stand; the
// other lanes' pass-2 terms go to ws.qpar and their bits to ws.mask[tile],
// for the deferred pass 2.  Keeping pass 2 out of this kernel keeps it under
// 80 SGPRs (8 waves per SIMD), and the deferred queries' pass 2, split into
// data segments, runs spread over the chip instead of as long waves at the
// end.
template <int K>
__device__ __forceinline__ void spec_tile(const ProblemF32& p, spec_args_ptr ka, int tile) {
    int qi[1], qs[1];
    float qx[1], qy[1];
    load_queries<1>(p, tile * kWaveSize, qi, qs, qx, qy);
    float top[1][K];
    int tix[1][1];
    init_lists<K, 1, false>(top, tix, p.ap.k);
    double Sw = 0.0, Swz = 0.0;
    const bool covered = knn_maybe_speculative<K>(p, 0, p.m, qx[0], qy[0], top[0], Sw, Swz);

    float na[1], aL0[1], d2min[1];
    int ipw;
    tile_powers<K, 1, false>(&ka->p, qi, qs, top, tix, na, aL0, d2min, ipw);
    const spec_args_ptr L = launder(ka);
    const int n = L->p.n;
    // the power whose sums cover every point
    const int spec = covered ? L->p.spec_power : 0;
    // A lane's sums stand when its pass 2 would be the unscaled loop of that
    // same power: what a wave of such queries computes (scan_wsum_any's
    // choice), bit for bit.
    const bool keep = spec != 0 && ipw == spec && unscaled_ok(aL0[0], L->p.zmax);
    if (keep && qi[0] < n) L->p.out[qs[0]] = (float)(Swz / Sw);
    const bool defer = !keep && qi[0] < n;
    const unsigned long long mask = __ballot(defer);
    // the tile index again from lane 0's position (a VGPR live anyway), so
    // that no SGPR holds it through the scan
    const int t = __builtin_amdgcn_readfirstlane(qi[0]) / kWaveSize;
    if (lane_id() == 0) L->ws.mask[t] = mask;
    if (defer) {
        float* const qpar = L->ws.qpar;
        qpar[qi[0]] = na[0];
        qpar[n + qi[0]] = aL0[0];
        qpar[2 * n + qi[0]] = sqrtf(d2min[0]);
        qpar[3 * n + qi[0]] = (float)ipw;
    }
}

template <int K, int Q, bool TRACK>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_fused(ProblemF32 p) {
    // p is the kernel's only explicit argument: it starts the kernarg segment
    fused_tile<K, Q, TRACK>(p, (prob_ptr)__builtin_amdgcn_kernarg_segment_ptr(),
                            wave_id() * Q * kWaveSize);
}

// The speculative launch: one wave per tile (see spec_tile).
template <int K>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_fused_spec(SpecArgs a) {
    const int tile = wave_id();
    if (tile * kWaveSize >= a.p.n) return;
    spec_tile<K>(a.p, (spec_args_ptr)__builtin_amdgcn_kernarg_segment_ptr(), tile);
}

// ---- batched: one wave per (problem, tile) item -------------------------------
template <int K>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_batch(const ProblemF32* __restrict__ probs,
                                                             const BatchItem* __restrict__ items,
                                                             int n_items) {
    const int it = wave_id();
    if (it >= n_items) return;
    const BatchItem w = items[it];
    fused_tile<K, 1, false>(probs[w.problem], (prob_ptr)&probs[w.problem], w.base);
}

// Per-segment k-nearest lists keep only the k real entries of each list,
// laid out [segment][k][n], so the layout depends on the problem's k alone
// and not on the register bucket of the kernel that writes or reads it.
template <int K>
__device__ __forceinline__ void store_partial(const float (&top)[K], const ProblemF32& p, int seg,
                                              int q, float* __restrict__ part) {
    if (q >= p.n) return;
    const int k = p.ap.k, pad = K - k;
    // padding entries are -inf, real ones >= 0: a test of the value, not of
    // i >= pad, whose uniform masks would stay in SGPRs through the scan
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (top[i] > -INFINITY) part[((int64_t)seg * k + (i - pad)) * p.n + q] = top[i];
}

// Fold the segment lists of query q in segment order (so equal distances
// keep scan order), then alpha and the pass-2 exponent terms.
template <int K>
__device__ __forceinline__ void merge_tile(const ProblemF32& p, const SplitPlan& sp,
                                           const float* __restrict__ part, float* __restrict__ qpar,
                                           int q) {
    const int k = p.ap.k;
    float top[1][K];
    int tix[1][1];
    init_lists<K, 1, false>(top, tix, k);
    for (int seg = 0; seg < sp.segments; ++seg) {
        for (int i = 0; i < k; ++i) {
            const float v = part[((int64_t)seg * k + i) * p.n + q];
            if (v < top[0][K - 1]) list_insert<K>(top[0], v);
        }
    }
    double r_obs, al;
    float na, aL0, d2min;
    query_power<K>(top[0], p.ap, r_obs, al, na, aL0, d2min);
    qpar[q] = na;
    qpar[p.n + q] = aL0;
    qpar[2 * p.n + q] = sqrtf(d2min);
    qpar[3 * p.n + q] = (float)integer_power(al, d2min);
    const int src = query_at(p, q);
    if (p.r_obs) p.r_obs[src] = r_obs;
    if (p.alpha) p.alpha[src] = al;
}

// ---- split-m ------------------------------------------------------------------
// End of the segment that starts at j0 (< m), formed in 64 bits: j0 + seg_len
// can pass 2^31 for the largest m.
__device__ __forceinline__ int seg_end(int m, int j0, int seg_len) {
    return (int)min((int64_t)m, (int64_t)j0 + seg_len);
}

// Waves are numbered segment-major so that the waves of one workgroup share a
// data segment.
// With p.spec_power set, an item also forms its segment's unscaled sums of
// that power (as the speculative single pass does for the whole range) and
// writes them where the segment's pass-2 item would, marking
// ws.seg_ok[seg][tile]; the merge then decides per tile whether pass 2 is
// needed at all.  The sums are those of the pass-2 item bit for bit (same
// batches from the segment start, same order and rounding).
template <int K>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_knn_part(ProblemF32 p, SplitPlan sp,
                                                                SplitWorkspace ws) {
    const int wave = wave_id();
    const int seg = wave / sp.tiles;
    const int tile = wave - seg * sp.tiles;
    if (seg >= sp.segments) return;
    const int j0 = seg * sp.seg_len;
    const int j1 = seg_end(p.m, j0, sp.seg_len);
    int qi[1], qs[1];
    float qx[1], qy[1];
    load_queries<1>(p, tile * kWaveSize, qi, qs, qx, qy);
    float top[1][K];
    int tix[1][1];
    init_lists<K, 1, false>(top, tix, p.ap.k);
    double Sw = 0.0, Swz = 0.0;
    const bool covered = knn_maybe_speculative<K>(p, j0, j1, qx[0], qy[0], top[0], Sw, Swz);
    store_partial<K>(top[0], p, seg, qi[0], ws.part);
    if (p.spec_power) {
        if (lane_id() == 0) ws.seg_ok[(int64_t)seg * sp.tiles + tile] = covered;
        if (covered && qi[0] < p.n) {
            ws.psum[((int64_t)seg * 2 + 0) * p.n + qi[0]] = Sw;
            ws.psum[((int64_t)seg * 2 + 1) * p.n + qi[0]] = Swz;
        }
    }
}

// Merge the segment lists of each query (in segment order), then alpha.
// A wave here is one 64-query tile.  With p.spec_power set it also decides
// whether the tile's speculative sums stand: every segment formed them and
// pass 2 would take the unscaled loop of that power in every lane (the
// choice scan_wsum_any makes).
template <int K>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_knn_merge(ProblemF32 p, SplitPlan sp,
                                                                 SplitWorkspace ws) {
    const int q = blockIdx.x * kGroupSize + threadIdx.x;
    if (q >= p.n) return;
    merge_tile<K>(p, sp, ws.part, ws.qpar, q);
    if (p.spec_power) {
        const int tile = q / kWaveSize;
        bool ok = (int)ws.qpar[3 * p.n + q] == p.spec_power && unscaled_ok(ws.qpar[p.n + q], p.zmax);
        for (int seg = 0; seg < sp.segments; ++seg) ok &= ws.seg_ok[(int64_t)seg * sp.tiles + tile] != 0;
        ok = __all(ok);
        if (lane_id() == 0) ws.tile_ok[tile] = ok;
    }
}

// Per-segment weighted sums: psum[(seg * 2 + {0: sum w, 1: sum w z}) * n + q]
// by pass-1 position q.  Items of tiles whose speculative sums stand
// (tile_ok, may be null) have nothing to do.  With `regroup` (may be null) a
// wave takes the 64 positions regroup[64 t ..] instead of tile t's: the
// positions sorted by the loop their pass 2 takes, so that nearly every
// wave takes one loop for all its lanes (pass 2 has no per-wave state but
// that choice).
__global__ __launch_bounds__(kGroupSize) void aidw_f32_wsum_part(ProblemF32 p, SplitPlan sp,
                                                                 const float* __restrict__ qpar,
                                                                 double* __restrict__ psum,
                                                                 const int* __restrict__ tile_ok,
                                                                 const int* __restrict__ regroup) {
    const int wave = wave_id();
    const int seg = wave / sp.tiles;
    const int tile = wave - seg * sp.tiles;
    if (seg >= sp.segments) return;
    if (tile_ok && tile_ok[tile]) return;
    const int j0 = seg * sp.seg_len;
    const int j1 = seg_end(p.m, j0, sp.seg_len);
    const int slot = tile * kWaveSize + lane_id();
    const int sc = slot < p.n ? slot : p.n - 1;
    const int c = regroup ? regroup[sc] : sc;  // pass-1 position
    const int qs = query_at(p, c);
    float qx[1] = {p.qx[qs]}, qy[1] = {p.qy[qs]};
    float na[1] = {qpar[c]}, aL0[1] = {qpar[p.n + c]};
    double Sw[1] = {0.0}, Swz[1] = {0.0};
    scan_wsum_any<1>(as_const(p.dx), as_const(p.dy), as_const(p.dz), j0, j1, qx, qy, na, aL0, Sw,
                     Swz, (int)qpar[3 * p.n + c], qpar[2 * p.n + c], p.zmax);
    if (slot < p.n) {
        psum[((int64_t)seg * 2 + 0) * p.n + c] = Sw[0];
        psum[((int64_t)seg * 2 + 1) * p.n + c] = Swz[0];
    }
}

// The pass-2 loop of each position as a sort key: 2 A + 1 for the unscaled
// and 2 A for the scaled loop of a whole power A, 1 for the exp2/log2 loop
// of a query on a data point (the guarded form), 0 for the exp2/log2 loop.
__global__ __launch_bounds__(256) void aidw_f32_pass2_keys(ProblemF32 p,
                                                           const float* __restrict__ qpar,
                                                           unsigned* __restrict__ keys) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= p.n) return;
    const int ipw = (int)qpar[3 * p.n + c];
    const float aL0 = qpar[p.n + c];
    keys[c] = ipw != 0 ? (unsigned)(2 * ipw + (unscaled_ok(aL0, p.zmax) ? 1 : 0))
                       : (coincident(aL0) ? 1u : 0u);
}

__global__ __launch_bounds__(kGroupSize) void aidw_f32_wsum_reduce(ProblemF32 p, SplitPlan sp,
                                                                   const double* __restrict__ psum) {
    const int q = blockIdx.x * kGroupSize + threadIdx.x;
    if (q >= p.n) return;
    double Sw = 0.0, Swz = 0.0;
    for (int seg = 0; seg < sp.segments; ++seg) {
        Sw += psum[((int64_t)seg * 2 + 0) * p.n + q];
        Swz += psum[((int64_t)seg * 2 + 1) * p.n + q];
    }
    p.out[query_at(p, q)] = (float)(Swz / Sw);
}


// ---- deferred pass 2 of the queries whose speculation failed ----------------
// `count` queries (only known on the device), in groups of 64 consecutive
// list entries, run as (group, data segment) items, S segments each with S
// chosen so that groups * S is about ws.target waves (one round of the
// chip): a few deferred queries then still fill the device.  Segments are
// whole 16-point batches of at least kDeferMinSegment points.
constexpr int kDeferMinSegment = 2048;

// At least ceil(m / kDeferL2Segment) segments (at most kDeferMaxL2Segments),
// so that when many queries are deferred the waves resident together read
// one segment of about 1.5 MB of x, y, z that stays in the XCD's L2 (as the
// grid mode's pass 2 does).
constexpr int kDeferL2Segment = 131072;
constexpr int kDeferMaxL2Segments = 8;

__device__ __forceinline__ void defer_plan(int m, int count, int target, int& segs, int& seg_len) {
    int want = count > 0 ? (target + count - 1) / count : 1;
    want = max(want, min(kDeferMaxL2Segments, (m + kDeferL2Segment - 1) / kDeferL2Segment));
    want = max(1, min(want, m / kDeferMinSegment));
    seg_len = (int)(((int64_t)m + want - 1) / want);
    seg_len = (seg_len + 15) & ~15;
    segs = (int)(((int64_t)m + seg_len - 1) / seg_len);
}

// The deferred queries' positions in ascending order, and their count, from
// the tiles' masks: one workgroup walks the tiles in chunks of 1024, a scan
// of the masks' bit counts giving each tile its first list slot.
constexpr int kDeferListThreads = 1024;

__global__ __launch_bounds__(kDeferListThreads) void aidw_f32_defer_list(int tiles,
                                                                          DeferWorkspace ws) {
    constexpr int W = kDeferListThreads / kWaveSize;
    __shared__ int wave_total[W];
    const int lane = lane_id(), w = threadIdx.x / kWaveSize;
    int carry = 0;
    for (int t0 = 0; t0 < tiles; t0 += kDeferListThreads) {
        const int t = t0 + (int)threadIdx.x;
        unsigned long long mk = t < tiles ? ws.mask[t] : 0ull;
        const int c = __popcll(mk);
        int incl = c;  // inclusive scan of the bit counts within the wave
        for (int o = 1; o < kWaveSize; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (lane == kWaveSize - 1) wave_total[w] = incl;
        __syncthreads();
        int before = 0, chunk = 0;
        for (int v = 0; v < W; ++v) {
            before += v < w ? wave_total[v] : 0;
            chunk += wave_total[v];
        }
        int slot = carry + before + incl - c;
        while (mk) {
            ws.list[slot++] = t * kWaveSize + (__ffsll((long long)mk) - 1);
            mk &= mk - 1ull;
        }
        carry += chunk;
        __syncthreads();  // wave_total is rewritten by the next chunk
    }
    if (threadIdx.x == 0) *ws.count = carry;
}

__device__ __forceinline__ int defer_count(const DeferWorkspace& ws) {
    return *(const __attribute__((address_space(4))) int*)ws.count;
}

// Item w: segment w / groups of list group w % groups (segment-major, so that
// the waves resident together read the same data segment).  Sums go to
// psum[(seg * 2 + {0, 1}) * groups * 64 + list slot].
__global__ __launch_bounds__(kGroupSize) void aidw_f32_defer_part(ProblemF32 p, DeferWorkspace ws) {
    const int count = defer_count(ws);
    const int groups = (count + kWaveSize - 1) / kWaveSize;
    int segs, seg_len;
    defer_plan(p.m, groups, ws.target, segs, seg_len);
    const int w = wave_id();
    if (w >= groups * segs) return;
    const int seg = w / groups;
    const int grp = w - seg * groups;
    const int j0 = seg * seg_len;
    const int j1 = seg_end(p.m, j0, seg_len);
    const int slot = grp * kWaveSize + lane_id();
    // lanes past the list's end repeat its last query and write slots that
    // the reduction skips
    const int c = ws.list[slot < count ? slot : count - 1];  // pass-1 position
    const int qs = query_at(p, c);
    const float* qp = ws.qpar;
    float qx[1] = {p.qx[qs]}, qy[1] = {p.qy[qs]};
    float na[1] = {qp[c]}, aL0[1] = {qp[p.n + c]};
    double Sw[1] = {0.0}, Swz[1] = {0.0};
    scan_wsum_any<1>(as_const(p.dx), as_const(p.dy), as_const(p.dz), j0, j1, qx, qy, na, aL0, Sw,
                     Swz, (int)qp[3 * p.n + c], qp[2 * p.n + c], p.zmax);
    const int64_t stride = (int64_t)groups * kWaveSize;
    ws.psum[(int64_t)seg * 2 * stride + slot] = Sw[0];
    ws.psum[((int64_t)seg * 2 + 1) * stride + slot] = Swz[0];
}

// The segments of each listed query added in order, then the ratio.
__global__ __launch_bounds__(kGroupSize) void aidw_f32_defer_reduce(ProblemF32 p,
                                                                    DeferWorkspace ws) {
    const int count = defer_count(ws);
    const int t = blockIdx.x * kGroupSize + threadIdx.x;
    if (t >= count) return;
    const int groups = (count + kWaveSize - 1) / kWaveSize;
    int segs, seg_len;
    defer_plan(p.m, groups, ws.target, segs, seg_len);
    const int64_t stride = (int64_t)groups * kWaveSize;
    double Sw = 0.0, Swz = 0.0;
    // in segment order; unrolled so that the loads of several segments are
    // in flight together
#pragma unroll 8
    for (int seg = 0; seg < segs; ++seg) {
        Sw += ws.psum[(int64_t)seg * 2 * stride + t];
        Swz += ws.psum[((int64_t)seg * 2 + 1) * stride + t];
    }
    p.out[query_at(p, ws.list[t])] = (float)(Swz / Sw);
}

// max |z| as the largest bit pattern of |z| (ordered like the values for
// non-negative floats; NaN patterns sort above infinity).
template <int T>
__device__ __forceinline__ void abs_max_block(const float* __restrict__ z, int m,
                                              float* __restrict__ out) {
    __shared__ unsigned s[T];
    constexpr unsigned kAbs = 0x7fffffffu;
    unsigned v = 0;
    int i = threadIdx.x;
    // four independent loads per step keep more of the walk in flight
    for (; i + 3 * T < m; i += 4 * T) {
        const unsigned a = __float_as_uint(z[i]) & kAbs, b = __float_as_uint(z[i + T]) & kAbs;
        const unsigned c = __float_as_uint(z[i + 2 * T]) & kAbs;
        const unsigned d = __float_as_uint(z[i + 3 * T]) & kAbs;
        v = max(v, max(max(a, b), max(c, d)));
    }
    for (; i < m; i += T) v = max(v, __float_as_uint(z[i]) & kAbs);
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = __uint_as_float(s[0]);
}

__global__ __launch_bounds__(1024) void aidw_abs_max(const float* __restrict__ z, int m,
                                                     float* __restrict__ out, int* clear) {
    if (clear && threadIdx.x == 0) *clear = 0;
    abs_max_block<1024>(z, m, out);
}

__global__ __launch_bounds__(256) void aidw_abs_max_tasks(const AbsMaxTask* __restrict__ tasks) {
    const AbsMaxTask t = tasks[blockIdx.x];
    abs_max_block<256>(t.z, t.m, t.out);
}

// ---- serving: fused tiles and split segments in one launch -----------------
// Pass-1 segment items write their partial lists; the last segment of a tile
// to arrive (an atomic count per tile, after a device-scope release fence)
// merges the tile's lists in segment order and writes the exponent terms.
// Pass-2 segment items run in a later launch; the last to arrive adds the
// tile's segment sums in order and writes the outputs.  The arithmetic is
// that of the split kernels above, so results do not depend on the order in
// which items run.
__device__ __forceinline__ bool last_arrival(int* counter, int expected) {
    __threadfence();  // publish this item's partial results device-wide
    int old = 0;
    if (lane_id() == 0) old = atomicAdd(counter, 1);
    old = __builtin_amdgcn_readfirstlane(old);
    const bool last = old == expected - 1;
    if (last) __threadfence();  // and see every other segment's
    return last;
}

template <int K>
__device__ __forceinline__ void serve_item(const ServeJob& J, const ServeItem& it) {
    const ProblemF32& p = J.p;
    if (it.phase == kServeFused) {
        fused_tile<K, 1, false>(p, (prob_ptr)&J.p, it.tile * kWaveSize);
        return;
    }
    const int j0 = it.seg * J.sp.seg_len;
    const int j1 = seg_end(p.m, j0, J.sp.seg_len);
    int qi[1], qs[1];
    float qx[1], qy[1];
    load_queries<1>(p, it.tile * kWaveSize, qi, qs, qx, qy);
    if (it.phase == kServeKnn) {
        float top[1][K];
        int tix[1][1];
        init_lists<K, 1, false>(top, tix, p.ap.k);
        scan_knn<K, 1, false>(as_const(p.dx), as_const(p.dy), j0, j1, qx, qy, top, tix);
        store_partial<K>(top[0], p, it.seg, qi[0], J.ws.part);
        if (last_arrival(&J.knn_arrivals[it.tile], J.sp.segments) && qi[0] < p.n)
            merge_tile<K>(p, J.sp, J.ws.part, J.ws.qpar, qi[0]);
        return;
    }
    const int c = qi[0] < p.n ? qi[0] : p.n - 1;
    float na[1] = {J.ws.qpar[c]}, aL0[1] = {J.ws.qpar[p.n + c]};
    double Sw[1] = {0.0}, Swz[1] = {0.0};
    scan_wsum_any<1>(as_const(p.dx), as_const(p.dy), as_const(p.dz), j0, j1, qx, qy, na, aL0, Sw,
                     Swz, (int)J.ws.qpar[3 * p.n + c], J.ws.qpar[2 * p.n + c], p.zmax);
    if (qi[0] < p.n) {
        J.ws.psum[((int64_t)it.seg * 2 + 0) * p.n + qi[0]] = Sw[0];
        J.ws.psum[((int64_t)it.seg * 2 + 1) * p.n + qi[0]] = Swz[0];
    }
    if (last_arrival(&J.sum_arrivals[it.tile], J.sp.segments) && qi[0] < p.n) {
        double sw = 0.0, swz = 0.0;
        for (int seg = 0; seg < J.sp.segments; ++seg) {
            sw += J.ws.psum[((int64_t)seg * 2 + 0) * p.n + qi[0]];
            swz += J.ws.psum[((int64_t)seg * 2 + 1) * p.n + qi[0]];
        }
        p.out[qs[0]] = (float)(swz / sw);
    }
}

template <int K, bool TRACK>
__global__ __launch_bounds__(kGroupSize) void aidw_f32_serve(const ServeJob* __restrict__ jobs,
                                                             const ServeItem* __restrict__ items,
                                                             int n_items) {
    const int it = wave_id();
    if (it >= n_items) return;
    const ServeItem w = items[it];
    if constexpr (TRACK)
        fused_tile<K, 1, true>(jobs[w.job].p, (prob_ptr)&jobs[w.job].p,
                               w.tile * kWaveSize);  // jobs with knn_idx: unsplit
    else
        serve_item<K>(jobs[w.job], w);
}

// ---- host-side launchers ----------------------------------------------------------
size_t occupancy_lds(const LaunchF32& cfg) {
    // Each workgroup holds one wave per SIMD, so W resident workgroups per CU
    // mean W waves per SIMD; reserving kLdsPerCU / W bytes caps it at W.
    if (cfg.max_waves_per_simd <= 0) return 0;
    return (size_t)(kLdsPerCU / cfg.max_waves_per_simd) & ~(size_t)1023;
}

template <typename Kern>
hipError_t allow_lds(Kern kern, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

unsigned groups_for(int64_t waves) {
    return (unsigned)((waves + kWavesPerGroup - 1) / kWavesPerGroup);
}

template <int K, int Q, bool TRACK>
hipError_t launch_fused(const ProblemF32& p, const LaunchF32& cfg, hipStream_t stream) {
    const int64_t tiles = (p.n + (int64_t)kWaveSize * Q - 1) / ((int64_t)kWaveSize * Q);
    const size_t lds = occupancy_lds(cfg);
    hipError_t e = allow_lds(aidw_f32_fused<K, Q, TRACK>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((aidw_f32_fused<K, Q, TRACK>), dim3(groups_for(tiles)), dim3(kGroupSize),
                       lds, stream, p);
    return hipGetLastError();
}

template <int K>
hipError_t launch_split(const ProblemF32& p, const SplitPlan& sp, const SplitWorkspace& ws,
                        hipStream_t stream) {
    const unsigned g_part = groups_for((int64_t)sp.tiles * sp.segments);
    const unsigned g_query = (unsigned)((p.n + kGroupSize - 1) / kGroupSize);
    hipLaunchKernelGGL((aidw_f32_knn_part<K>), dim3(g_part), dim3(kGroupSize), 0, stream, p, sp,
                       ws);
    hipLaunchKernelGGL((aidw_f32_knn_merge<K>), dim3(g_query), dim3(kGroupSize), 0, stream, p, sp,
                       ws);
    const int* regroup = nullptr;
    if (ws.p2order && !p.spec_power) {
        hipLaunchKernelGGL(aidw_f32_pass2_keys, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0,
                           stream, p, ws.qpar, ws.p2key);
        const hipError_t e = launch_key_order(ws.p2key, p.n, ws.p2hist, ws.p2order, stream);
        if (e != hipSuccess) return e;
        regroup = ws.p2order;
    }
    hipLaunchKernelGGL(aidw_f32_wsum_part, dim3(g_part), dim3(kGroupSize), 0, stream, p, sp,
                       ws.qpar, ws.psum, p.spec_power ? ws.tile_ok : nullptr, regroup);
    hipLaunchKernelGGL(aidw_f32_wsum_reduce, dim3(g_query), dim3(kGroupSize), 0, stream, p, sp,
                       ws.psum);
    return hipGetLastError();
}

template <int K>
hipError_t launch_single_k(const ProblemF32& p, const LaunchF32& cfg, const SplitPlan* sp,
                           const SplitWorkspace* ws, hipStream_t stream) {
    if (p.knn) return launch_fused<K, 1, true>(p, cfg, stream);
    if (sp && sp->segments > 1) return launch_split<K>(p, *sp, *ws, stream);
    switch (cfg.q_per_lane) {
        case 1: return launch_fused<K, 1, false>(p, cfg, stream);
        case 2: return launch_fused<K, 2, false>(p, cfg, stream);
        case 4: return launch_fused<K, 4, false>(p, cfg, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int K>
hipError_t launch_batch_k(const BatchLaunch& b, hipStream_t stream) {
    if (b.n_tasks > 0)
        hipLaunchKernelGGL(aidw_abs_max_tasks, dim3((unsigned)b.n_tasks), dim3(256), 0, stream,
                           b.tasks);
    const hipError_t e = launch_query_order(b.order, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((aidw_f32_batch<K>), dim3(groups_for(b.n_items)), dim3(kGroupSize), 0,
                       stream, b.problems, b.items, b.n_items);
    return hipGetLastError();
}

template <int K>
hipError_t launch_serve_k(const ServeLaunch& sl, hipStream_t stream) {
    if (sl.n_tasks > 0)
        hipLaunchKernelGGL(aidw_abs_max_tasks, dim3((unsigned)sl.n_tasks), dim3(256), 0, stream,
                           sl.tasks);
    if (sl.track)
        hipLaunchKernelGGL((aidw_f32_serve<K, true>), dim3(groups_for(sl.n_items)),
                           dim3(kGroupSize), 0, stream, sl.jobs, sl.items, sl.n_items);
    else
        hipLaunchKernelGGL((aidw_f32_serve<K, false>), dim3(groups_for(sl.n_items)),
                           dim3(kGroupSize), 0, stream, sl.jobs, sl.items, sl.n_items);
    return hipGetLastError();
}

#define AIDW_K_DISPATCH(K_RUNTIME, CALL) \
    switch (K_RUNTIME) {                 \
        case 4: return CALL(4);          \
        case 8: return CALL(8);          \
        case 10: return CALL(10);        \
        case 12: return CALL(12);        \
        case 16: return CALL(16);        \
        case 20: return CALL(20);        \
        case 24: return CALL(24);        \
        case 32: return CALL(32);        \
        default: break;                  \
    }

}  // namespace

hipError_t launch_aidw_f32(const ProblemF32& p, const LaunchF32& cfg, const SplitPlan* sp,
                           const SplitWorkspace* ws, hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
#define CALL(KK) launch_single_k<KK>(p, cfg, sp, ws, stream)
    AIDW_K_DISPATCH(k_bucket(p.ap.k), CALL)
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_abs_max(const float* z, int m, float* out, hipStream_t s, int* clear) {
    hipLaunchKernelGGL(aidw_abs_max, dim3(1), dim3(1024), 0, s, z, m, out, clear);
    return hipGetLastError();
}

// Most (group, segment) items the deferred pass 2 can have: defer_plan gives
// g groups of 64 deferred queries at most max(ceil(target / g),
// kDeferMaxL2Segments) segments, so g * segments <= max(target + g,
// kDeferMaxL2Segments * g), with g <= tiles.  The workspace and the launch
// both take this.
static int64_t defer_items_max(int64_t tiles, int target) {
    return std::max<int64_t>(target + tiles, kDeferMaxL2Segments * tiles);
}

size_t spec_workspace_bytes(int64_t n, int target, DeferWorkspace* ws, char* base) {
    const int64_t tiles = (n + kWaveSize - 1) / kWaveSize;
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    const int64_t items = defer_items_max(tiles, target);
    const size_t sizes[5] = {sizeof(int), sizeof(int) * (size_t)n, 4 * sizeof(float) * (size_t)n,
                             2 * sizeof(double) * (size_t)kWaveSize * (size_t)items,
                             sizeof(unsigned long long) * (size_t)tiles};
    size_t off[5], bytes = 0;
    for (int i = 0; i < 5; ++i) {
        off[i] = bytes;
        bytes += up(sizes[i]);
    }
    if (ws) {
        ws->count = reinterpret_cast<int*>(base + off[0]);
        ws->list = reinterpret_cast<int*>(base + off[1]);
        ws->qpar = reinterpret_cast<float*>(base + off[2]);
        ws->psum = reinterpret_cast<double*>(base + off[3]);
        ws->mask = reinterpret_cast<unsigned long long*>(base + off[4]);
        ws->target = target;
    }
    return bytes;
}

template <int K>
hipError_t launch_spec_k(const ProblemF32& p, const DeferWorkspace& ws, hipStream_t stream) {
    const int64_t tiles = (p.n + kWaveSize - 1) / kWaveSize;
    hipLaunchKernelGGL((aidw_f32_fused_spec<K>), dim3(groups_for(tiles)), dim3(kGroupSize), 0,
                       stream, SpecArgs{p, ws});
    hipLaunchKernelGGL(aidw_f32_defer_list, dim3(1), dim3(kDeferListThreads), 0, stream,
                       (int)tiles, ws);
    // one wave per possible item (the kernel reads the count and the plan;
    // waves past groups * segments return at once)
    hipLaunchKernelGGL(aidw_f32_defer_part, dim3(groups_for(defer_items_max(tiles, ws.target))),
                       dim3(kGroupSize), 0, stream, p, ws);
    hipLaunchKernelGGL(aidw_f32_defer_reduce,
                       dim3((unsigned)((tiles * kWaveSize + kGroupSize - 1) / kGroupSize)),
                       dim3(kGroupSize), 0, stream, p, ws);
    return hipGetLastError();
}

hipError_t launch_abs_max_tasks(const AbsMaxTask* tasks, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(aidw_abs_max_tasks, dim3((unsigned)count), dim3(256), 0, s, tasks);
    return hipGetLastError();
}

hipError_t launch_aidw_f32_pass2(const ProblemF32& p, SplitPlan sp, const float* qpar,
                                 double* psum, hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
    sp.tiles = (int)((p.n + kWaveSize - 1) / kWaveSize);
    hipLaunchKernelGGL(aidw_f32_wsum_part, dim3(groups_for((int64_t)sp.segments * sp.tiles)),
                       dim3(kGroupSize), 0, stream, p, sp, qpar, psum, (const int*)nullptr,
                       (const int*)nullptr);
    hipLaunchKernelGGL(aidw_f32_wsum_reduce, dim3((unsigned)((p.n + kGroupSize - 1) / kGroupSize)),
                       dim3(kGroupSize), 0, stream, p, sp, psum);
    return hipGetLastError();
}

hipError_t launch_aidw_f32_spec(const ProblemF32& p, const DeferWorkspace& ws,
                                hipStream_t stream) {
    if (p.n <= 0) return hipSuccess;
    if (p.spec_power < 1 || p.spec_power > 8) return hipErrorInvalidValue;
#define CALL(KK) launch_spec_k<KK>(p, ws, stream)
    AIDW_K_DISPATCH(k_bucket(p.ap.k), CALL)
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_aidw_f32_batch(const BatchLaunch& b, hipStream_t stream) {
    if (b.n_items <= 0) return hipSuccess;
#define CALL(KK) launch_batch_k<KK>(b, stream)
    AIDW_K_DISPATCH(b.K, CALL)
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_aidw_f32_serve(const ServeLaunch& sl, hipStream_t stream) {
    if (sl.n_items <= 0) return hipSuccess;
#define CALL(KK) launch_serve_k<KK>(sl, stream)
    AIDW_K_DISPATCH(sl.K, CALL)
#undef CALL
    return hipErrorInvalidValue;
}

}  // namespace aidw
