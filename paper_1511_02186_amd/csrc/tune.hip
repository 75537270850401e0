// Autotuner of libaidw: times candidate launch shapes of the FP32-scaled
// path on synthetic points and keeps the fastest per size class
// (declared in include/aidw.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "handle.h"

using namespace aidw::detail;

namespace {

// Uniform points in [0, 1]^2 from a counter-based hash (splitmix64), one
// value per thread; z = x + y.
__device__ __forceinline__ float unit_hash(uint64_t i) {
    uint64_t x = i + 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (float)(x >> 40) * (1.0f / 16777216.0f);
}

__global__ void fill_points(float* __restrict__ xy, float* __restrict__ z, int64_t count,
                            uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float x = unit_hash(seed + 2 * (uint64_t)i);
    const float y = unit_hash(seed + 2 * (uint64_t)i + 1);
    xy[i] = x;
    xy[count + i] = y;
    if (z) z[i] = x + y;
}

// Clustered points: 90 % from 16 isotropic Gaussians (centres uniform in
// [0, 1]^2, sigma log-uniform in [1e-4, 1e-1], normals by the Box-Muller
// transform), 10 % uniform; z = x + y.  With uniform queries alpha then
// varies from query to query (the general-alpha pass 2), where uniform data
// give alpha_5 nearly everywhere.
__global__ void fill_clustered(float* __restrict__ xy, float* __restrict__ z, int64_t count,
                               uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t b = seed + 4 * (uint64_t)i;
    float x, y;
    if (unit_hash(b) < 0.1f) {
        x = unit_hash(b + 1);
        y = unit_hash(b + 2);
    } else {
        const uint64_t c = (uint64_t)(unit_hash(b + 1) * 16.0f);  // 0..15
        const uint64_t cb = (seed ^ 0x5DEECE66Dull) + 4 * c;
        const float cx = unit_hash(cb), cy = unit_hash(cb + 1);
        const float sigma = exp10f(-4.0f + 3.0f * unit_hash(cb + 2));
        const float u1 = fmaxf(unit_hash(b + 2), 1.0f / 16777216.0f), u2 = unit_hash(b + 3);
        const float r = sigma * sqrtf(-2.0f * logf(u1));
        float sn, cs;
        sincosf(6.2831853f * u2, &sn, &cs);
        x = cx + r * cs;
        y = cy + r * sn;
    }
    xy[i] = x;
    xy[count + i] = y;
    z[i] = x + y;
}

int log2_bucket(int64_t v) {
    int b = 0;
    while (((int64_t)1 << (b + 1)) <= v) ++b;
    return b;
}

}  // namespace

namespace aidw {
namespace detail {

bool tuned_shape(const aidw_ctx* h, int64_t m, int64_t n, int k, aidw_tuning* out) {
    const int km = log2_bucket(m), kn = log2_bucket(n), kb = k_bucket(k);
    for (const TuneEntry& e : h->tune_table)
        if (e.m_log2 == km && e.n_log2 == kn && e.K == kb) {
            *out = e.shape;
            return true;
        }
    return false;
}

}  // namespace detail
}  // namespace aidw

extern "C" {

aidw_status aidw_tune(aidw_t h, int64_t m, int64_t n, int k, double budget_s, aidw_tuning* best) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (m < 1 || n < 1 || m > INT32_MAX || n > INT32_MAX)
        return fail(AIDW_EINVAL, "need 1 <= m, n <= 2^31-1");
    if (k < 1 || k > AIDW_KMAX || k > m) return fail(AIDW_EINVAL, "k out of range");
    if (!(budget_s > 0)) budget_s = 10.0;

    // two data sets (uniform, clustered) sharing the uniform queries
    const size_t bytes = sizeof(float) * (6 * (size_t)m + 3 * (size_t)n) + 1024;
    void* mem = nullptr;
    aidw_status st = device_alloc(h, bytes, &mem);
    if (st != AIDW_OK) return st;
    float* dxy = static_cast<float*>(mem);
    float* dz = dxy + 2 * m;
    float* cxy = dz + m;
    float* cz = cxy + 2 * m;
    float* qxy = cz + m;
    float* out = qxy + 2 * n;
    const unsigned g_m = (unsigned)((m + 255) / 256), g_n = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(fill_points, dim3(g_m), dim3(256), 0, h->stream, dxy, dz, m, 17ull);
    hipLaunchKernelGGL(fill_clustered, dim3(g_m), dim3(256), 0, h->stream, cxy, cz, m, 23ull);
    hipLaunchKernelGGL(fill_points, dim3(g_n), dim3(256), 0, h->stream, qxy, (float*)nullptr, n,
                       1ull << 40);

    aidw_problem p;
    memset(&p, 0, sizeof p);
    p.precision = AIDW_FP32_SCALED;
    p.data_xy = dxy;
    p.data_z = dz;
    p.m = m;
    p.query_xy = qxy;
    p.n = n;
    p.k = k;
    for (int j = 0; j < 5; ++j) p.alpha_levels[j] = 1.0 + j;
    p.R_min = 0.0;
    p.R_max = 2.0;
    p.area = 1.0;
    p.out = out;
    p.flags = AIDW_FLAG_ASYNC;

    // Candidates: queries per lane x data segments (the automatic split, half
    // and twice as many, none) x occupancy cap (none, 4 waves per SIMD), and
    // for split launches with or without the speculative sums per segment.
    // Each is timed on both data sets; the least total wins.
    const aidw_tuning saved = h->tuning;
    h->tuning = aidw_tuning{1, 0, 0};
    const aidw::SplitPlan autoplan = split_plan_for(h, aidw_tuning{1, 0, 0}, m, n);
    std::vector<int> segs{1};
    if (autoplan.segments > 1)
        for (int s : {autoplan.segments / 2, autoplan.segments, autoplan.segments * 2})
            if (s > 1 && std::find(segs.begin(), segs.end(), s) == segs.end()) segs.push_back(s);
    std::vector<aidw_tuning> cands;
    for (int q : {1, 2, 4})
        for (int s : segs)
            for (int cap : {0, 4})
                for (int spec : {0, 2}) {
                    if (s > 1 && q != 1) continue;      // split launches use one query per lane
                    if (spec == 2 && s == 1) continue;  // per-segment sums need segments
                    cands.push_back(aidw_tuning{q, cap, s, spec});
                }
    const void* data_sets[2][2] = {{dxy, dz}, {cxy, cz}};

    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        h->tuning = saved;
        device_free(h, mem, bytes);
        return hip_fail(he, "hipEventCreate");
    }
    double spent = 0.0, best_ms = 1e300;
    aidw_tuning best_t = cands[0];
    st = AIDW_OK;
    for (const aidw_tuning& c : cands) {
        if (spent > budget_s && best_ms < 1e300) break;
        h->tuning = c;
        double total = 0.0;
        for (const auto& ds : data_sets) {
            p.data_xy = ds[0];
            p.data_z = ds[1];
            float ms_best = 1e30f;
            for (int rep = 0; rep < 3 && st == AIDW_OK; ++rep) {  // first run warms up
                (void)hipEventRecord(e0, h->stream);
                st = aidw_interpolate_ex(h, &p);
                (void)hipEventRecord(e1, h->stream);
                if (st != AIDW_OK) break;
                he = hipEventSynchronize(e1);
                if (he != hipSuccess) {
                    st = hip_fail(he, "hipEventSynchronize");
                    break;
                }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                spent += ms * 1e-3;
                if (rep > 0) ms_best = std::min(ms_best, ms);
                if (spent > budget_s && rep > 0) break;
            }
            if (st != AIDW_OK) break;
            total += ms_best;
        }
        if (st != AIDW_OK) break;
        if (total < best_ms) {
            best_ms = total;
            best_t = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->tuning = saved;
    device_free(h, mem, bytes);
    if (st != AIDW_OK) return st;

    TuneEntry e{log2_bucket(m), log2_bucket(n), aidw::k_bucket(k), best_t, best_ms};
    bool replaced = false;
    for (TuneEntry& t : h->tune_table)
        if (t.m_log2 == e.m_log2 && t.n_log2 == e.n_log2 && t.K == e.K) {
            t = e;
            replaced = true;
        }
    if (!replaced) h->tune_table.push_back(e);
    if (best) *best = best_t;
    return AIDW_OK;
}

aidw_status aidw_tune_save(aidw_t h, const char* path) {
    ErrorScope es(h);
    if (!h || !path) return fail(AIDW_EINVAL, "handle or path is NULL");
    FILE* f = fopen(path, "w");
    if (!f) return fail(AIDW_EINVAL, "cannot write %s", path);
    fprintf(f, "{\"format\": \"libaidw-tuning-1\", \"entries\": [\n");
    for (size_t i = 0; i < h->tune_table.size(); ++i) {
        const TuneEntry& e = h->tune_table[i];
        fprintf(f,
                "  {\"m_log2\": %d, \"n_log2\": %d, \"K\": %d, \"q_per_lane\": %d, "
                "\"max_waves_per_simd\": %d, \"split_segments\": %d, \"speculate\": %d, "
                "\"ms\": %.6f}%s\n",
                e.m_log2, e.n_log2, e.K, e.shape.q_per_lane, e.shape.max_waves_per_simd,
                e.shape.split_segments, e.shape.speculate, e.ms,
                i + 1 < h->tune_table.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    return fclose(f) == 0 ? AIDW_OK : fail(AIDW_EINVAL, "cannot write %s", path);
}

aidw_status aidw_tune_load(aidw_t h, const char* path) {
    ErrorScope es(h);
    if (!h || !path) return fail(AIDW_EINVAL, "handle or path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return fail(AIDW_ENOTFOUND, "cannot read %s", path);
    std::vector<TuneEntry> table;
    char line[512];
    bool header = false;
    while (fgets(line, sizeof line, f)) {
        if (strstr(line, "\"libaidw-tuning-1\"")) header = true;
        TuneEntry e{};
        // entries written before the speculate field have none (0)
        if (sscanf(line,
                   " {\"m_log2\": %d, \"n_log2\": %d, \"K\": %d, \"q_per_lane\": %d, "
                   "\"max_waves_per_simd\": %d, \"split_segments\": %d, \"speculate\": %d, "
                   "\"ms\": %lf}",
                   &e.m_log2, &e.n_log2, &e.K, &e.shape.q_per_lane, &e.shape.max_waves_per_simd,
                   &e.shape.split_segments, &e.shape.speculate, &e.ms) != 8) {
            e = TuneEntry{};
            if (sscanf(line,
                       " {\"m_log2\": %d, \"n_log2\": %d, \"K\": %d, \"q_per_lane\": %d, "
                       "\"max_waves_per_simd\": %d, \"split_segments\": %d, \"ms\": %lf}",
                       &e.m_log2, &e.n_log2, &e.K, &e.shape.q_per_lane,
                       &e.shape.max_waves_per_simd, &e.shape.split_segments, &e.ms) != 7)
                continue;
        }
        const aidw_tuning& s = e.shape;
        if (aidw::k_bucket(e.K) != e.K || (s.q_per_lane != 1 && s.q_per_lane != 2 &&
                                           s.q_per_lane != 4) ||
            s.max_waves_per_simd < 0 || s.max_waves_per_simd > 8 || s.split_segments < 0 ||
            (s.speculate != 0 && s.speculate != 2)) {
            fclose(f);
            return fail(AIDW_EINVAL, "%s: invalid entry", path);
        }
        table.push_back(e);
    }
    fclose(f);
    if (!header) return fail(AIDW_EINVAL, "%s is not a libaidw tuning file", path);
    h->tune_table = table;
    return AIDW_OK;
}

}  // extern "C"
