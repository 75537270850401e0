// C-ABI entry points of libaidw (declared in include/aidw.h): handles,
// argument validation, per-problem constants and kernel dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "../../include/aidw.h"
#include "common.h"

namespace {

thread_local std::string g_last_error;

aidw_status fail(aidw_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
aidw_status fail(aidw_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

aidw_status hip_fail(hipError_t e, const char* what) {
    return fail(AIDW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

struct aidw_ctx {
    int device = 0;
    aidw_precision default_precision = AIDW_FP32_SCALED;
    size_t hbm_budget = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    int q_per_lane = 0;  // 0: automatic
};

namespace aidw {

int k_bucket(int k) {
    static const int buckets[] = {4, 8, 10, 12, 16, 20, 24, 32};
    for (int b : buckets)
        if (k <= b) return b;
    return -1;
}

}  // namespace aidw

namespace {

bool finite(double v) { return std::isfinite(v); }

// Host-side validation of everything the kernels assume (include/aidw.h).
aidw_status validate(const aidw_problem* p) {
    if (!p) return fail(AIDW_EINVAL, "problem is NULL");
    if (p->precision != AIDW_FP32_SCALED && p->precision != AIDW_FP64)
        return fail(AIDW_EINVAL, "unknown precision %d", (int)p->precision);
    if (p->m < 1 || p->m > INT32_MAX) return fail(AIDW_EINVAL, "m = %lld out of [1, 2^31-1]", (long long)p->m);
    if (p->n < 0 || p->n > INT32_MAX) return fail(AIDW_EINVAL, "n = %lld out of [0, 2^31-1]", (long long)p->n);
    if (p->k < 1 || p->k > AIDW_KMAX || (int64_t)p->k > p->m)
        return fail(AIDW_EINVAL, "k = %d out of [1, min(m, %d)]", p->k, AIDW_KMAX);
    if (!finite(p->area) || p->area <= 0.0) return fail(AIDW_EINVAL, "area must be finite and > 0");
    if (!finite(p->R_min) || !finite(p->R_max) || p->R_max <= p->R_min || p->R_max <= 0.0)
        return fail(AIDW_EINVAL, "need finite R_max > R_min and R_max > 0");
    for (int j = 0; j < 5; ++j)
        if (!finite(p->alpha_levels[j]) || p->alpha_levels[j] < 0.0)
            return fail(AIDW_EINVAL, "alpha level %d must be finite and >= 0", j + 1);
    if (p->n > 0 && (!p->data_xy || !p->data_z || !p->query_xy || !p->out))
        return fail(AIDW_EINVAL, "NULL data, query or output pointer");
    const size_t el = p->precision == AIDW_FP64 ? 8 : 4;
    const void* ptrs[] = {p->data_xy, p->data_z, p->query_xy, p->out};
    for (const void* q : ptrs)
        if ((uintptr_t)q % el) return fail(AIDW_EINVAL, "pointer not aligned to its element size");
    if (((uintptr_t)p->r_obs | (uintptr_t)p->alpha) % 8 || (uintptr_t)p->knn_idx % 4)
        return fail(AIDW_EINVAL, "diagnostic pointer misaligned");
    return AIDW_OK;
}

aidw::AlphaParams alpha_params(const aidw_problem* p) {
    aidw::AlphaParams ap;
    for (int j = 0; j < 5; ++j) ap.levels[j] = p->alpha_levels[j];
    ap.R_min = p->R_min;
    ap.R_max = p->R_max;
    // Eq. 2: expected nearest-neighbour distance of m random points on area A.
    ap.r_exp = 1.0 / (2.0 * std::sqrt((double)p->m / p->area));
    ap.k = p->k;
    return ap;
}

int default_q_per_lane(const aidw_ctx* h, int64_t n) {
    // Keep at least ~4 waves per SIMD in flight before giving lanes more queries.
    const int64_t simds = (int64_t)(h->cu_count > 0 ? h->cu_count : 256) * 4;
    if (n >= simds * 4 * aidw::kWaveSize * 4) return 4;
    if (n >= simds * 4 * aidw::kWaveSize * 2) return 2;
    return 1;
}

aidw_status run_problem(aidw_t h, const aidw_problem* p) {
    aidw_status st = validate(p);
    if (st != AIDW_OK) return st;
    if (p->n == 0) return AIDW_OK;
    const aidw::AlphaParams ap = alpha_params(p);
    hipError_t e;
    const int m = (int)p->m, n = (int)p->n;
    if (p->precision == AIDW_FP32_SCALED) {
        const float* xy = static_cast<const float*>(p->data_xy);
        const float* qxy = static_cast<const float*>(p->query_xy);
        aidw::ProblemF32 q{xy, xy + m, static_cast<const float*>(p->data_z), qxy, qxy + n,
                           static_cast<float*>(p->out), p->r_obs, p->alpha, p->knn_idx, m, n, ap};
        aidw::LaunchF32 cfg{h->q_per_lane ? h->q_per_lane : default_q_per_lane(h, n)};
        e = aidw::launch_aidw_f32(q, cfg, h->stream);
    } else {
        const double* xy = static_cast<const double*>(p->data_xy);
        const double* qxy = static_cast<const double*>(p->query_xy);
        aidw::ProblemF64 q{xy, xy + m, static_cast<const double*>(p->data_z), qxy, qxy + n,
                           static_cast<double*>(p->out), p->r_obs, p->alpha, p->knn_idx, m, n, ap};
        e = aidw::launch_aidw_f64(q, h->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (!(p->flags & AIDW_FLAG_ASYNC)) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    return AIDW_OK;
}

}  // namespace

extern "C" {

aidw_status aidw_create(aidw_t* out, const aidw_options* opt) {
    if (!out) return fail(AIDW_EINVAL, "out is NULL");
    *out = nullptr;
    aidw_options o{};
    if (opt) o = *opt;
    if (o.default_precision != AIDW_FP32_SCALED && o.default_precision != AIDW_FP64)
        return fail(AIDW_EINVAL, "unknown default precision");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (o.device < 0 || o.device >= count)
        return fail(AIDW_EINVAL, "device %d not in [0, %d)", o.device, count);
    e = hipSetDevice(o.device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    aidw_ctx* h = new (std::nothrow) aidw_ctx;
    if (!h) return fail(AIDW_ENOMEM, "host allocation failed");
    h->device = o.device;
    h->default_precision = o.default_precision;
    h->hbm_budget = o.hbm_budget_bytes;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, o.device) == hipSuccess)
        h->cu_count = cus;
    *out = h;
    return AIDW_OK;
}

void aidw_destroy(aidw_t h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

aidw_status aidw_set_stream(aidw_t h, void* stream) {
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    h->stream = static_cast<hipStream_t>(stream);
    return AIDW_OK;
}

aidw_status aidw_interpolate(aidw_t h, const void* data_xy, const void* data_z, int64_t m,
                             const void* query_xy, int64_t n, int k,
                             const double alpha_levels[5], double R_min, double R_max,
                             double area, void* out) {
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (!alpha_levels) return fail(AIDW_EINVAL, "alpha_levels is NULL");
    aidw_problem p;
    memset(&p, 0, sizeof p);
    p.precision = h->default_precision;
    p.data_xy = data_xy;
    p.data_z = data_z;
    p.m = m;
    p.query_xy = query_xy;
    p.n = n;
    p.k = k;
    for (int j = 0; j < 5; ++j) p.alpha_levels[j] = alpha_levels[j];
    p.R_min = R_min;
    p.R_max = R_max;
    p.area = area;
    p.out = out;
    return run_problem(h, &p);
}

aidw_status aidw_interpolate_ex(aidw_t h, const aidw_problem* p) {
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    return run_problem(h, p);
}

aidw_status aidw_set_tuning(aidw_t h, int q_per_lane) {
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (q_per_lane != 0 && q_per_lane != 1 && q_per_lane != 2 && q_per_lane != 4)
        return fail(AIDW_EINVAL, "q_per_lane must be 0, 1, 2 or 4");
    h->q_per_lane = q_per_lane;
    return AIDW_OK;
}

aidw_status aidw_synchronize(aidw_t h) {
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    hipError_t e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? AIDW_OK : hip_fail(e, "hipStreamSynchronize");
}

const char* aidw_last_error(void) { return g_last_error.c_str(); }

const char* aidw_status_string(aidw_status s) {
    switch (s) {
        case AIDW_OK: return "AIDW_OK";
        case AIDW_EINVAL: return "AIDW_EINVAL";
        case AIDW_ENOMEM: return "AIDW_ENOMEM";
        case AIDW_EDEVICE: return "AIDW_EDEVICE";
        case AIDW_EAGAIN: return "AIDW_EAGAIN";
        case AIDW_ENOTFOUND: return "AIDW_ENOTFOUND";
    }
    return "AIDW_UNKNOWN";
}

int aidw_version(void) { return (AIDW_VERSION_MAJOR << 16) | AIDW_VERSION_MINOR; }

}  // extern "C"
