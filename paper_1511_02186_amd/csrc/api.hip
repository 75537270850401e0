// C-ABI entry points of libaidw (declared in include/aidw.h): handles,
// argument validation, per-problem constants and kernel dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "../../include/aidw.h"
#include "common.h"
#include "handle.h"

namespace {
// Messages of the calling thread: its most recent error of any call, and its
// most recent error per handle.
thread_local std::string g_last_error;
thread_local std::unordered_map<const aidw_ctx*, std::string> g_handle_error;
thread_local const aidw_ctx* g_scope = nullptr;
}  // namespace

namespace aidw {
namespace detail {

aidw_status fail(aidw_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    if (g_scope) g_handle_error[g_scope] = buf;
    return s;
}

ErrorScope::ErrorScope(const aidw_ctx* h) : prev_(g_scope) {
    if (h) g_scope = h;
}
ErrorScope::~ErrorScope() { g_scope = prev_; }

void forget_errors(const aidw_ctx* h) { g_handle_error.erase(h); }

aidw_status hip_fail(hipError_t e, const char* what) {
    return fail(AIDW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace detail
}  // namespace aidw

using namespace aidw::detail;

struct aidw_batch {
    aidw_t h = nullptr;
    int count = 0;
    aidw::BatchLaunch launch{};
    void* device_block = nullptr;  // problems, items, max-|z| tasks and slots
    size_t device_bytes = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace aidw {

int k_bucket(int k) {
    static const int buckets[] = {4, 8, 10, 12, 16, 20, 24, 32};
    for (int b : buckets)
        if (k <= b) return b;
    return -1;
}

}  // namespace aidw

namespace aidw {
namespace detail {

static bool finite(double v) { return std::isfinite(v); }

// Host-side validation of everything the kernels assume (include/aidw.h).
aidw_status validate(const aidw_problem* p) {
    if (!p) return fail(AIDW_EINVAL, "problem is NULL");
    if (p->precision != AIDW_FP32_SCALED && p->precision != AIDW_FP64)
        return fail(AIDW_EINVAL, "unknown precision %d", (int)p->precision);
    if (p->m < 1 || p->m > AIDW_MAX_POINTS)
        return fail(AIDW_EINVAL, "m = %lld out of [1, %lld]", (long long)p->m,
                    (long long)AIDW_MAX_POINTS);
    if (p->n < 0 || p->n > AIDW_MAX_POINTS)
        return fail(AIDW_EINVAL, "n = %lld out of [0, %lld]", (long long)p->n,
                    (long long)AIDW_MAX_POINTS);
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

}  // namespace detail
}  // namespace aidw

namespace {

int default_q_per_lane(const aidw_ctx*, int64_t) {
    // One query per lane: the lean register footprint (about 60 VGPRs) keeps
    // 8 waves per SIMD resident, which hides the scalar-load and
    // transcendental latencies better than more queries per lane did on
    // MI355X at every size measured.
    return 1;
}

// Library-owned device allocations are counted against the handle's budget.
}  // namespace

namespace aidw {
namespace detail {

aidw_status device_alloc(aidw_t h, size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) return AIDW_OK;
    {
        // check and reserve in one step: the serving worker allocates too
        std::lock_guard<std::mutex> lk(h->mu);
        if (h->hbm_budget && h->hbm_in_use + bytes > h->hbm_budget)
            return fail(AIDW_ENOMEM, "device budget exceeded: %zu in use + %zu requested > %zu",
                        h->hbm_in_use, bytes, h->hbm_budget);
        h->hbm_in_use += bytes;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        std::lock_guard<std::mutex> lk(h->mu);
        h->hbm_in_use -= bytes;
        return fail(AIDW_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    return AIDW_OK;
}

void device_free(aidw_t h, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    std::lock_guard<std::mutex> lk(h->mu);
    h->hbm_in_use -= bytes;
}

}  // namespace detail
}  // namespace aidw

namespace {

aidw_status ensure_workspace(aidw_t h, size_t bytes) {
    if (bytes <= h->workspace_bytes) return AIDW_OK;
    hipError_t e = hipStreamSynchronize(h->stream);  // the old buffer may still be in use
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    device_free(h, h->workspace, h->workspace_bytes);
    h->workspace = nullptr;
    h->workspace_bytes = 0;
    aidw_status st = device_alloc(h, bytes, &h->workspace);
    if (st == AIDW_OK) h->workspace_bytes = bytes;
    return st;
}

}  // namespace

namespace aidw {
namespace detail {

// Number of data segments for an FP32-scaled problem.  1 (the fused kernel)
// when the 64-query tiles alone give at least two rounds of 8 waves per
// SIMD (plan_f32 lowers that to 1.5 rounds for the speculative single
// pass).  Below that the fused kernel leaves SIMDs short of waves to pair
// instructions from (one round or less: 102 ms fused against 81 ms in 8
// segments at m = 2^20, n = 2^18), so the problem runs as (tile, segment)
// waves, about eight rounds' worth, with segments of at least kMinSegment
// points.  At two rounds the two are even (m = n = 2^20: 306 ms fused,
// 300-306 ms in 2-8 segments), and the fused kernel needs no workspace.
// Eight rounds rather than four: tiles differ in cost (the one- or the
// two-transcendental pass 2), and smaller items even out the last round
// (in spatial tile order, 8 against 16 segments: clustered m = n = 2^18
// 21.4 / 20.9 ms, m = 2^20, n = 2^18 76.8 / 74.2 ms, the same clustered
// 83.8 / 80.9 ms; 32 segments gain under 1 % more).
constexpr int kMinSegment = 2048;

aidw::SplitPlan split_plan_for(const aidw_ctx* h, const aidw_tuning& t, int64_t m, int64_t n) {
    aidw::SplitPlan sp{1, (int)m, (int)((n + aidw::kWaveSize - 1) / aidw::kWaveSize)};
    int want = t.split_segments;
    if (want == 0) {
        const int64_t round = (int64_t)(h->cu_count > 0 ? h->cu_count : 256) * 4 * 8;
        if (sp.tiles >= 2 * round) return sp;
        want = (int)std::min<int64_t>((8 * round + sp.tiles - 1) / sp.tiles, 1 << 20);
    }
    int64_t seg = (m + want - 1) / want;
    if (t.split_segments == 0) seg = std::max<int64_t>(seg, kMinSegment);
    seg = (seg + 31) / 32 * 32;  // whole scalar-load batches
    if (seg >= m) return sp;
    sp.seg_len = (int)seg;
    sp.segments = (int)((m + seg - 1) / seg);
    return sp;
}

// Pass 2 on its own (after the grid search) runs in data segments of about
// kGridPass2Segment points even when the queries fill the device: waves are
// numbered segment-major, so the resident waves read one segment at a time,
// and 128 K points of x, y, z (1.5 MB) stay in the XCD's 4 MB L2 instead of
// streaming the whole set through it (239 -> 216 ms at m = n = 2^20 with 8
// segments).  Up to 8 segments; an explicit tuning wins.
constexpr int64_t kGridPass2Segment = 131072;

aidw::SplitPlan grid_pass2_plan(const aidw_ctx* h, const aidw_tuning& t, int64_t m, int64_t n) {
    aidw::SplitPlan sp = split_plan_for(h, t, m, n);
    if (h->deterministic) sp = aidw::SplitPlan{1, (int)m, sp.tiles};  // by m alone
    else if (t.split_segments != 0 || sp.segments > 1) return sp;
    const int64_t want = std::min<int64_t>(8, m / kGridPass2Segment);
    if (want < 2) return sp;
    int64_t seg = (m + want - 1) / want;
    seg = (seg + 31) / 32 * 32;  // whole scalar-load batches
    sp.seg_len = (int)seg;
    sp.segments = (int)((m + seg - 1) / seg);
    return sp;
}

size_t split_workspace_bytes(const aidw::SplitPlan& sp, int k, int64_t n, aidw::SplitWorkspace* ws,
                             char* base, bool regroup) {
    const int64_t tiles = (n + aidw::kWaveSize - 1) / aidw::kWaveSize;
    const size_t part = (size_t)sp.segments * k * n * sizeof(float);
    const size_t qpar = 4 * (size_t)n * sizeof(float);
    const size_t psum = (size_t)sp.segments * 2 * n * sizeof(double);
    const size_t seg_ok = (size_t)sp.segments * tiles * sizeof(int);
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    const size_t o_qpar = up(part);
    const size_t o_psum = up(o_qpar + qpar);
    const size_t o_seg = up(o_psum + psum);
    const size_t o_tile = up(o_seg + seg_ok);
    const size_t end_tile = o_tile + tiles * sizeof(int);
    // pass-2 regrouping: keys, sort histogram, the regrouped order
    const size_t blocks = (size_t)((n + aidw::kOrderBlock - 1) / aidw::kOrderBlock);
    const size_t o_key = up(end_tile);
    const size_t o_hist = up(o_key + sizeof(unsigned) * (size_t)n);
    const size_t o_ord = up(o_hist + sizeof(int) * 256 * blocks);
    if (ws) {
        ws->part = reinterpret_cast<float*>(base);
        ws->qpar = reinterpret_cast<float*>(base + o_qpar);
        ws->psum = reinterpret_cast<double*>(base + o_psum);
        ws->seg_ok = reinterpret_cast<int*>(base + o_seg);
        ws->tile_ok = reinterpret_cast<int*>(base + o_tile);
        ws->p2key = regroup ? reinterpret_cast<unsigned*>(base + o_key) : nullptr;
        ws->p2hist = regroup ? reinterpret_cast<int*>(base + o_hist) : nullptr;
        ws->p2order = regroup ? reinterpret_cast<int*>(base + o_ord) : nullptr;
    }
    return regroup ? o_ord + sizeof(int) * (size_t)n : end_tile;
}

// Problems of fewer data points than this keep the two passes: the single
// pass gains little there.
constexpr int64_t kSpecMinPoints = 1024;

aidw::ProblemF32 problem_f32(const aidw_problem* p) {
    const int m = (int)p->m, n = (int)p->n;
    const float* xy = static_cast<const float*>(p->data_xy);
    const float* qxy = static_cast<const float*>(p->query_xy);
    aidw::ProblemF32 q{xy, xy + m, static_cast<const float*>(p->data_z), qxy, qxy + n,
                       static_cast<float*>(p->out), p->r_obs, p->alpha, p->knn_idx, m, n,
                       alpha_params(p)};
    // The speculative single pass assumes alpha = alpha_5, which Eq. 6 gives
    // for mu_R >= 0.9; it is worth it only when that power is whole (one
    // transcendental per pair).  Eq. 5 reaches mu = 0.9 at
    // R_min + acos(-0.8) R_max / pi (or at R_max, if that comes first).
    const double a5 = p->alpha_levels[4];
    if (a5 >= 1.0 && a5 <= 8.0 && a5 == std::floor(a5) && p->m >= kSpecMinPoints) {
        q.spec_power = (int)a5;
        const double R90 = std::min(p->R_max, p->R_min + std::acos(-0.8) * p->R_max / M_PI);
        q.spec_dist_sum = (float)(p->k * R90 * q.ap.r_exp * (1.0 - 1e-4));
        // with all five levels equal alpha never leaves alpha_5 (standard IDW):
        // never stop speculating early
        bool constant = true;
        for (int j = 0; j < 4; ++j) constant &= p->alpha_levels[j] == a5;
        if (constant) q.spec_dist_sum = 0.0f;
    }
    return q;
}

// Fewer data points than this: the scans are short, and the order's seven
// small launches would cost more than tile coherence saves.
constexpr int64_t kOrderMinPoints = 1024;

int order_bits_for(int mode, int64_t m, int64_t n) {
    if (mode == 1 || (mode == 0 && m < kOrderMinPoints)) return 0;
    return aidw::order_bits(n);
}

int order_passes(int bits) { return (2 * bits + 7) / 8; }
int order_blocks(int64_t n) { return (int)((n + aidw::kOrderBlock - 1) / aidw::kOrderBlock); }

aidw::ProblemF64 problem_f64(const aidw_problem* p) {
    const int m = (int)p->m, n = (int)p->n;
    const double* xy = static_cast<const double*>(p->data_xy);
    const double* qxy = static_cast<const double*>(p->query_xy);
    return aidw::ProblemF64{xy, xy + m, static_cast<const double*>(p->data_z), qxy, qxy + n,
                            static_cast<double*>(p->out), p->r_obs, p->alpha, p->knn_idx, m, n,
                            alpha_params(p)};
}

}  // namespace detail
}  // namespace aidw

namespace {

// Bytes at the start of the handle workspace that hold max |z| of the call.
constexpr size_t kZmaxSlot = 256;

// Pass 1 through the uniform grid, then pass 2 over all points.
hipError_t run_grid(aidw_t h, const aidw_problem* p, aidw_status* st_out) {
    const int m = (int)p->m, n = (int)p->n;
    aidw::ProblemF32 q = problem_f32(p);
    aidw::GridWorkspace gw{};
    gw.cells = aidw::grid_cells(m);
    gw.nparts = (int)std::min<int64_t>(1024, ((int64_t)m + 255) / 256);
    gw.temp_bytes = aidw::grid_temp_bytes(gw.cells);
    const size_t cells = (size_t)gw.cells;
    // pass 2 over data segments: for L2 locality, or when there are too few
    // queries to fill the chip
    const aidw::SplitPlan sp = grid_pass2_plan(h, h->tuning, m, n);
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    size_t off[10], bytes = 0;
    const size_t sizes[10] = {kZmaxSlot, sizeof(aidw::GridGeom), sizeof(float4) * (size_t)gw.nparts,
                             sizeof(int) * (cells + 1), sizeof(int) * (cells + 1),
                             sizeof(int) * cells, sizeof(float2) * (size_t)m, gw.temp_bytes,
                             4 * sizeof(float) * (size_t)n,
                             2 * sizeof(double) * (size_t)n * (size_t)sp.segments};
    for (int i = 0; i < 10; ++i) {
        off[i] = bytes;
        bytes += up(sizes[i]);
    }
    *st_out = ensure_workspace(h, bytes);
    if (*st_out != AIDW_OK) return hipSuccess;
    char* w = static_cast<char*>(h->workspace);
    float* zmax = reinterpret_cast<float*>(w + off[0]);
    gw.geo = reinterpret_cast<aidw::GridGeom*>(w + off[1]);
    gw.part = reinterpret_cast<float4*>(w + off[2]);
    gw.counts = reinterpret_cast<int*>(w + off[3]);
    gw.start = reinterpret_cast<int*>(w + off[4]);
    gw.cursor = reinterpret_cast<int*>(w + off[5]);
    gw.sorted = reinterpret_cast<float2*>(w + off[6]);
    gw.temp = w + off[7];
    gw.qpar = reinterpret_cast<float*>(w + off[8]);
    gw.psum = reinterpret_cast<double*>(w + off[9]);
    q.zmax = zmax;
    hipError_t e = aidw::launch_abs_max(q.dz, m, zmax, h->stream);
    if (e == hipSuccess) e = aidw::launch_grid_knn_all(q, gw, h->stream);
    if (e == hipSuccess) e = aidw::launch_aidw_f32_pass2(q, sp, gw.qpar, gw.psum, h->stream);
    return e;
}


// Launch shape and data segments of an FP32-scaled full-scan problem.
struct F32Plan {
    aidw::LaunchF32 cfg;
    aidw::SplitPlan sp;
    bool spec;  // the speculative single pass, with pass 2 deferred for missed queries
    int order_bits;  // Morton bits per axis of the spatial tile order (0: caller's order)
    bool split_spec = false;  // speculative sums per data segment in the split kernels
    bool regroup = false;     // split pass 2 in waves regrouped by their loop
};

// Order workspace of one problem (plan pl); with L given, laid out at base.
size_t order_bytes(const F32Plan& pl, int64_t n, aidw::OrderLaunch* L, char* base) {
    if (!pl.order_bits) return 0;
    return aidw::order_workspace_bytes(n, order_blocks(n), 1, order_passes(pl.order_bits), L,
                                       base);
}

// Speculative sums (the single pass, or per segment in the split kernels)
// unless the handle is deterministic or its tuning turns them off.
bool speculation_allowed(const aidw_ctx* h) { return !h->deterministic && h->tuning.speculate != 1; }

// Waves in one round of the device (8 per SIMD, 4 SIMDs per CU): what the
// deferred pass 2 of the speculative launch aims to fill.
int round_waves(const aidw_ctx* h) { return (h->cu_count > 0 ? h->cu_count : 256) * 4 * 8; }

F32Plan plan_f32(const aidw_ctx* h, const aidw_problem* p) {
    aidw_tuning t = h->tuning;
    aidw_tuning tuned;
    if (h->deterministic)
        t = aidw_tuning{1, 0, 1};  // the unsplit one-query-per-lane kernel
    else if (!t.q_per_lane && !t.max_waves_per_simd && !t.split_segments &&
             tuned_shape(h, p->m, p->n, p->k, &tuned)) {
        if (t.speculate == 0) t.speculate = tuned.speculate;  // else the handle's choice
        tuned.speculate = t.speculate;
        t = tuned;
    }
    F32Plan pl{aidw::LaunchF32{t.q_per_lane ? t.q_per_lane : default_q_per_lane(h, p->n),
                               t.max_waves_per_simd},
               aidw::SplitPlan{1, (int)p->m, 0}, false,
               order_bits_for(h->deterministic ? 0 : h->tuning.query_order, p->m, p->n)};
    if (!p->knn_idx) pl.sp = split_plan_for(h, t, p->m, p->n);
    // The speculative single pass replaces the unsplit one-query-per-lane
    // kernel when alpha_5 is a whole power (a split problem speculates per
    // segment, inside the split kernels); it is off in deterministic mode,
    // which promises the kernel batched launches use.
    const bool spec_ok = !h->deterministic && !p->knn_idx && pl.cfg.q_per_lane == 1 &&
                         pl.cfg.max_waves_per_simd == 0 && speculation_allowed(h) &&
                         problem_f32(p).spec_power != 0;
    // The single pass holds the unsplit launch down to 1.5 rounds of tiles
    // (two for the two-pass kernel).  Measured, unsplit against the
    // automatic split, uniform + clustered data of m = n: 1.95 rounds 545
    // against 577 ms, 1.5 rounds 338 against 348, 1.2 rounds 228 against
    // 224, 0.95 rounds 147 against 141.
    if (spec_ok && t.split_segments == 0 && pl.sp.segments > 1 &&
        2 * (int64_t)pl.sp.tiles >= 3 * (int64_t)round_waves(h))
        pl.sp = aidw::SplitPlan{1, (int)p->m, pl.sp.tiles};
    pl.spec = spec_ok && pl.sp.segments == 1;
    // Speculative sums inside the split kernels only when the tuning (the
    // handle's, else the autotuner's shape for the size class) asks for them
    // (speculate = 2).  There a tile that keeps them saves little over the
    // one-transcendental pass 2 it replaces (the distances, about 8 % of that
    // pass measured on uniform data), while a tile that forms them and then
    // misses alpha_5 pays a second pass 1; each segment decides from 1/32 of
    // its own points, so on clustered data many tiles do (m = n = 2^18
    // clustered: 25.9 ms with them, 21.7 ms without; uniform: 18.5 against
    // 19.8 ms).
    pl.split_spec = speculation_allowed(h) && t.speculate == 2;
    // Split pass 2 runs after alpha is known everywhere: its waves can take
    // the positions regrouped by the loop they need (the caller's order, 1,
    // keeps the pass-1 tiles).
    pl.regroup = pl.sp.segments > 1 && !pl.split_spec &&
                 (h->deterministic ? 0 : h->tuning.query_order) != 1;
    return pl;
}

// Workspace of an FP32-scaled problem: max |z| in the first slot, the tile
// order, then the buffers of the speculative or the split launch.
size_t f32_workspace_bytes(const aidw_ctx* h, const F32Plan& pl, const aidw_problem* p) {
    const size_t head = kZmaxSlot + order_bytes(pl, p->n, nullptr, nullptr);
    if (pl.spec) return head + aidw::spec_workspace_bytes(p->n, round_waves(h), nullptr, nullptr);
    return head +
           (pl.sp.segments > 1 ? split_workspace_bytes(pl.sp, p->k, p->n, nullptr, nullptr,
                                                       pl.regroup)
                               : 0);
}

// Queue the tile-order kernels of plan pl (order workspace at base) and
// point q at the order.
hipError_t launch_order(aidw_t h, const F32Plan& pl, aidw::ProblemF32& q, char* base) {
    if (!pl.order_bits) return hipSuccess;
    aidw::OrderLaunch L{};
    order_bytes(pl, q.n, &L, base);
    L.one = aidw::OrderSeg{q.qx, q.qy, q.n, 0, 0, order_blocks(q.n), pl.order_bits};
    L.segments = 1;
    L.blocks = order_blocks(q.n);
    L.passes = order_passes(pl.order_bits);
    q.order = L.order;
    return aidw::launch_query_order(L, h->stream);
}

// Queue the max-|z| reduction and the FP32-scaled kernels of plan pl, with
// the workspace at w (f32_workspace_bytes(h, pl, p) bytes, 256-byte aligned).
hipError_t launch_f32(aidw_t h, const aidw_problem* p, const F32Plan& pl, char* w) {
    aidw::ProblemF32 q = problem_f32(p);
    hipError_t e = launch_order(h, pl, q, w + kZmaxSlot);
    if (e != hipSuccess) return e;
    char* rest = w + kZmaxSlot + order_bytes(pl, p->n, nullptr, nullptr);
    float* zmax = reinterpret_cast<float*>(w);
    q.zmax = zmax;
    if (pl.spec) {
        aidw::DeferWorkspace dw{};
        aidw::spec_workspace_bytes(p->n, round_waves(h), &dw, rest);
        e = aidw::launch_abs_max(q.dz, q.m, zmax, h->stream, dw.count);
        if (e == hipSuccess) e = aidw::launch_aidw_f32_spec(q, dw, h->stream);
        return e;
    }
    if (!pl.split_spec) q.spec_power = 0;  // the split kernels speculate when it is set
    aidw::SplitWorkspace ws{};
    if (pl.sp.segments > 1) split_workspace_bytes(pl.sp, p->k, p->n, &ws, rest, pl.regroup);
    e = aidw::launch_abs_max(q.dz, q.m, zmax, h->stream);
    if (e == hipSuccess) e = aidw::launch_aidw_f32(q, pl.cfg, &pl.sp, &ws, h->stream);
    return e;
}

// Report a failed launch, or wait for the work unless the call is asynchronous.
aidw_status finish_launch(aidw_t h, const aidw_problem* p, hipError_t e) {
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (!(p->flags & AIDW_FLAG_ASYNC)) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    return AIDW_OK;
}

aidw_status run_problem(aidw_t h, const aidw_problem* p) {
    aidw_status st = validate(p);
    if (st != AIDW_OK) return st;
    if (p->n == 0) return AIDW_OK;
    hipError_t e;
    if (p->flags & AIDW_FLAG_GRID_KNN) {
        if (p->precision != AIDW_FP32_SCALED)
            return fail(AIDW_EINVAL, "AIDW_FLAG_GRID_KNN needs the FP32-scaled precision");
        if (p->knn_idx) return fail(AIDW_EINVAL, "AIDW_FLAG_GRID_KNN does not produce knn_idx");
        aidw_status gst = AIDW_OK;
        e = run_grid(h, p, &gst);
        if (gst != AIDW_OK) return gst;
    } else if (p->precision == AIDW_FP32_SCALED) {
        F32Plan pl = plan_f32(h, p);
        st = ensure_workspace(h, f32_workspace_bytes(h, pl, p));
        if (st == AIDW_ENOMEM && pl.order_bits) {
            // the tile order only sets the speed: without its ~20 n bytes
            pl.order_bits = 0;
            st = ensure_workspace(h, f32_workspace_bytes(h, pl, p));
        }
        if (st != AIDW_OK) return st;
        e = launch_f32(h, p, pl, static_cast<char*>(h->workspace));
    } else {
        e = aidw::launch_aidw_f64(problem_f64(p), h->stream);
    }
    return finish_launch(h, p, e);
}

}  // namespace

// ---- Device scratch of the allocation-free entry point ----------------------
// aidw_interpolate_noalloc keeps max |z| and the split-m buffers here instead
// of in the handle's workspace.  Every device the library runs on holds its
// own copy until the process ends.  On the host the array's name is not a
// device address: host code uses only the per-device address that
// hipGetSymbolAddress returns (looked up in aidw_create).
static __device__ __align__(256) unsigned char scratch[AIDW_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // this device's copy of `scratch`, once looked up

// The address of `scratch` on `device`, which must be the current device.
aidw_status noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return fail(AIDW_EINVAL, "device %d beyond the %d the library tracks", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(AIDW_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return AIDW_OK;
}

// The most data segments (at most sp.segments) whose split workspace, after
// the max-|z| slot, fits in `cap` bytes; one segment (the fused kernel,
// which needs only the slot) when not even two fit.
aidw::SplitPlan fit_split(aidw::SplitPlan sp, int k, int64_t n, int64_t m, size_t cap) {
    auto need = [&](const aidw::SplitPlan& s) {
        return kZmaxSlot + split_workspace_bytes(s, k, n, nullptr, nullptr);
    };
    if (sp.segments <= 1 || need(sp) <= cap) return sp;
    const size_t fixed = kZmaxSlot + 4 * sizeof(float) * (size_t)n + 512;
    const size_t per_segment = (size_t)k * n * sizeof(float) + 2 * sizeof(double) * (size_t)n;
    int64_t want = cap > fixed ? (int64_t)((cap - fixed) / per_segment) : 0;
    want = std::min<int64_t>(want, sp.segments - 1);
    for (; want >= 2; --want) {
        int64_t seg = (m + want - 1) / want;
        seg = (seg + 31) / 32 * 32;  // whole scalar-load batches
        aidw::SplitPlan t{(int)((m + seg - 1) / seg), (int)seg, sp.tiles};
        if (t.segments > 1 && need(t) <= cap) return t;
    }
    return aidw::SplitPlan{1, (int)m, sp.tiles};
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
    h->deterministic = o.deterministic != 0;
    h->hbm_budget = o.hbm_budget_bytes;
    const aidw_status sst = noalloc_scratch(o.device, &h->scratch);
    if (sst != AIDW_OK) {
        delete h;
        return sst;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, o.device) == hipSuccess)
        h->cu_count = cus;
    if (o.tune_path) {
        const aidw_status st = aidw_tune_load(h, o.tune_path);
        if (st != AIDW_OK && st != AIDW_ENOTFOUND) {
            delete h;
            return st;  // the message of aidw_tune_load stays
        }
    }
    *out = h;
    return AIDW_OK;
}

void aidw_destroy(aidw_t h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->server) aidw_server_destroy(h->server);  // finishes its jobs
    h->server = nullptr;
    (void)hipStreamSynchronize(h->stream);
    device_free(h, h->workspace, h->workspace_bytes);
    forget_errors(h);
    delete h;
}

aidw_status aidw_set_stream(aidw_t h, void* stream) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (s != h->stream) {
        // library-owned scratch is reused by the next call: let the old stream drain
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        h->stream = s;
    }
    return AIDW_OK;
}

aidw_status aidw_interpolate(aidw_t h, const void* data_xy, const void* data_z, int64_t m,
                             const void* query_xy, int64_t n, int k,
                             const double alpha_levels[5], double R_min, double R_max,
                             double area, void* out) {
    ErrorScope es(h);
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
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    return run_problem(h, p);
}

aidw_status aidw_describe_launch(aidw_t h, const aidw_problem* p, char* buf, size_t cap) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (!buf || cap == 0) return fail(AIDW_EINVAL, "buffer is NULL or empty");
    aidw_status st = validate(p);
    if (st != AIDW_OK) return st;
    std::string d;
    const int K = aidw::k_bucket(p->k);
    const std::string k = "<" + std::to_string(K);
    if (p->n == 0) {
        d = "";
    } else if (p->flags & AIDW_FLAG_GRID_KNN) {
        d = "aidw_abs_max + bbox_partial + grid_setup + grid_clear + grid_count + "
            "(device scan) + grid_scatter + grid_knn" + k + "> + aidw_f32_wsum_part + "
            "aidw_f32_wsum_reduce";
    } else if (p->precision == AIDW_FP64) {
        d = "aidw_f64_plain" + k + (p->knn_idx ? ", true>" : ", false>");
    } else {
        const F32Plan pl = plan_f32(h, p);
        if (pl.order_bits)
            d = "aidw_order_box_part + aidw_order_bbox + (aidw_order_hist + aidw_order_scan + "
                "aidw_order_scatter) x " +
                std::to_string(order_passes(pl.order_bits)) + " + ";
        if (pl.spec)
            d += "aidw_abs_max + aidw_f32_fused_spec" + k + "> + aidw_f32_defer_list + "
                 "aidw_f32_defer_part + aidw_f32_defer_reduce";
        else if (pl.sp.segments > 1)
            d += "aidw_abs_max + aidw_f32_knn_part" + k + "> + aidw_f32_knn_merge" + k + "> + " +
                 (pl.regroup ? "aidw_f32_pass2_keys + aidw_order_hist + aidw_order_scan + "
                               "aidw_order_scatter (pass 2 regrouped by loop) + "
                             : "") +
                 "aidw_f32_wsum_part + aidw_f32_wsum_reduce (" + std::to_string(pl.sp.segments) +
                 " data segments)";
        else
            d += "aidw_abs_max + aidw_f32_fused" + k + ", " + std::to_string(pl.cfg.q_per_lane) +
                 (p->knn_idx ? ", true>" : ", false>");
    }
    const size_t len = std::min(d.size(), cap - 1);
    memcpy(buf, d.data(), len);
    buf[len] = '\0';
    return AIDW_OK;
}

aidw_status aidw_query_order(aidw_t h, const void* query_xy, int64_t n, int32_t* order) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (n < 0 || n > AIDW_MAX_POINTS) return fail(AIDW_EINVAL, "n = %lld out of range", (long long)n);
    if (n == 0) return AIDW_OK;
    if (!query_xy || !order) return fail(AIDW_EINVAL, "query_xy or order is NULL");
    const int bits = std::max(1, aidw::order_bits(n));
    const int passes = order_passes(bits), blocks = order_blocks(n);
    aidw_status st = ensure_workspace(h, aidw::order_workspace_bytes(n, blocks, 1, passes, nullptr,
                                                                     nullptr));
    if (st != AIDW_OK) return st;
    aidw::OrderLaunch L{};
    aidw::order_workspace_bytes(n, blocks, 1, passes, &L, static_cast<char*>(h->workspace));
    const float* qx = static_cast<const float*>(query_xy);
    L.one = aidw::OrderSeg{qx, qx + n, (int)n, 0, 0, blocks, bits};
    L.segments = 1;
    L.blocks = blocks;
    L.passes = passes;
    L.order = order;
    hipError_t e = aidw::launch_query_order(L, h->stream);
    if (e != hipSuccess) return hip_fail(e, "order launch");
    e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? AIDW_OK : hip_fail(e, "hipStreamSynchronize");
}

aidw_status aidw_interpolate_noalloc(aidw_t h, const aidw_problem* p) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_status st = validate(p);
    if (st != AIDW_OK) return st;
    if (p->flags & AIDW_FLAG_GRID_KNN)
        return fail(AIDW_EINVAL, "AIDW_FLAG_GRID_KNN needs the handle's workspace "
                                 "(aidw_interpolate_ex)");
    if (p->n == 0) return AIDW_OK;
    hipError_t e;
    if (p->precision == AIDW_FP64) {
        e = aidw::launch_aidw_f64(problem_f64(p), h->stream);  // uses no scratch
    } else {
        F32Plan pl = plan_f32(h, p);
        const size_t cap = AIDW_NOALLOC_SCRATCH_BYTES;
        // the tile order stays unless it alone would leave no room for the
        // rest (about 20 n bytes: beyond 3 million queries)
        if (pl.order_bits && kZmaxSlot + order_bytes(pl, p->n, nullptr, nullptr) + (1 << 20) > cap)
            pl.order_bits = 0;
        const size_t cap_rest = cap - order_bytes(pl, p->n, nullptr, nullptr);
        if (pl.spec && f32_workspace_bytes(h, pl, p) > cap) pl.spec = false;
        if (pl.regroup && f32_workspace_bytes(h, pl, p) > cap) pl.regroup = false;
        if (f32_workspace_bytes(h, pl, p) > cap) {
            if (h->tuning.split_segments > 1)
                return fail(AIDW_ENOMEM,
                            "split into %d segments the problem needs %zu bytes of scratch, "
                            "more than the %zu of the allocation-free entry point",
                            pl.sp.segments, f32_workspace_bytes(h, pl, p), cap);
            pl.sp = fit_split(pl.sp, p->k, p->n, p->m, cap_rest);
        }
        if (f32_workspace_bytes(h, pl, p) > cap)  // unreachable: one segment fits beside the order
            return fail(AIDW_ENOMEM, "scratch of %zu bytes exceeded", cap);
        e = launch_f32(h, p, pl, static_cast<char*>(h->scratch));
    }
    return finish_launch(h, p, e);
}

aidw_status aidw_idw(aidw_t h, const aidw_problem* p, double power) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (!p) return fail(AIDW_EINVAL, "problem is NULL");
    if (!std::isfinite(power) || power < 0.0)
        return fail(AIDW_EINVAL, "power must be finite and >= 0");
    aidw_problem q = *p;
    q.k = 1;
    for (int j = 0; j < 5; ++j) q.alpha_levels[j] = power;
    q.R_min = 0.0;
    q.R_max = 1.0;
    q.area = 1.0;
    return run_problem(h, &q);
}

aidw_status aidw_interpolate_variant(aidw_t h, const aidw_problem* p, aidw_access access,
                                     aidw_layout layout) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_status st = validate(p);
    if (st != AIDW_OK) return st;
    if (p->flags & AIDW_FLAG_GRID_KNN) return fail(AIDW_EINVAL, "access variants scan all points");
    if (p->precision == AIDW_FP32_SCALED && p->knn_idx)
        return fail(AIDW_EINVAL, "FP32-scaled access variants do not produce knn_idx");
    if ((int)access < 0 || (int)access > 2) return fail(AIDW_EINVAL, "unknown access %d", (int)access);
    if ((int)layout < 0 || (int)layout > 1) return fail(AIDW_EINVAL, "unknown layout %d", (int)layout);
    if (p->n == 0) return AIDW_OK;
    const bool f64 = p->precision == AIDW_FP64;
    void* aos = nullptr;
    if (layout == AIDW_LAYOUT_AOAS) {
        st = ensure_workspace(h, (f64 ? sizeof(double4) : sizeof(float4)) * (size_t)p->m);
        if (st != AIDW_OK) return st;
        aos = h->workspace;
    }
    hipError_t e =
        f64 ? aidw::launch_aidw_f64_variant(problem_f64(p), (int)access, (int)layout,
                                            static_cast<double4*>(aos), h->stream)
            : aidw::launch_aidw_f32_variant(problem_f32(p), (int)access, (int)layout,
                                            static_cast<float4*>(aos), h->stream);
    return finish_launch(h, p, e);
}

aidw_status aidw_set_tuning(aidw_t h, const aidw_tuning* t) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    if (!t) {
        h->tuning = aidw_tuning{0, 0, 0};
        return AIDW_OK;
    }
    if (t->split_segments < 0) return fail(AIDW_EINVAL, "split_segments must be >= 0");
    if (t->q_per_lane != 0 && t->q_per_lane != 1 && t->q_per_lane != 2 && t->q_per_lane != 4)
        return fail(AIDW_EINVAL, "q_per_lane must be 0, 1, 2 or 4");
    if (t->max_waves_per_simd < 0 || t->max_waves_per_simd > 8)
        return fail(AIDW_EINVAL, "max_waves_per_simd must be in [0, 8]");
    if (t->speculate < 0 || t->speculate > 2) return fail(AIDW_EINVAL, "speculate must be 0, 1 or 2");
    if (t->query_order < 0 || t->query_order > 2)
        return fail(AIDW_EINVAL, "query_order must be 0, 1 or 2");
    h->tuning = *t;
    return AIDW_OK;
}

aidw_status aidw_synchronize(aidw_t h) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    hipError_t e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? AIDW_OK : hip_fail(e, "hipStreamSynchronize");
}

const char* aidw_last_error(aidw_t h) {
    if (!h) return g_last_error.c_str();
    auto it = g_handle_error.find(h);
    return it == g_handle_error.end() ? "" : it->second.c_str();
}

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

// ---- batched problems ------------------------------------------------------------

namespace {

aidw_status batch_build(aidw_t h, const aidw_problem* problems, int count, aidw_batch* b) {
    if (count < 0) return fail(AIDW_EINVAL, "count = %d < 0", count);
    if (count > 0 && !problems) return fail(AIDW_EINVAL, "problems is NULL");
    std::vector<aidw::ProblemF32> probs((size_t)count);
    std::vector<aidw::BatchItem> items;
    int kmax = 1;
    for (int i = 0; i < count; ++i) {
        const aidw_problem* p = &problems[i];
        aidw_status st = validate(p);
        if (st != AIDW_OK)
            return fail(st, "problem %d: %s", i, std::string(aidw_last_error(nullptr)).c_str());
        if (p->precision != AIDW_FP32_SCALED)
            return fail(AIDW_EINVAL, "problem %d: batched problems must be AIDW_FP32_SCALED", i);
        if (p->knn_idx)
            return fail(AIDW_EINVAL, "problem %d: knn_idx is not produced by batched launches", i);
        probs[i] = problem_f32(p);
        kmax = std::max(kmax, p->k);
        for (int64_t base = 0; base < p->n; base += aidw::kWaveSize)
            items.push_back(aidw::BatchItem{i, (int)base});
    }
    if (items.size() > (size_t)INT32_MAX) return fail(AIDW_EINVAL, "too many query tiles");
    // Longest first: an item's cost is proportional to its problem's m.
    std::stable_sort(items.begin(), items.end(),
                     [&](const aidw::BatchItem& x, const aidw::BatchItem& y) {
                         return probs[x.problem].m > probs[y.problem].m;
                     });
    // Tile order of every problem with more than one tile (the automatic
    // choice of a single launch), all sorted by one set of launches, each
    // problem within its own range of positions.
    std::vector<aidw::OrderSeg> segs;
    std::vector<int> seg_problem, block_seg;
    int64_t total = 0;
    int max_bits = 0;
    for (int i = 0; i < count; ++i) {
        const int bits = order_bits_for(0, problems[i].m, problems[i].n);
        if (!bits) continue;
        const int nb = order_blocks(problems[i].n);
        segs.push_back(aidw::OrderSeg{probs[i].qx, probs[i].qy, probs[i].n, (int)total,
                                      (int)block_seg.size(), nb, bits});
        seg_problem.push_back(i);
        block_seg.insert(block_seg.end(), (size_t)nb, (int)segs.size() - 1);
        total += problems[i].n;
        max_bits = std::max(max_bits, bits);
        if (total > (int64_t)INT32_MAX - aidw::kOrderBlock) {  // positions are 32-bit
            segs.clear();
            block_seg.clear();
            break;
        }
    }
    if (segs.empty()) total = 0;
    const int passes = segs.empty() ? 0 : order_passes(max_bits);
    // device block: problems | items | max-|z| tasks | max-|z| slots | order
    // segments | sort block -> segment | order workspace
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    const size_t sz_p = up(sizeof(aidw::ProblemF32) * probs.size());
    const size_t sz_i = up(sizeof(aidw::BatchItem) * items.size());
    const size_t sz_t = up(sizeof(aidw::AbsMaxTask) * probs.size());
    const size_t o_t = sz_p + sz_i, o_z = o_t + sz_t;
    const size_t o_s = o_z + up(sizeof(float) * probs.size());
    const size_t o_b = o_s + up(sizeof(aidw::OrderSeg) * segs.size());
    const size_t o_w = o_b + up(sizeof(int) * block_seg.size());
    const size_t bytes =
        o_w + (segs.empty() ? 0
                            : aidw::order_workspace_bytes(total, (int)block_seg.size(),
                                                          (int)segs.size(), passes, nullptr,
                                                          nullptr));
    aidw_status st = device_alloc(h, bytes, &b->device_block);
    if (st != AIDW_OK) return st;
    b->device_bytes = bytes;
    char* base = static_cast<char*>(b->device_block);
    aidw::OrderLaunch& L = b->launch.order;
    L = aidw::OrderLaunch{};
    if (!segs.empty()) {
        aidw::order_workspace_bytes(total, (int)block_seg.size(), (int)segs.size(), passes, &L,
                                    base + o_w);
        L.table = reinterpret_cast<const aidw::OrderSeg*>(base + o_s);
        L.block_seg = reinterpret_cast<const int*>(base + o_b);
        L.segments = (int)segs.size();
        L.blocks = (int)block_seg.size();
        L.passes = passes;
        for (size_t j = 0; j < segs.size(); ++j)
            probs[seg_problem[j]].order = L.order + segs[j].base;
    }
    float* zslots = reinterpret_cast<float*>(base + o_z);
    std::vector<aidw::AbsMaxTask> tasks(probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        probs[i].zmax = zslots + i;
        tasks[i] = aidw::AbsMaxTask{probs[i].dz, zslots + i, probs[i].m};
    }
    hipError_t e = hipMemcpy(base, probs.data(), sizeof(aidw::ProblemF32) * probs.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(base + sz_p, items.data(), sizeof(aidw::BatchItem) * items.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !tasks.empty())
        e = hipMemcpy(base + o_t, tasks.data(), sizeof(aidw::AbsMaxTask) * tasks.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !segs.empty())
        e = hipMemcpy(base + o_s, segs.data(), sizeof(aidw::OrderSeg) * segs.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !block_seg.empty())
        e = hipMemcpy(base + o_b, block_seg.data(), sizeof(int) * block_seg.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    b->h = h;
    b->count = count;
    b->launch.problems = reinterpret_cast<const aidw::ProblemF32*>(base);
    b->launch.items = reinterpret_cast<const aidw::BatchItem*>(base + sz_p);
    b->launch.tasks = reinterpret_cast<const aidw::AbsMaxTask*>(base + o_t);
    b->launch.n_tasks = (int)tasks.size();
    b->launch.n_items = (int)items.size();
    b->launch.K = aidw::k_bucket(kmax);
    return AIDW_OK;
}

void batch_release(aidw_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->h) device_free(b->h, b->device_block, b->device_bytes);
    b->exec = nullptr;
    b->graph = nullptr;
    b->capture_stream = nullptr;
    b->device_block = nullptr;
}

aidw_status batch_capture(aidw_batch* b) {
    hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = aidw::launch_aidw_f32_batch(b->launch, b->capture_stream);
    e = hipStreamEndCapture(b->capture_stream, &b->graph);
    if (le != hipSuccess) return hip_fail(le, "batched launch during capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return AIDW_OK;
}

}  // namespace

extern "C" {

aidw_status aidw_batch_create(aidw_t h, const aidw_problem* problems, int count,
                              aidw_batch_t* out) {
    ErrorScope es(h);
    if (!h || !out) return fail(AIDW_EINVAL, "handle or out is NULL");
    *out = nullptr;
    aidw_batch* b = new (std::nothrow) aidw_batch;
    if (!b) return fail(AIDW_ENOMEM, "host allocation failed");
    aidw_status st = batch_build(h, problems, count, b);
    if (st == AIDW_OK && b->launch.n_items > 0) st = batch_capture(b);
    if (st != AIDW_OK) {
        batch_release(b);
        delete b;
        return st;
    }
    *out = b;
    return AIDW_OK;
}

aidw_status aidw_batch_launch(aidw_batch_t b, unsigned flags) {
    ErrorScope es(b ? b->h : nullptr);
    if (!b) return fail(AIDW_EINVAL, "batch is NULL");
    if (b->launch.n_items == 0) return AIDW_OK;
    hipError_t e = hipGraphLaunch(b->exec, b->h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if (!(flags & AIDW_FLAG_ASYNC)) {
        e = hipStreamSynchronize(b->h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    return AIDW_OK;
}

void aidw_batch_destroy(aidw_batch_t b) {
    ErrorScope es(b ? b->h : nullptr);
    if (!b) return;
    if (b->h) (void)hipStreamSynchronize(b->h->stream);
    batch_release(b);
    delete b;
}

aidw_status aidw_interpolate_batch(aidw_t h, const aidw_problem* problems, int count,
                                   unsigned flags) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_batch b;
    aidw_status st = batch_build(h, problems, count, &b);
    if (st == AIDW_OK && b.launch.n_items > 0) {
        hipError_t e = aidw::launch_aidw_f32_batch(b.launch, h->stream);
        if (e != hipSuccess) st = hip_fail(e, "batched launch");
        // the work list lives until the launch completes
        hipError_t se = hipStreamSynchronize(h->stream);
        if (st == AIDW_OK && se != hipSuccess) st = hip_fail(se, "hipStreamSynchronize");
    }
    (void)flags;
    batch_release(&b);
    return st;
}

}  // extern "C"
