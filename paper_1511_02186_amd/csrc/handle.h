// Internal definition of the library handle and the host helpers shared by
// the translation units that implement the C ABI (api.hip, serve.hip).
#pragma once

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/aidw.h"
#include "common.h"

// A data set copied into library-owned device memory (aidw_dataset_register).
struct aidw_dataset_rec {
    float* xy = nullptr;  // [2][m]
    float* z = nullptr;   // [m]
    int64_t m = 0;
    double area = 0.0;
    size_t bytes = 0;
    int refs = 0;         // jobs in flight that read it
};

// Fastest launch shape measured for a size class (aidw_tune).
struct TuneEntry {
    int m_log2, n_log2, K;
    aidw_tuning shape;
    double ms;
};

struct aidw_server;

struct aidw_ctx {
    int device = 0;
    aidw_precision default_precision = AIDW_FP32_SCALED;
    bool deterministic = false;   // fixed launch shape for FP32-scaled problems
    size_t hbm_budget = 0;        // 0: unlimited
    size_t hbm_in_use = 0;        // library-owned device bytes
    hipStream_t stream = nullptr;
    int cu_count = 0;
    aidw_tuning tuning{0, 0, 0};  // zero fields: automatic
    void* workspace = nullptr;    // split-m scratch, grown on demand
    size_t workspace_bytes = 0;
    void* scratch = nullptr;      // this device's fixed scratch (aidw_interpolate_noalloc)
    // Registered data sets; the mutex also guards hbm_in_use, which servers
    // running on their own threads update.
    std::mutex mu;
    std::unordered_map<uint64_t, aidw_dataset_rec> datasets;
    uint64_t next_dataset = 1;
    std::vector<TuneEntry> tune_table;  // consulted when `tuning` is all automatic
    // The handle's own serving loop (aidw_submit / aidw_poll), created on first use.
    std::mutex server_mu;
    aidw_server* server = nullptr;
};

namespace aidw {
namespace detail {

// Record an error message for the calling thread (and for the handle of the
// innermost ErrorScope) and return s.
aidw_status fail(aidw_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Every public entry point that works on a handle opens one: errors raised
// while it is alive are also kept as the handle's message for this thread
// (aidw_last_error(h)).
class ErrorScope {
   public:
    explicit ErrorScope(const aidw_ctx* h);
    ~ErrorScope();
    ErrorScope(const ErrorScope&) = delete;
    ErrorScope& operator=(const ErrorScope&) = delete;

   private:
    const aidw_ctx* prev_;
};
// Forget the calling thread's message for h (the handle is being destroyed).
void forget_errors(const aidw_ctx* h);
aidw_status hip_fail(hipError_t e, const char* what);
aidw_status validate(const aidw_problem* p);
AlphaParams alpha_params(const aidw_problem* p);
ProblemF32 problem_f32(const aidw_problem* p);
// Morton bits of the spatial tile order of a problem (0: the caller's
// order).  mode: aidw_tuning.query_order (0 automatic: more than one tile
// and at least 1024 data points; 1 never; 2 whenever there is more than one
// tile).  Batched launches, serving and deterministic handles use 0.
int order_bits_for(int mode, int64_t m, int64_t n);
int order_passes(int bits);   // 8-bit radix passes for 2 * bits key bits
int order_blocks(int64_t n);  // sort blocks of n queries
ProblemF64 problem_f64(const aidw_problem* p);
aidw_status device_alloc(aidw_t h, size_t bytes, void** out);
void device_free(aidw_t h, void* p, size_t bytes);
// Bytes of a split workspace; with ws/base given, also lays it out at base.
size_t split_workspace_bytes(const SplitPlan& sp, int k, int64_t n, SplitWorkspace* ws,
                             char* base, bool regroup = false);
// Data segments of a problem under launch shape t (t.split_segments: 0
// automatic, 1 never split, S forced).
SplitPlan split_plan_for(const aidw_ctx* h, const aidw_tuning& t, int64_t m, int64_t n);
// The tuned shape of the size class of (m, n, k), if aidw_tune measured one.
bool tuned_shape(const aidw_ctx* h, int64_t m, int64_t n, int k, aidw_tuning* out);

}  // namespace detail
}  // namespace aidw
