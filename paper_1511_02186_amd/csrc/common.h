// Internal declarations shared by the libaidw host code and its kernel
// translation units.  Not part of the public C ABI (see include/aidw.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aidw {

constexpr int kWaveSize = 64;
constexpr int kWavesPerGroup = 4;
constexpr int kGroupSize = kWaveSize * kWavesPerGroup;

// Largest k handled in registers (matches AIDW_KMAX).
constexpr int kKMax = 32;

// Per-problem constants of the alpha determination (Sec. 2.2, Eq. 2-6).
struct AlphaParams {
    double levels[5];  // alpha_1..alpha_5
    double R_min, R_max;
    double r_exp;      // Eq. 2, computed once per problem on the host
    int k;
};

// One FP32-scaled problem: planar device arrays, optional diagnostics.
struct ProblemF32 {
    const float* dx;
    const float* dy;
    const float* dz;
    const float* qx;
    const float* qy;
    float* out;
    double* r_obs;     // optional
    double* alpha;     // optional
    int32_t* knn;      // optional [n][k]
    int m;
    int n;
    AlphaParams ap;
    // optional: max |z| over the data (written by launch_abs_max before the
    // pass-2 kernels); lets whole-power waves skip the d_min rescaling
    const float* zmax;
    // Speculative single pass (set by the host): the whole power alpha_5 that
    // pass 1 may form the pass-2 sums for (0: none), and the sum of the k
    // neighbour distances below which a query no longer reaches that power's
    // range (mu_R >= 0.9 in Eq. 5), used to stop speculating early.
    int spec_power;
    float spec_dist_sum;
    // Optional tile order: position -> query index (null: the caller's
    // order).  Tiles are 64 consecutive positions; per-query results go to
    // the query's own index, internal per-query buffers are by position.
    const int* order;
};

struct ProblemF64 {
    const double* dx;
    const double* dy;
    const double* dz;
    const double* qx;
    const double* qy;
    double* out;
    double* r_obs;
    double* alpha;
    int32_t* knn;
    int m;
    int n;
    AlphaParams ap;
};

// Register bucket used for a given k: the top-k list holds K >= k entries,
// the first K - k of which are fixed at -infinity.
int k_bucket(int k);

// Launch configuration of the FP32-scaled fused kernel.
struct LaunchF32 {
    int q_per_lane;          // queries owned by each lane: 1, 2 or 4
    int max_waves_per_simd;  // 0: no cap; else LDS is reserved so that at most
                             // this many workgroups (one wave per SIMD each) share a CU
};

// LDS per compute unit on gfx950.
constexpr int kLdsPerCU = 160 * 1024;

// Split of the m data points into `segments` contiguous ranges of `seg_len`
// points (the last may be shorter), for problems with too few queries to
// fill the device.  tiles = ceil(n / 64).
struct SplitPlan {
    int segments;
    int seg_len;
    int tiles;
};

// Device workspace of a split launch (sizes in split_workspace_bytes).
struct SplitWorkspace {
    float* part;   // [segments][k][n] per-segment k nearest squared distances
    float* qpar;   // [4][n] per query: -alpha/2, (alpha/2) log2 d_min^2, d_min,
                   // and the whole power of the one-transcendental pass 2 (0: none)
    double* psum;  // [segments][2][n] per-segment sum w and sum w z
    // speculative sums (when the problem's spec_power is set):
    int* seg_ok;   // [segments][tiles] 1 where pass 1 formed the segment's sums
    int* tile_ok;  // [tiles] 1 where those sums stand for every segment
    // Pass-2 regrouping (null p2order: pass 2 takes the pass-1 tiles): the
    // positions sorted by their pass-2 loop (whole power, unscaled or not)
    unsigned* p2key;  // [n]
    int* p2hist;      // [256 * ceil(n / kOrderBlock)]
    int* p2order;     // [n] pass-2 slot -> position
};

// Workspace of the speculative single-pass launch (spec_workspace_bytes):
// queries whose speculative sums do not stand leave their pass-2 terms in
// qpar and a bit in their tile's mask; a list kernel turns the masks into
// their positions in position order (so the deferred waves, and with them
// each query's pass-2 loop, do not depend on timing), and the deferred pass
// 2 runs them, 64 list entries per wave, in data segments.
struct DeferWorkspace {
    int* count;    // queries listed (written by the list kernel)
    int* list;     // [n] positions of the listed queries, ascending
    unsigned long long* mask;  // [tiles] per tile: bit l set when lane l is deferred
    float* qpar;   // [4][n] as SplitWorkspace::qpar, for listed queries only
    double* psum;  // [segments][2][groups * 64] per-segment sums, by list slot
    int target;    // waves the deferred pass 2 aims for (one round of the chip)
};

// ---- spatial order of the queries ----------------------------------------------
// Queries are grouped into 64-query tiles in Morton order of their position
// in the bounding box of the problem's queries (2^bits cells per axis), so
// that a tile's queries are neighbours: their k-nearest screens trigger
// together, and on clustered data most tiles hold queries of one alpha.  The
// order is a stable LSD radix sort of the cell codes (8-bit digits), one or
// more independent problems (segments) at a time.
constexpr int kOrderThreads = 256;
constexpr int kOrderItems = 16;
constexpr int kOrderBlock = kOrderThreads * kOrderItems;  // queries per sort block

struct OrderSeg {
    const float* qx;
    const float* qy;
    int n;        // queries of this problem
    int base;     // its first position in the concatenated order
    int block0;   // its first sort block
    int nblocks;  // ceil(n / kOrderBlock)
    int bits;     // Morton bits per axis
};

// One order computation.  `table` (device array of `segments` entries, with
// block_seg[b] the segment of sort block b) or, when table is null, the
// single segment `one`.
struct OrderLaunch {
    const OrderSeg* table;
    const int* block_seg;
    OrderSeg one;
    int segments;
    int blocks;
    int passes;          // ceil(2 * max bits / 8)
    float4* bbox;        // [segments] x0, y0 and cells per unit in x and y
    float4* part;        // [blocks] each sort block's x0, x1, y0, y1
    unsigned* keys[2];   // [total] keys between passes
    int* vals[2];        // [total] query indices between passes
    int* hist;           // [blocks][256] digit counts, then scatter offsets
    int* order;          // [total] result: position -> query index in its problem
};

// Morton bits per axis for n queries (0: no order for a single tile).
int order_bits(int64_t n);
// Bytes of the order workspace for `total` queries in `blocks` sort blocks
// and `segments` problems; with L given, also lays it out at base.
size_t order_workspace_bytes(int64_t total, int blocks, int segments, int passes, OrderLaunch* L,
                             char* base);
hipError_t launch_query_order(const OrderLaunch& L, hipStream_t stream);
// Stable one-pass sort of positions 0..n-1 by keys[] < 256: order[slot] =
// position (hist: 256 * ceil(n / kOrderBlock) ints of workspace).
hipError_t launch_key_order(const unsigned* keys, int n, int* hist, int* order,
                            hipStream_t stream);

// One unit of batched work: 64 consecutive queries of one problem.
struct BatchItem {
    int problem;
    int base;  // first query of the tile
};

// max |z| of one problem's data into *out (each problem's zmax slot).
struct AbsMaxTask {
    const float* z;
    float* out;
    int m;
};

// A batched launch: one wave per item; the hardware dispatches workgroups in
// index order, so items sorted longest first start longest first.
struct BatchLaunch {
    const ProblemF32* problems;  // device array
    const BatchItem* items;      // device array, longest first
    const AbsMaxTask* tasks;     // device array, one per problem (fills problems[i].zmax)
    int n_tasks;
    int n_items;
    int K;                       // register bucket >= every problem's k
    OrderLaunch order;           // tile order of every problem (order.blocks 0: none)
};

// ---- serving: one launch per scheduling tick --------------------------------
// A job in a tick: its problem, its split and, for split jobs, its device
// workspace (partial lists, exponent terms, partial sums and two per-tile
// arrival counters that the last segment of a tile uses to merge or reduce).
struct ServeJob {
    ProblemF32 p;
    SplitPlan sp;       // sp.segments == 1: fused items only
    SplitWorkspace ws;  // unused when sp.segments == 1
    int* knn_arrivals;  // [tiles], zero before the job's first pass-1 item
    int* sum_arrivals;  // [tiles], zero before the job's first pass-2 item
};

enum ServePhase : int { kServeFused = 0, kServeKnn = 1, kServeSum = 2 };

struct ServeItem {
    int job;    // index into the tick's ServeJob array
    int phase;  // ServePhase
    int tile;   // 64-query tile
    int seg;    // data segment (split phases)
};

// One launch per tick, one wave per item.
struct ServeLaunch {
    const ServeJob* jobs;       // device array
    const ServeItem* items;     // device array
    const AbsMaxTask* tasks;    // device array, one per job (fills jobs[i].p.zmax)
    int n_tasks;
    int n_items;
    int K;
    bool track;                 // every item is a fused item of a job that wants knn_idx
};

hipError_t launch_aidw_f32_serve(const ServeLaunch& s, hipStream_t stream);
// FP64 jobs of a tick: one wave per (job, 64-query tile) item, phase ignored.
hipError_t launch_aidw_f64_serve(const ProblemF64* jobs, const ServeItem* items, int n_items,
                                 int K, bool track, hipStream_t stream);

// ---- k nearest through a uniform grid (pass 1 without the full scan) -------
struct GridGeom {
    int gx, gy;         // gx x gy cells over the data's bounding box
    float x0, y0;       // lower corner
    float cw, ch;       // cell width and height
    float inv_cw, inv_ch;
};

struct GridWorkspace {
    GridGeom* geo;
    float4* part;       // [nparts] partial bounding boxes
    int nparts;
    int cells;          // cap on gx * gy, fixed on the host
    int* counts;        // [cells + 1]
    int* start;         // [cells + 1] exclusive prefix sums of counts
    int* cursor;        // [cells]
    float2* sorted;     // [m] points ordered by cell
    void* temp;         // scan scratch
    size_t temp_bytes;
    float* qpar;        // [4][n] as in SplitWorkspace
    double* psum;       // [segments][2][n]
};

// max |z_i| over m values into *out (one workgroup; NaN wins, inf is kept).
// Also zeroes *clear when it is not null.
hipError_t launch_abs_max(const float* z, int m, float* out, hipStream_t s, int* clear = nullptr);
// The same for many arrays, one workgroup per task.
hipError_t launch_abs_max_tasks(const AbsMaxTask* tasks, int count, hipStream_t s);

int grid_cells(int64_t m);
size_t grid_temp_bytes(int cells);
// Build the grid and write each query's pass-2 terms (and r_obs / alpha).
hipError_t launch_grid_knn_all(const ProblemF32& p, const GridWorkspace& ws, hipStream_t s);
// Pass 2 over all m points from precomputed per-query terms (qpar), then the
// ratio: the split path's pass-2 kernels (sp.tiles is set here).
hipError_t launch_aidw_f32_pass2(const ProblemF32& p, SplitPlan sp, const float* qpar,
                                 double* psum, hipStream_t stream);

hipError_t launch_aidw_f32(const ProblemF32& p, const LaunchF32& cfg, const SplitPlan* sp,
                           const SplitWorkspace* ws, hipStream_t stream);
// The speculative single pass (p.spec_power != 0, one query per lane), then
// pass 2 of the tiles whose speculation failed.  p.zmax must have been written
// and *ws.count zeroed before (launch_abs_max with clear = ws.count).
hipError_t launch_aidw_f32_spec(const ProblemF32& p, const DeferWorkspace& ws, hipStream_t stream);
// Bytes of DeferWorkspace for n queries; with ws/base given, also lays it out
// at base (256-byte aligned).
size_t spec_workspace_bytes(int64_t n, int target, DeferWorkspace* ws, char* base);
hipError_t launch_aidw_f32_batch(const BatchLaunch& b, hipStream_t stream);
hipError_t launch_aidw_f64(const ProblemF64& p, hipStream_t stream);
// Data-access variants (0 scalar, 1 LDS tiles, 2 per-lane loads) x layouts
// (0 SoA, 1 AoaS packed into `aos`, m float4), same arithmetic.
hipError_t launch_aidw_f32_variant(const ProblemF32& p, int access, int layout, float4* aos,
                                   hipStream_t stream);
// The same designs for the plain FP64 kernel (access 0 with layout 0 is that
// kernel), `aos` m double4; bit-identical to it.
hipError_t launch_aidw_f64_variant(const ProblemF64& p, int access, int layout, double4* aos,
                                   hipStream_t stream);

}  // namespace aidw
