/*
 * libaidw -- Adaptive Inverse Distance Weighting on AMD Instinct MI355X
 * (gfx950), after Mei, Xu & Xu, "Accelerating Adaptive IDW Interpolation
 * Algorithm on a Single GPU" (arXiv 1511.02186).
 *
 * For every interpolated (query) point the library runs the paper's two full
 * passes over all m data points (Sec. 3.2, naive and tiled versions):
 *   pass 1: the k nearest data points -> r_obs (Eq. 3), R = r_obs / r_exp
 *           (Eq. 2, 4), mu_R (Eq. 5), the adaptive power alpha (Eq. 6);
 *   pass 2: Z = sum(d_i^-alpha z_i) / sum(d_i^-alpha) over all m points
 *           (Eq. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Geometry is 2-D.  Point sets are PLANAR structure-of-arrays in DEVICE
 *    memory: data_xy is [2][m] (the m x coordinates, then the m y
 *    coordinates), data_z is [m], query_xy is [2][n], out is [n].  The element
 *    type is float for AIDW_FP32_SCALED and double for AIDW_FP64.  Every
 *    pointer must be aligned to its element size.
 *  - The caller owns every buffer it passes; the library never frees or
 *    retains them past the call (or, for asynchronous calls, past the work's
 *    completion on the handle's stream).
 *  - Arguments are validated on the host before any device work.  On error
 *    nothing is launched, `out` is left untouched, and aidw_last_error(h)
 *    returns a message for the calling thread.
 *  - n == 0 is a valid no-op.
 *  - Work is issued on the handle's stream (aidw_set_stream; the NULL stream
 *    by default).  Unless AIDW_FLAG_ASYNC is given, calls return after the
 *    work has completed.
 *  - Handles are not thread-safe: use one handle per host thread.
 *
 * Readings of points the paper leaves open:
 *  - m in Eq. 2 is the number of data points (Sec. 2 names it n; Sec. 3
 *    renames it m); the study area A (`area`) is supplied by the caller.
 *  - Eq. 5 is evaluated literally with the argument (pi / R_max)(R - R_min);
 *    where the closed intervals of Eq. 5 and Eq. 6 overlap, the first listed
 *    case applies.
 *  - A query that coincides with data points (d = 0) returns the mean z of
 *    those points when alpha > 0; when alpha == 0 all weights are 1.
 *  - Equal distances in the kNN keep the smaller data index first.
 */
#ifndef AIDW_H
#define AIDW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AIDW_VERSION_MAJOR 0
#define AIDW_VERSION_MINOR 3

/* Largest supported k (neighbours kept in registers per query). */
#define AIDW_KMAX 32

/* Largest number of data points m, and of queries n, of one problem:
 * 2^31 - 2^16, so that every point index and every scan bound the kernels
 * form stays inside 32-bit signed arithmetic. */
#define AIDW_MAX_POINTS 2147418112LL

typedef enum aidw_status {
    AIDW_OK = 0,
    AIDW_EINVAL = -1,   /* an argument is out of its documented range */
    AIDW_ENOMEM = -2,   /* device or host allocation failed */
    AIDW_EDEVICE = -3,  /* a HIP call failed; the handle should be destroyed */
    AIDW_EAGAIN = -4,   /* not finished yet */
    AIDW_ENOTFOUND = -5 /* unknown ticket or dataset id */
} aidw_status;

typedef enum aidw_precision {
    /* float inputs and output; FP32 pair arithmetic with weights rescaled per
     * query as (d_min^2 / d^2)^(alpha/2) = exp2((alpha/2)(log2 d_min^2 -
     * log2 d^2)), or, where every query of a 64-query tile has the same
     * whole alpha in [1, 8], rsq(d^2)^alpha (times d_min^alpha unless max|z|
     * and d_min keep the unscaled sums inside the FP32 range); FP32 partial
     * sums folded into FP64 accumulators, FP64 r_obs / R / mu_R / alpha and
     * final division. */
    AIDW_FP32_SCALED = 0,
    /* double inputs and output; plain FP64: d^2 without FMA contraction,
     * weights pow(d, -alpha), compensated FP64 sums. */
    AIDW_FP64 = 1
} aidw_precision;

/* Flags for aidw_problem.flags. */
#define AIDW_FLAG_ASYNC 1u     /* return once the work is queued on the stream */
#define AIDW_FLAG_GRID_KNN 2u  /* FP32-scaled: find the k nearest through a uniform grid
                                  over the data (about 2 points per cell) instead of a
                                  full scan; the k nearest distances, r_obs and alpha
                                  are bit-identical to the full scan's, the output
                                  equal up to the order of its FP64 sums.  Pass 2
                                  still sums over all m points.  Not with knn_idx,
                                  FP32-scaled only.  Uses about 14 m + (16 + 16 S) n
                                  bytes of library workspace (S data segments of
                                  pass 2: about one per 128 K data points, at most 8,
                                  more when there are few queries). */

typedef struct aidw_options {
    int device;                        /* HIP device ordinal */
    aidw_precision default_precision;  /* used by aidw_interpolate() */
    size_t hbm_budget_bytes;           /* cap on library-owned device memory; 0 = none */
    const char* tune_path;             /* host string or NULL: a file written by
                                          aidw_tune_save, loaded at creation (a
                                          missing file is ignored, an invalid one
                                          fails creation with AIDW_EINVAL) */
    int deterministic;                 /* Every path of the library is deterministic run
                                          to run (no floating-point atomics; every sum
                                          has a fixed order).  Nonzero additionally makes
                                          FP32-scaled results independent of the
                                          automatic launch-shape choices, which depend on
                                          the device's compute-unit count and on tuning
                                          tables: such problems then always run the
                                          unsplit one-query-per-lane kernel (the kernel
                                          batched launches use), and grid-mode pass 2
                                          splits the data by m alone. */
} aidw_options;

typedef struct aidw_ctx* aidw_t;

/* One AIDW problem.  Pointer fields are device pointers unless stated. */
typedef struct aidw_problem {
    aidw_precision precision;
    const void* data_xy;     /* [2][m] planar x row then y row */
    const void* data_z;      /* [m] */
    int64_t m;               /* data points, 1 <= m <= AIDW_MAX_POINTS */
    const void* query_xy;    /* [2][n] planar */
    int64_t n;               /* queries, 0 <= n <= AIDW_MAX_POINTS */
    int k;                   /* neighbours for r_obs (Eq. 3), 1 <= k <= min(m, AIDW_KMAX) */
    double alpha_levels[5];  /* alpha_1..alpha_5 of Eq. 6; finite, >= 0 */
    double R_min, R_max;     /* Eq. 5 bounds; R_max > R_min, R_max > 0 */
    double area;             /* A of Eq. 2; finite, > 0 */
    void* out;               /* [n] interpolated values (float or double) */
    double* r_obs;           /* optional [n] observed mean kNN distance, or NULL */
    double* alpha;           /* optional [n] adaptive power, or NULL */
    int32_t* knn_idx;        /* optional [n][k] neighbour indices sorted by
                                (distance, index), or NULL */
    unsigned flags;          /* AIDW_FLAG_* */
} aidw_problem;

/* Create a handle on opt->device (opt may be NULL: device 0, FP32-scaled,
 * no budget, not deterministic).  Returns AIDW_EINVAL for a bad device, AIDW_EDEVICE if HIP
 * cannot be initialised. */
aidw_status aidw_create(aidw_t* out, const aidw_options* opt);

/* Finish the jobs submitted to the handle's serving loop, wait for the
 * handle's outstanding work, free library-owned memory and the handle.  NULL
 * is ignored. */
void aidw_destroy(aidw_t h);

/* Issue subsequent work on `stream` (a hipStream_t of the handle's device,
 * e.g. torch.cuda.current_stream().cuda_stream); NULL selects the default
 * stream.  Switching to another stream first waits for the work queued on
 * the previous one, since later calls reuse the handle's workspace. */
aidw_status aidw_set_stream(aidw_t h, void* stream);

/* AIDW of n queries over m data points (Eq. 1-6), in the handle's default
 * precision, synchronous.  Arguments as in aidw_problem; alpha_levels is a
 * host array of 5 doubles. */
aidw_status aidw_interpolate(aidw_t h, const void* data_xy, const void* data_z, int64_t m,
                             const void* query_xy, int64_t n, int k,
                             const double alpha_levels[5], double R_min, double R_max,
                             double area, void* out);

/* AIDW of one problem with an explicit precision, optional per-query
 * diagnostics (r_obs, alpha, kNN indices) and flags.  A call may grow the
 * handle's workspace (hipMalloc), so it is not meant to be recorded into a
 * hipGraph; aidw_batch_* captures and replays launches. */
aidw_status aidw_interpolate_ex(aidw_t h, const aidw_problem* p);

/* The kernels that aidw_interpolate_ex would launch for *p on this handle
 * (its tuning and options included), as text: kernel names as a profiler
 * shows them, joined by " + " in launch order, with the template arguments
 * of the k bucket (and queries per lane) chosen; empty for n == 0.  Writes at
 * most cap bytes including the terminating NUL (longer text is cut).
 * Launches nothing.  AIDW_EINVAL for an invalid problem or a NULL or empty
 * buffer. */
aidw_status aidw_describe_launch(aidw_t h, const aidw_problem* p, char* buf, size_t cap);

/* The spatial tile order that FP32-scaled launches use for these queries
 * (aidw_tuning.query_order): order[pos] (device array of n int32) receives
 * the index of the query at position pos, where positions 64 t .. 64 t + 63
 * form tile t.  The queries (planar [2][n] FP32 device array) are sorted,
 * stably, by the Morton code of their cell in a 2^b x 2^b grid over their
 * bounding box, b = the least b >= 1 with 16 * 4^b >= n, at most 11 (cell
 * index floor((x - x_min) * (2^b / (x_max - x_min))), in FP32, clamped to
 * [0, 2^b - 1]; 0 where the extent is zero or not finite).  Launches keep the
 * caller's order for a single tile (n <= 64); this function sorts any n >= 1.
 * Independent of the handle's tuning.  May grow the handle's workspace; waits
 * for the result.  Not part of the method: every query's result is its own in
 * any order. */
aidw_status aidw_query_order(aidw_t h, const void* query_xy, int64_t n, int32_t* order);

/* For callers that cannot allocate device memory: code being captured into
 * a hipGraph, tight serving loops, harnesses that forbid hipMalloc.  Same
 * problem, results and errors as aidw_interpolate_ex, but the call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * The buffers the FP32-scaled kernels need beyond inputs and outputs (max |z|
 * and the split-m partial lists and sums) live in a fixed device array of
 * AIDW_NOALLOC_SCRATCH_BYTES per device, which the library holds from the
 * first aidw_create on that device until the process ends (it is not
 * counted against hbm_budget_bytes).  Every kernel writes the scratch it
 * later reads within the same call, so no part of it must start at zero.
 * When the automatic split of the data would need more scratch than that,
 * the problem runs in as many segments as fit (down to the unsplit kernel,
 * which needs 256 bytes), so its output can differ from
 * aidw_interpolate_ex's in the last bits of the FP64 sums; when the split
 * fits, the output is bit-identical.  A split forced by aidw_set_tuning that
 * does not fit fails with AIDW_ENOMEM, and AIDW_FLAG_GRID_KNN with
 * AIDW_EINVAL.  FP64 problems use no scratch.  All calls on one device
 * share its array: calls that overlap on a device (several handles or
 * streams, or AIDW_FLAG_ASYNC calls not yet finished on another stream)
 * race, and must be serialised by the caller. */
#define AIDW_NOALLOC_SCRATCH_BYTES (64ull << 20)
aidw_status aidw_interpolate_noalloc(aidw_t h, const aidw_problem* p);

/* Standard IDW (Sec. 2.1, Eq. 1): every query uses the constant power
 * `power` (finite, >= 0) over all m data points.  Fields of *p as in
 * aidw_interpolate_ex; its k, alpha_levels, R_min, R_max and area are
 * ignored.  Runs the same kernels with every level set to `power` and k = 1
 * (the nearest distance, which the FP32-scaled weights are rescaled by);
 * the optional r_obs output then holds the nearest distance and knn_idx
 * (with k = 1) the nearest data index. */
aidw_status aidw_idw(aidw_t h, const aidw_problem* p, double power);

/* Data-access designs, for comparing the paper's implementation choices on
 * this GPU (Sec. 3.1.3 data layouts; Sec. 3.2 naive and tiled versions).
 * Every variant of a precision does the same arithmetic and differs only in
 * how data points reach the lanes. */
typedef enum aidw_access {
    AIDW_ACCESS_SCALAR = 0,  /* wave-uniform scalar loads (the production design) */
    AIDW_ACCESS_TILED = 1,   /* 256-point tiles staged in LDS per workgroup */
    AIDW_ACCESS_NAIVE = 2    /* one global load per lane per data point */
} aidw_access;
typedef enum aidw_layout {
    AIDW_LAYOUT_SOA = 0,   /* x[], y[], z[] as given */
    AIDW_LAYOUT_AOAS = 1   /* {x, y, z, pad} per point, aligned to its size, packed by
                              the library into its workspace */
} aidw_layout;

/* One problem with a given access design and layout.  Fields as in
 * aidw_interpolate_ex.  FP32-scaled variants do the arithmetic of
 * aidw_interpolate_ex with one query per lane (knn_idx must be NULL); FP64
 * variants are bit-identical to the plain FP64 kernel (knn_idx allowed).
 * AoaS needs 16 m (FP32) or 32 m (FP64) bytes of library workspace.
 * AIDW_FLAG_GRID_KNN is rejected (AIDW_EINVAL). */
aidw_status aidw_interpolate_variant(aidw_t h, const aidw_problem* p, aidw_access access,
                                     aidw_layout layout);

/* Launch shape of the FP32-scaled kernels.  Zero fields mean "automatic". */
typedef struct aidw_tuning {
    int q_per_lane;          /* queries owned by each lane: 1, 2 or 4 */
    int max_waves_per_simd;  /* cap on resident waves per SIMD (1..8), enforced by
                                reserving LDS per workgroup */
    int split_segments;      /* split the m data points into this many segments
                                processed in parallel (1: never split); chosen
                                automatically when the 64-query tiles give fewer
                                than two rounds of 8 waves per SIMD (1.5 rounds
                                when the speculative single pass applies) */
    int speculate;           /* 0: when alpha_5 is a whole power in [1, 8], pass 1
                                of the unsplit launch also forms the pass-2 sums of
                                that power, which stand for every query that ends
                                at alpha_5 with unscaled weights allowed (pass 2
                                then runs only for the other queries; results equal
                                to the two-pass kernel's to rounding, bit for bit
                                in every 64-query tile whose queries all kept
                                them); 1: never; 2: as 0, and also per data segment
                                in the split kernels (pays on data where nearly
                                every tile ends at alpha_5, such as uniform points;
                                costs on clustered data) */
    int query_order;         /* which queries share a 64-query tile.  0: Morton order
                                of their cells in the bounding box of the queries
                                (neighbours share a tile: their k-nearest screens
                                agree and, on clustered data, most tiles hold one
                                alpha), when there is more than one tile and at
                                least 1024 data points; 1: the caller's order;
                                2: Morton order whenever there is more than one
                                tile.  Unless 1, a split problem's pass 2 (alpha is
                                then known for every query) also regroups its
                                waves by the loop they take (whole power or not),
                                as long as no speculative sums are formed.  Each
                                query's result is its own in every
                                order; the grouping only sets which pass-2 loop a
                                wave takes, so results agree to rounding.  Batched
                                launches and deterministic handles use 0.  The
                                order needs about 20 n bytes of workspace; a call
                                whose HBM budget cannot hold it runs without. */
} aidw_tuning;

/* Fix the launch shape used for FP32-scaled problems (NULL restores the
 * automatic choice).  Returns AIDW_EINVAL for values outside the ranges
 * above. */
aidw_status aidw_set_tuning(aidw_t h, const aidw_tuning* t);

/* Autotuner.  Times the candidate launch shapes (queries per lane 1/2/4,
 * no split or the automatic number of data segments, half and twice it,
 * occupancy cap none/4, and for split launches speculate 0 or 2) of an
 * FP32-scaled problem of m data points, n queries and this k, on two
 * synthetic data sets with the same uniform queries: uniform points (alpha
 * ends at alpha_5 nearly everywhere) and clustered points (16 Gaussians of
 * widths 1e-4..1e-1 plus 10 % uniform: alpha varies), within about budget_s
 * seconds of GPU time, and records the shape with the least total time for
 * the size class (floor(log2 m), floor(log2 n), k bucket).  While the
 * handle's queries per lane, occupancy cap and split are automatic, later
 * calls in that class use the recorded shape (a nonzero speculate of the
 * handle's tuning still wins).  *best (may be NULL) receives it.  Uses
 * about 24 m + 12 n bytes of temporary device memory. */
aidw_status aidw_tune(aidw_t h, int64_t m, int64_t n, int k, double budget_s, aidw_tuning* best);
/* Write the handle's tuning table to `path` as JSON. */
aidw_status aidw_tune_save(aidw_t h, const char* path);
/* Replace the handle's tuning table by the one in `path` (written by
 * aidw_tune_save).  AIDW_ENOTFOUND if it cannot be read, AIDW_EINVAL if it
 * is not a tuning file or holds an invalid entry (the table is unchanged). */
aidw_status aidw_tune_load(aidw_t h, const char* path);

/* ---- Issue-cost probe --------------------------------------------------------
 * Not part of the method: a measurement of the device that bounds the FP32
 * kernels.  Their time is set by how long the instructions occupy a SIMD,
 * and without packed FP32 (disabled in every kernel of this library) that
 * is not what the 157.3 TFLOP/s packed-FMA figure assumes.  Runs five short
 * probe kernels (about 0.1 s) on the handle's stream; each value is SIMD
 * cycles per wave64 instruction. */
typedef struct aidw_issue_costs {
    double fma_cycles;             /* FP32 FMA, FMA-only waves (2.0 would be the packed peak) */
    double exp_cycles;             /* v_exp_f32, in waves that mix it with FMAs */
    double exp_cycles_beside_fma;  /* v_exp_f32 when other waves of the SIMD run FMAs */
    double clock_ghz;              /* clock used for the conversion */
    int compute_units;
    /* Two VALU instructions of different waves can issue in the same cycle
     * unless both read an SGPR (a data point's coordinate, in these
     * kernels): */
    double sgpr_operand_cycles;      /* v_sub_f32 v, s, v only */
    double sgpr_beside_vgpr_cycles;  /* the same alternating with VGPR-only multiplies */
} aidw_issue_costs;

aidw_status aidw_probe_issue_costs(aidw_t h, aidw_issue_costs* out);

/* ---- Batches: many independent problems in one launch ----------------------
 * Every problem must be AIDW_FP32_SCALED and may not request knn_idx.  The
 * (problem, 64-query tile) work items are ordered longest-first (by m) and
 * run one per wave in a single launch, so problems of very uneven size share
 * the GPU.  Results per query are bit-identical to aidw_interpolate_ex on
 * the same problem with q_per_lane = 1, no split and speculate = 1 (the
 * two-pass kernel). */
typedef struct aidw_batch* aidw_batch_t;

/* Validate the problems, upload the work list and capture the launch as a
 * hipGraph.  The problems' device buffers must stay valid while the batch
 * exists; their contents may change between launches.  On error nothing is
 * kept and aidw_last_error() names the offending problem. */
aidw_status aidw_batch_create(aidw_t h, const aidw_problem* problems, int count,
                              aidw_batch_t* out);

/* Replay the captured graph on the handle's current stream (synchronous
 * unless flags has AIDW_FLAG_ASYNC).  Launches of one batch must not
 * overlap: they share the batch's per-problem max-|z| slots. */
aidw_status aidw_batch_launch(aidw_batch_t b, unsigned flags);

/* Free the batch's device memory and graph (waits for the handle's stream). */
void aidw_batch_destroy(aidw_batch_t b);

/* One-shot batch: build, launch once, wait, free. */
aidw_status aidw_interpolate_batch(aidw_t h, const aidw_problem* problems, int count,
                                   unsigned flags);

/* ---- Serving: continuous batching of submitted jobs -----------------------
 * A server owns a worker thread, `streams` HIP streams and a device arena.
 * Submitted jobs are admitted in arrival order while the arena has room for
 * their workspace (FP32-scaled jobs whose data set exceeds `segment_points`
 * points are split into data segments and need a workspace; the others need
 * none).  A job that does not fit does not hold back later jobs that need no
 * workspace; later jobs that need workspace pass it only until it has waited
 * max_wait_s.  Each scheduling tick packs work items of all admitted jobs --
 * jobs that waited longer than max_wait_s first, then the shortest remaining
 * work -- into about tick_pair_evals distance evaluations (FP64 jobs counted
 * at 20 times their pair count, their relative cost), launched on one
 * stream, and up to `streams` ticks run at once, so jobs that arrive while
 * others are on the GPU start with the next tick.  A job's result does not
 * depend on which other jobs it shares ticks with.
 *
 * Each handle has a serving loop of its own, created with default options by
 * its first aidw_submit / aidw_submit_batch and finished by aidw_destroy;
 * aidw_server_create makes further servers with explicit options. */

/* A data set copied into library-owned device memory (counted against the
 * handle's budget).  data_xy [2][m] and data_z [m] are float device
 * pointers; the copy is complete when the call returns.  Registered data
 * sets serve FP32-scaled jobs. */
aidw_status aidw_dataset_register(aidw_t h, const void* data_xy, const void* data_z, int64_t m,
                                  double area, uint64_t* id);
/* Free a registered data set.  AIDW_EAGAIN while unfinished jobs read it,
 * AIDW_ENOTFOUND for an unknown id. */
aidw_status aidw_dataset_release(aidw_t h, uint64_t id);

typedef struct aidw_server_options {
    size_t arena_bytes;       /* device workspace for admitted split jobs, counted
                                 against the handle's budget (0: 2 GiB) */
    int streams;              /* ticks in flight, 1..8 (0: 2) */
    double tick_pair_evals;   /* distance evaluations per tick (0: 4e10) */
    double max_wait_s;        /* jobs older than this are served first (0: 0.25) */
    int64_t segment_points;   /* data points per segment of a split job (0: 32768) */
} aidw_server_options;

typedef struct aidw_server* aidw_server_t;

/* Start a server on the handle's device (opt may be NULL).  The handle must
 * outlive the server. */
aidw_status aidw_server_create(aidw_t h, const aidw_server_options* opt, aidw_server_t* out);
/* Finish every submitted job, then stop the worker and free the server. */
void aidw_server_destroy(aidw_server_t s);

/* One job (Eq. 1-6 for n queries over m data points, as aidw_problem).
 * Pointers are device pointers (float for AIDW_FP32_SCALED, double for
 * AIDW_FP64) that must stay valid, and the inputs unchanged, until the job
 * is reported done. */
typedef struct aidw_job {
    uint64_t dataset;        /* a registered data set (FP32-scaled jobs only), or 0 to
                                use the next four fields */
    const void* data_xy;     /* [2][m] */
    const void* data_z;      /* [m] */
    int64_t m;
    double area;             /* A of Eq. 2 */
    const void* query_xy;    /* [2][n] */
    int64_t n;
    int k;
    double alpha_levels[5];
    double R_min, R_max;
    aidw_precision precision; /* AIDW_FP32_SCALED or AIDW_FP64 (the plain FP64 kernel;
                                 never split into data segments) */
    void* out;               /* [n] */
    double* r_obs;           /* optional [n] */
    double* alpha;           /* optional [n] */
    int32_t* knn_idx;        /* optional [n][k], sorted by (distance, index); an
                                FP32-scaled job that asks for it is not split */
} aidw_job;

/* Validate and enqueue a job on the server; *ticket identifies it.
 * Thread-safe.  A job whose workspace can never fit the arena is accepted
 * and reported as failed with AIDW_ENOMEM by aidw_server_poll. */
aidw_status aidw_server_submit(aidw_server_t s, const aidw_job* job, uint64_t* ticket);
/* Validate and enqueue `count` jobs at once (host array jobs[count]);
 * tickets[i] identifies jobs[i].  All or nothing: if any job is invalid (the
 * error names its index) or names an unknown data set, none is enqueued and
 * every ticket is 0.  Jobs submitted together reach the scheduler together,
 * so they share ticks as far as the arena and the tick quota allow.
 * Thread-safe. */
aidw_status aidw_server_submit_batch(aidw_server_t s, const aidw_job* jobs, int count,
                                     uint64_t* tickets);
/* AIDW_EAGAIN while the job is queued or running.  Once it has finished,
 * returns AIDW_OK with *job_status (AIDW_OK or the job's error) and
 * *latency_s (seconds from submission to completion), then forgets the
 * ticket (later polls: AIDW_ENOTFOUND).  A failed job is reported only once
 * no kernel touches its buffers.  Thread-safe. */
aidw_status aidw_server_poll(aidw_server_t s, uint64_t ticket, aidw_status* job_status,
                             double* latency_s);
/* aidw_server_poll until the job finishes or timeout_s passes (AIDW_EAGAIN);
 * timeout_s < 0 waits indefinitely. */
aidw_status aidw_server_wait(aidw_server_t s, uint64_t ticket, double timeout_s,
                             aidw_status* job_status, double* latency_s);

/* The same four calls on the handle's own serving loop (created on first
 * use with default server options; its arena counts against the handle's
 * budget).  Tickets of different servers are unrelated. */
aidw_status aidw_submit(aidw_t h, const aidw_job* job, uint64_t* ticket);
aidw_status aidw_submit_batch(aidw_t h, const aidw_job* jobs, int count, uint64_t* tickets);
aidw_status aidw_poll(aidw_t h, uint64_t ticket, aidw_status* job_status, double* latency_s);
aidw_status aidw_wait(aidw_t h, uint64_t ticket, double timeout_s, aidw_status* job_status,
                      double* latency_s);

typedef struct aidw_server_counters {
    uint64_t submitted, completed, failed, ticks;
    double pair_evals;       /* distance evaluations of completed ticks */
    size_t arena_in_use;
    uint64_t queued, admitted;
} aidw_server_counters;

/* Counters of the server.  Returns the first device error the worker met,
 * if any. */
aidw_status aidw_server_stats(aidw_server_t s, aidw_server_counters* out);

/* Wait until all work issued on the handle's stream has finished. */
aidw_status aidw_synchronize(aidw_t h);

/* Message describing the calling thread's most recent failed call on handle
 * h (calls on its batches and servers included), or, with h == NULL, the
 * calling thread's most recent failed call of any kind (aidw_create
 * included).  "" if there is none.  The string stays valid until the calling
 * thread's next call into the library. */
const char* aidw_last_error(aidw_t h);

/* Static name of a status code. */
const char* aidw_status_string(aidw_status s);

/* Library version as (major << 16) | minor. */
int aidw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AIDW_H */
