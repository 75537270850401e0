// Scheduler of the AIDW serving loop: admission under a device-memory
// budget, continuous batching of work items into ticks, completion and
// latency accounting.  Pure C++ (no HIP): the device side is reached through
// the Executor interface, so the policy can be exercised with a fake
// executor and a fake clock.
#pragma once

#include <algorithm>
#include <array>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace aidw {
namespace serve {

// First-fit allocator of offsets inside a fixed arena [0, size).
class Arena {
   public:
    explicit Arena(size_t size = 0, size_t align = 256);
    bool alloc(size_t bytes, size_t* offset);
    void free(size_t offset);
    size_t size() const { return size_; }
    // Bytes a request of `bytes` occupies once rounded to the alignment.
    size_t rounded(size_t bytes) const { return (std::max<size_t>(bytes, 1) + align_ - 1) / align_ * align_; }
    size_t in_use() const { return in_use_; }

   private:
    std::map<size_t, size_t> free_;  // offset -> length, coalesced
    std::map<size_t, size_t> used_;  // offset -> length
    size_t size_, align_, in_use_ = 0;
};

enum class JobState { Queued, Admitted, Done, Failed };

enum Phase : int { kFused = 0, kKnn = 1, kSum = 2 };

// What the scheduler needs to know about a job.
struct JobSpec {
    int64_t m = 0;          // data points
    int64_t n = 0;          // queries
    int segments = 1;       // data segments (1: fused 64-query tiles)
    int64_t seg_len = 0;    // points per segment (== m when segments == 1)
    size_t ws_bytes = 0;    // device workspace held from admission to completion
    double cost_scale = 1.0;  // device time per distance evaluation relative to the
                              // FP32-scaled kernels (FP64 jobs are slower)
};

struct Item {
    uint64_t ticket;
    int phase;  // Phase
    int tile;   // 64-query tile
    int seg;    // data segment
};

struct TickPlan {
    std::vector<Item> items;
    std::vector<uint64_t> jobs;   // distinct tickets referenced by items, in first-use order
    double pair_evals = 0.0;      // distance evaluations in this tick
};

struct Config {
    size_t arena_bytes = 0;     // 0: no workspace can be admitted (fused jobs only)
    int slots = 2;              // ticks in flight (one stream each)
    double tick_pairs = 2e10;   // distance evaluations per tick (a soft quota)
    double max_wait_s = 0.25;   // older jobs are served first, in arrival order; a job
                                // that waits for workspace longer than this stops
                                // later workspace jobs from passing it
};

struct Stats {
    uint64_t submitted = 0, completed = 0, failed = 0, ticks = 0;
    double pair_evals = 0.0;    // completed distance evaluations
    size_t arena_in_use = 0;
    uint64_t queued = 0, admitted = 0;
};

class Executor {
   public:
    virtual ~Executor() = default;
    virtual double now() = 0;
    // The job is admitted; its workspace (if any) starts at ws_offset.
    // Returns 0, or a nonzero error that fails the job.
    virtual int admit(uint64_t ticket, size_t ws_offset) = 0;
    // Enqueue one tick on slot `slot`.  Returns 0 or an error (the tick's jobs fail).
    virtual int launch(const TickPlan& plan, int slot) = 0;
    // Has the last tick launched on `slot` completed?
    virtual bool done(int slot) = 0;
    // The job finished with `status` (0 = success); its resources may go.
    virtual void retire(uint64_t ticket, int status) = 0;
};

class Scheduler {
   public:
    Scheduler(Executor* ex, const Config& cfg);

    // Register a job.  Returns its ticket (> 0).  A job whose workspace can
    // never fit the arena fails at once (state Failed, status -2).
    //
    // Admission: queued jobs are admitted in arrival order while their
    // workspace fits the arena.  A job that does not fit does not block the
    // jobs behind it that need no workspace; jobs behind it that need
    // workspace may pass it only until it has waited max_wait_s, after which
    // the arena drains toward it.
    //
    // A job whose launch fails is reported Failed only once no tick that
    // carries its items is still in flight, so that no kernel reads or writes
    // its buffers, data set or workspace after the report; its workspace
    // returns to the arena at the same moment.
    uint64_t submit(const JobSpec& spec);
    // State of a job; latency (seconds from submit to completion) and
    // status are set once it is Done or Failed.  Unknown tickets: false.
    bool poll(uint64_t ticket, JobState* state, double* latency, int* status) const;
    // Drop the record of a finished job.
    void forget(uint64_t ticket);
    // One round: retire completed ticks, admit queued jobs, launch ticks on
    // free slots.  Returns true if anything changed.
    bool step();
    // No queued, admitted or in-flight work.
    bool idle() const;
    Stats stats() const;

   private:
    struct Job {
        JobSpec spec;
        JobState state = JobState::Queued;
        int status = 0;
        double t_submit = 0.0, t_done = 0.0;
        size_t ws_offset = 0;
        bool has_ws = false;
        int64_t tiles = 0;
        int64_t issued[3] = {0, 0, 0};  // items issued per phase
        int64_t done[3] = {0, 0, 0};    // items completed per phase
        double remaining = 0.0;         // distance evaluations not yet issued
        int inflight = 0;               // ticks in flight that carry its items
        bool failing = false;           // failed; completes when inflight reaches 0
        int fail_status = 0;
    };
    struct InFlight {
        bool busy = false;
        std::vector<std::pair<uint64_t, std::array<int64_t, 3>>> credits;
        double pair_evals = 0.0;
    };

    int64_t total_items(const Job& j, int phase) const;
    double item_cost(const Job& j, int phase) const;
    bool finished(const Job& j) const;
    void complete(uint64_t ticket, Job& j, int status);
    // Fail the job now, or once its in-flight ticks have completed.
    void fail(uint64_t ticket, Job& j, int status);
    bool retire_ticks();
    bool admit_jobs();
    bool launch_ticks();
    bool build_tick(TickPlan* plan, std::vector<std::pair<uint64_t, std::array<int64_t, 3>>>* credits);

    Executor* ex_;
    Config cfg_;
    Arena arena_;
    uint64_t next_ticket_ = 1;
    std::unordered_map<uint64_t, Job> jobs_;
    std::deque<uint64_t> queue_;      // submitted, not yet admitted (FIFO)
    std::vector<uint64_t> active_;    // admitted, not finished
    std::vector<InFlight> slots_;
    Stats stats_;
};

}  // namespace serve
}  // namespace aidw
