// Serving loop of libaidw: registered data sets, job submission and
// polling, and the HIP executor that turns each scheduling tick into one
// launch of the serving kernel (declared in include/aidw.h).
//
// Threads: client threads call aidw_server_submit / _poll / _wait (or the
// handle-level aidw_submit / aidw_poll / aidw_wait); one worker thread per
// server runs the scheduler.  Every scheduler and executor call happens
// under the server's mutex.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "handle.h"
#include "serve_sched.h"

using namespace aidw::detail;
namespace sv = aidw::serve;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Device time of a plain FP64 distance evaluation relative to an
// FP32-scaled one (the FP64 kernel runs about 20x slower per pair); the
// scheduler weighs FP64 jobs by it against the tick quota.
constexpr double kF64CostScale = 20.0;

struct JobRec {
    aidw_precision precision = AIDW_FP32_SCALED;
    aidw::ProblemF32 p{};       // FP32-scaled jobs
    aidw::ProblemF64 p64{};     // FP64 jobs
    aidw::SplitPlan sp{};
    int K = 4;
    bool track = false;         // knn_idx wanted: fused items only, index-tracking kernel
    int order_bits = 0;         // spatial tile order (computed at admission), 0: none
    size_t ws_bytes = 0;        // tile order, split workspace, two arrival-counter arrays
    size_t split_off = 0;       // offset of the split workspace inside the job's workspace
    size_t counters_off = 0;    // offset of the counters inside the job's workspace
    char* ws = nullptr;         // device address of the job's workspace
    uint64_t zero_seq = 0;      // admin-stream sequence number that cleared its counters
    uint64_t dataset = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    uint64_t admin_seen = 0;  // admin-stream work this stream has been ordered after
    void* host = nullptr;     // pinned staging of the tick's jobs and items
    size_t host_cap = 0;
    void* dev = nullptr;
    size_t dev_cap = 0;
};

// Item kinds of a tick, one kernel launch each (on the tick's stream).
enum Kind { kF32 = 0, kF32Track = 1, kF64 = 2, kF64Track = 3, kKinds = 4 };

class HipExecutor : public sv::Executor {
   public:
    aidw_t h = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::unordered_map<uint64_t, JobRec> jobs;
    std::vector<Slot> slots;
    // Split jobs' arrival counters are cleared on this stream when the job
    // is admitted; every slot stream waits for `admin_done` before it runs a
    // tick that carries a job it has not yet been ordered after.
    hipStream_t admin = nullptr;
    hipEvent_t admin_done = nullptr;
    uint64_t admin_seq = 0;
    aidw_status error = AIDW_OK;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // The job's tile order and its split counters are set up on the admin
    // stream, which every tick carrying the job waits for.
    int admit(uint64_t t, size_t off) override {
        JobRec& r = jobs[t];
        if (r.ws_bytes == 0) return 0;
        r.ws = arena + off;
        hipError_t e = hipSuccess;
        if (r.order_bits) {
            aidw::OrderLaunch L{};
            const int passes = order_passes(r.order_bits), blocks = order_blocks(r.p.n);
            aidw::order_workspace_bytes(r.p.n, blocks, 1, passes, &L, r.ws);
            L.one = aidw::OrderSeg{r.p.qx, r.p.qy, r.p.n, 0, 0, blocks, r.order_bits};
            L.segments = 1;
            L.blocks = blocks;
            L.passes = passes;
            e = aidw::launch_query_order(L, admin);
            r.p.order = L.order;
        }
        if (e == hipSuccess && r.sp.segments > 1)
            e = hipMemsetAsync(r.ws + r.counters_off, 0, 2 * sizeof(int) * (size_t)r.sp.tiles,
                               admin);
        if (e == hipSuccess) e = hipEventRecord(admin_done, admin);
        if (e != hipSuccess) {
            error = hip_fail(e, "job set-up on the admin stream");
            return AIDW_EDEVICE;
        }
        r.zero_seq = ++admin_seq;
        return 0;
    }

    int launch(const sv::TickPlan& plan, int slot) override {
        Slot& s = slots[(size_t)slot];
        std::unordered_map<uint64_t, int> index;
        std::vector<aidw::ServeJob> sj;
        std::vector<aidw::ProblemF64> sj64;
        uint64_t need_seq = 0;
        for (uint64_t t : plan.jobs) {
            JobRec& r = jobs[t];
            need_seq = std::max(need_seq, r.zero_seq);
            if (r.precision == AIDW_FP64) {
                index[t] = (int)sj64.size();
                sj64.push_back(r.p64);
                continue;
            }
            index[t] = (int)sj.size();
            aidw::ServeJob j{};
            j.p = r.p;
            j.sp = r.sp;
            if (r.sp.segments > 1) {
                split_workspace_bytes(r.sp, r.p.ap.k, r.p.n, &j.ws, r.ws + r.split_off);
                j.knn_arrivals = reinterpret_cast<int*>(r.ws + r.counters_off);
                j.sum_arrivals = j.knn_arrivals + r.sp.tiles;
            }
            sj.push_back(j);
        }
        // items grouped by kernel, each group in plan order
        std::vector<aidw::ServeItem> items[kKinds];
        int K[kKinds] = {4, 4, 4, 4};
        for (const sv::Item& it : plan.items) {
            const JobRec& r = jobs[it.ticket];
            const int kind = (r.precision == AIDW_FP64 ? kF64 : kF32) + (r.track ? 1 : 0);
            items[kind].push_back(aidw::ServeItem{index[it.ticket], it.phase, it.tile, it.seg});
            K[kind] = std::max(K[kind], r.K);
        }
        // staging: f32 jobs | f64 jobs | items of each kind | max-|z| tasks |
        // max-|z| slots (one per f32 job, recomputed by every tick that
        // carries the job, on the tick's own stream)
        size_t off = 0;
        const size_t o_jobs = off;
        off += align_up(sizeof(aidw::ServeJob) * sj.size());
        const size_t o_jobs64 = off;
        off += align_up(sizeof(aidw::ProblemF64) * sj64.size());
        size_t o_items[kKinds];
        for (int k = 0; k < kKinds; ++k) {
            o_items[k] = off;
            off += align_up(sizeof(aidw::ServeItem) * items[k].size());
        }
        const size_t o_tasks = off;
        off += align_up(sizeof(aidw::AbsMaxTask) * sj.size());
        const size_t o_z = off;
        const size_t bytes = o_z + align_up(sizeof(float) * sj.size());
        if (grow(s, bytes) != AIDW_OK) return AIDW_ENOMEM;
        char* host = static_cast<char*>(s.host);
        char* dev = static_cast<char*>(s.dev);
        float* zslots = reinterpret_cast<float*>(dev + o_z);
        std::vector<aidw::AbsMaxTask> tasks(sj.size());
        for (size_t i = 0; i < sj.size(); ++i) {
            sj[i].p.zmax = zslots + i;
            tasks[i] = aidw::AbsMaxTask{sj[i].p.dz, zslots + i, sj[i].p.m};
        }
        if (!sj.empty()) memcpy(host + o_jobs, sj.data(), sizeof(aidw::ServeJob) * sj.size());
        if (!sj64.empty())
            memcpy(host + o_jobs64, sj64.data(), sizeof(aidw::ProblemF64) * sj64.size());
        for (int k = 0; k < kKinds; ++k)
            if (!items[k].empty())
                memcpy(host + o_items[k], items[k].data(), sizeof(aidw::ServeItem) * items[k].size());
        if (!tasks.empty())
            memcpy(host + o_tasks, tasks.data(), sizeof(aidw::AbsMaxTask) * tasks.size());
        hipError_t e = hipMemcpyAsync(dev, host, o_z, hipMemcpyHostToDevice, s.stream);
        // the counters of every split job in this tick were cleared on the
        // admin stream: order this stream after that
        if (e == hipSuccess && need_seq > s.admin_seen) {
            e = hipStreamWaitEvent(s.stream, admin_done, 0);
            s.admin_seen = admin_seq;
        }
        if (e != hipSuccess) {
            error = hip_fail(e, "tick upload");
            return AIDW_EDEVICE;
        }
        int tasks_left = (int)tasks.size();  // max |z| runs before the first f32 launch
        for (int k = kF32; k <= kF32Track && e == hipSuccess; ++k) {
            if (items[k].empty()) continue;
            aidw::ServeLaunch sl{};
            sl.jobs = reinterpret_cast<const aidw::ServeJob*>(dev + o_jobs);
            sl.items = reinterpret_cast<const aidw::ServeItem*>(dev + o_items[k]);
            sl.tasks = reinterpret_cast<const aidw::AbsMaxTask*>(dev + o_tasks);
            sl.n_tasks = tasks_left;
            sl.n_items = (int)items[k].size();
            sl.K = aidw::k_bucket(K[k]);
            sl.track = k == kF32Track;
            e = aidw::launch_aidw_f32_serve(sl, s.stream);
            tasks_left = 0;
        }
        for (int k = kF64; k <= kF64Track && e == hipSuccess; ++k) {
            if (items[k].empty()) continue;
            e = aidw::launch_aidw_f64_serve(
                reinterpret_cast<const aidw::ProblemF64*>(dev + o_jobs64),
                reinterpret_cast<const aidw::ServeItem*>(dev + o_items[k]), (int)items[k].size(),
                aidw::k_bucket(K[k]), k == kF64Track, s.stream);
        }
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) {
            error = hip_fail(e, "tick launch");
            return AIDW_EDEVICE;
        }
        s.launched = true;
        return 0;
    }

    bool done(int slot) override {
        Slot& s = slots[(size_t)slot];
        if (!s.launched) return true;
        const hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) error = hip_fail(e, "tick completion");
        s.launched = false;
        return true;
    }

    void retire(uint64_t t, int) override {
        auto it = jobs.find(t);
        if (it == jobs.end()) return;
        if (it->second.dataset) {
            std::lock_guard<std::mutex> lk(h->mu);
            auto d = h->datasets.find(it->second.dataset);
            if (d != h->datasets.end()) --d->second.refs;
        }
        jobs.erase(it);
    }

   private:
    aidw_status grow(Slot& s, size_t bytes) {
        if (bytes > s.host_cap) {
            if (s.host) (void)hipHostFree(s.host);
            s.host = nullptr;
            s.host_cap = 0;
            if (hipHostMalloc(&s.host, bytes * 2, hipHostMallocDefault) != hipSuccess) {
                s.host = nullptr;
                return fail(AIDW_ENOMEM, "pinned staging of %zu bytes", bytes * 2);
            }
            s.host_cap = bytes * 2;
        }
        if (bytes > s.dev_cap) {
            device_free(h, s.dev, s.dev_cap);
            s.dev = nullptr;
            s.dev_cap = 0;
            aidw_status st = device_alloc(h, bytes * 2, &s.dev);
            if (st != AIDW_OK) return st;
            s.dev_cap = bytes * 2;
        }
        return AIDW_OK;
    }
};

aidw_status to_status(int rc) {
    if (rc == 0) return AIDW_OK;
    if (rc == -2) return AIDW_ENOMEM;
    return rc < 0 ? (aidw_status)rc : AIDW_EDEVICE;
}

}  // namespace

struct aidw_server {
    aidw_t h = nullptr;
    HipExecutor ex;
    sv::Scheduler* sched = nullptr;
    aidw_server_options opt{};
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;

    void run() {
        (void)hipSetDevice(h->device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            const bool changed = sched->step();
            if (stop && sched->idle()) break;
            if (!changed) cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
};

namespace {

// Validate one job and build its record and scheduler spec (no server lock).
aidw_status prepare_job(aidw_server* s, const aidw_job* job, JobRec* out, sv::JobSpec* spec_out) {
    aidw_problem p;
    memset(&p, 0, sizeof p);
    p.precision = job->precision;
    p.data_xy = job->data_xy;
    p.data_z = job->data_z;
    p.m = job->m;
    p.area = job->area;
    aidw_t h = s->h;
    if (job->dataset) {
        if (job->precision != AIDW_FP32_SCALED)
            return fail(AIDW_EINVAL, "registered data sets hold FP32 data: FP32-scaled jobs only");
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->datasets.find(job->dataset);
        if (it == h->datasets.end())
            return fail(AIDW_ENOTFOUND, "no dataset %llu", (unsigned long long)job->dataset);
        p.data_xy = it->second.xy;
        p.data_z = it->second.z;
        p.m = it->second.m;
        p.area = it->second.area;
    }
    p.query_xy = job->query_xy;
    p.n = job->n;
    p.k = job->k;
    for (int i = 0; i < 5; ++i) p.alpha_levels[i] = job->alpha_levels[i];
    p.R_min = job->R_min;
    p.R_max = job->R_max;
    p.out = job->out;
    p.r_obs = job->r_obs;
    p.alpha = job->alpha;
    p.knn_idx = job->knn_idx;
    aidw_status st = validate(&p);
    if (st != AIDW_OK) return st;

    JobRec r;
    r.precision = p.precision;
    r.K = aidw::k_bucket(p.k);
    r.track = p.knn_idx != nullptr;
    r.sp = aidw::SplitPlan{1, (int)p.m, (int)((p.n + 63) / 64)};
    sv::JobSpec spec;
    spec.m = p.m;
    spec.n = p.n;
    if (p.precision == AIDW_FP64) {
        // the plain FP64 kernel, 64-query tiles over all m points
        r.p64 = problem_f64(&p);
        spec.cost_scale = kF64CostScale;
    } else {
        r.p = problem_f32(&p);
        // workspace: tile order | split buffers | arrival counters.  The order
        // is left out where it would take more than an eighth of the arena.
        r.order_bits = order_bits_for(0, p.m, p.n);
        size_t order_bytes = 0;
        if (r.order_bits) {
            order_bytes = align_up(aidw::order_workspace_bytes(
                p.n, order_blocks(p.n), 1, order_passes(r.order_bits), nullptr, nullptr));
            if (order_bytes > s->ex.arena_bytes / 8) {
                r.order_bits = 0;
                order_bytes = 0;
            }
        }
        r.split_off = order_bytes;
        r.ws_bytes = order_bytes;
        const int64_t seg = (s->opt.segment_points + 31) / 32 * 32;
        if (p.m > seg && p.n > 0 && !r.track) {
            r.sp.seg_len = (int)seg;
            r.sp.segments = (int)((p.m + seg - 1) / seg);
            r.counters_off =
                r.split_off + align_up(split_workspace_bytes(r.sp, p.k, p.n, nullptr, nullptr));
            r.ws_bytes = r.counters_off + 2 * sizeof(int) * (size_t)r.sp.tiles;
            spec.segments = r.sp.segments;
            spec.seg_len = seg;
        }
        spec.ws_bytes = r.ws_bytes;
    }
    r.dataset = job->dataset;
    *out = r;
    *spec_out = spec;
    return AIDW_OK;
}

// The handle's own serving loop, created with default options on first use.
aidw_status handle_server(aidw_t h, bool create, aidw_server** out) {
    std::lock_guard<std::mutex> lk(h->server_mu);
    if (!h->server && create) {
        aidw_status st = aidw_server_create(h, nullptr, &h->server);
        if (st != AIDW_OK) return st;
    }
    *out = h->server;
    return AIDW_OK;
}

}  // namespace

extern "C" {

aidw_status aidw_dataset_register(aidw_t h, const void* data_xy, const void* data_z, int64_t m,
                                  double area, uint64_t* id) {
    ErrorScope es(h);
    if (!h || !id) return fail(AIDW_EINVAL, "handle or id is NULL");
    *id = 0;
    if (m < 1 || m > AIDW_MAX_POINTS)
        return fail(AIDW_EINVAL, "m = %lld out of [1, %lld]", (long long)m, (long long)AIDW_MAX_POINTS);
    if (!std::isfinite(area) || area <= 0.0) return fail(AIDW_EINVAL, "area must be finite and > 0");
    if (!data_xy || !data_z) return fail(AIDW_EINVAL, "NULL data pointer");
    if ((uintptr_t)data_xy % 4 || (uintptr_t)data_z % 4)
        return fail(AIDW_EINVAL, "pointer not aligned to 4 bytes");
    const size_t bxy = align_up(2 * sizeof(float) * (size_t)m);
    const size_t bytes = bxy + sizeof(float) * (size_t)m;
    void* mem = nullptr;
    aidw_status st = device_alloc(h, bytes, &mem);
    if (st != AIDW_OK) return st;
    char* base = static_cast<char*>(mem);
    hipError_t e = hipMemcpyAsync(base, data_xy, 2 * sizeof(float) * (size_t)m,
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + bxy, data_z, sizeof(float) * (size_t)m, hipMemcpyDeviceToDevice,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        device_free(h, mem, bytes);
        return hip_fail(e, "dataset copy");
    }
    std::lock_guard<std::mutex> lk(h->mu);
    aidw_dataset_rec r;
    r.xy = reinterpret_cast<float*>(base);
    r.z = reinterpret_cast<float*>(base + bxy);
    r.m = m;
    r.area = area;
    r.bytes = bytes;
    *id = h->next_dataset++;
    h->datasets[*id] = r;
    return AIDW_OK;
}

aidw_status aidw_dataset_release(aidw_t h, uint64_t id) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_dataset_rec r;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->datasets.find(id);
        if (it == h->datasets.end()) return fail(AIDW_ENOTFOUND, "no dataset %llu", (unsigned long long)id);
        if (it->second.refs > 0)
            return fail(AIDW_EAGAIN, "dataset %llu is read by %d unfinished jobs",
                        (unsigned long long)id, it->second.refs);
        r = it->second;
        h->datasets.erase(it);
    }
    device_free(h, r.xy, r.bytes);
    return AIDW_OK;
}

aidw_status aidw_server_create(aidw_t h, const aidw_server_options* opt, aidw_server_t* out) {
    ErrorScope es(h);
    if (!h || !out) return fail(AIDW_EINVAL, "handle or out is NULL");
    *out = nullptr;
    aidw_server_options o{};
    if (opt) o = *opt;
    if (o.arena_bytes == 0) o.arena_bytes = (size_t)2 << 30;
    if (o.streams <= 0) o.streams = 2;
    if (o.tick_pair_evals <= 0) o.tick_pair_evals = 4e10;
    if (o.max_wait_s <= 0) o.max_wait_s = 0.25;
    if (o.segment_points <= 0) o.segment_points = 32768;
    if (o.streams > 8) return fail(AIDW_EINVAL, "streams = %d > 8", o.streams);
    aidw_server* s = new (std::nothrow) aidw_server;
    if (!s) return fail(AIDW_ENOMEM, "host allocation failed");
    s->h = h;
    s->opt = o;
    s->ex.h = h;
    void* arena = nullptr;
    aidw_status st = device_alloc(h, o.arena_bytes, &arena);
    if (st != AIDW_OK) {
        delete s;
        return st;
    }
    s->ex.arena = static_cast<char*>(arena);
    s->ex.arena_bytes = o.arena_bytes;
    s->ex.slots.resize((size_t)o.streams);
    {
        hipError_t e = hipStreamCreateWithFlags(&s->ex.admin, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ex.admin_done, hipEventDisableTiming);
        if (e != hipSuccess) {
            st = hip_fail(e, "stream or event creation");
            aidw_server_destroy(s);
            return st;
        }
    }
    for (Slot& sl : s->ex.slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            st = hip_fail(e, "stream or event creation");
            aidw_server_destroy(s);
            return st;
        }
    }
    sv::Config cfg;
    cfg.arena_bytes = o.arena_bytes;
    cfg.slots = o.streams;
    cfg.tick_pairs = o.tick_pair_evals;
    cfg.max_wait_s = o.max_wait_s;
    s->sched = new (std::nothrow) sv::Scheduler(&s->ex, cfg);
    if (!s->sched) {
        aidw_server_destroy(s);
        return fail(AIDW_ENOMEM, "host allocation failed");
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return AIDW_OK;
}

void aidw_server_destroy(aidw_server_t s) {
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        s->worker.join();
    }
    for (Slot& sl : s->ex.slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.host) (void)hipHostFree(sl.host);
        device_free(s->h, sl.dev, sl.dev_cap);
    }
    if (s->ex.admin) (void)hipStreamSynchronize(s->ex.admin);
    if (s->ex.admin_done) (void)hipEventDestroy(s->ex.admin_done);
    if (s->ex.admin) (void)hipStreamDestroy(s->ex.admin);
    device_free(s->h, s->ex.arena, s->ex.arena_bytes);
    delete s->sched;
    delete s;
}

aidw_status aidw_server_submit(aidw_server_t s, const aidw_job* job, uint64_t* ticket) {
    ErrorScope es(s ? s->h : nullptr);
    if (!s || !job || !ticket) return fail(AIDW_EINVAL, "server, job or ticket is NULL");
    return aidw_server_submit_batch(s, job, 1, ticket);
}

aidw_status aidw_server_submit_batch(aidw_server_t s, const aidw_job* jobs, int count,
                                     uint64_t* tickets) {
    ErrorScope es(s ? s->h : nullptr);
    if (!s || count < 0 || (count > 0 && (!jobs || !tickets)))
        return fail(AIDW_EINVAL, "server, jobs or tickets is NULL, or count < 0");
    for (int i = 0; i < count; ++i) tickets[i] = 0;
    std::vector<JobRec> recs((size_t)count);
    std::vector<sv::JobSpec> specs((size_t)count);
    for (int i = 0; i < count; ++i) {
        const aidw_status st = prepare_job(s, &jobs[i], &recs[(size_t)i], &specs[(size_t)i]);
        if (st != AIDW_OK) {
            const std::string msg = aidw_last_error(nullptr);
            return count == 1 ? fail(st, "%s", msg.c_str())
                              : fail(st, "job %d: %s", i, msg.c_str());
        }
    }
    aidw_t h = s->h;
    std::lock_guard<std::mutex> lk(s->mu);
    {
        // data sets may have been released since validation: check them all,
        // then take every reference, so that either all jobs enter or none
        std::lock_guard<std::mutex> lk2(h->mu);
        for (int i = 0; i < count; ++i) {
            const uint64_t d = recs[(size_t)i].dataset;
            if (d && h->datasets.find(d) == h->datasets.end())
                return fail(AIDW_ENOTFOUND, "job %d: no dataset %llu", i, (unsigned long long)d);
        }
        for (int i = 0; i < count; ++i)
            if (recs[(size_t)i].dataset) ++h->datasets.find(recs[(size_t)i].dataset)->second.refs;
    }
    for (int i = 0; i < count; ++i) {
        const uint64_t t = s->sched->submit(specs[(size_t)i]);
        sv::JobState state;
        s->sched->poll(t, &state, nullptr, nullptr);
        s->ex.jobs[t] = recs[(size_t)i];
        if (state == sv::JobState::Failed) s->ex.retire(t, -2);  // drops the dataset reference
        tickets[i] = t;
    }
    s->cv.notify_one();
    return AIDW_OK;
}

aidw_status aidw_server_poll(aidw_server_t s, uint64_t ticket, aidw_status* job_status,
                             double* latency_s) {
    ErrorScope es(s ? s->h : nullptr);
    if (!s) return fail(AIDW_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    sv::JobState state;
    double lat = 0.0;
    int rc = 0;
    if (!s->sched->poll(ticket, &state, &lat, &rc))
        return fail(AIDW_ENOTFOUND, "no ticket %llu", (unsigned long long)ticket);
    if (state == sv::JobState::Queued || state == sv::JobState::Admitted) return AIDW_EAGAIN;
    if (job_status) *job_status = to_status(rc);
    if (latency_s) *latency_s = lat;
    s->sched->forget(ticket);
    return AIDW_OK;
}

aidw_status aidw_server_wait(aidw_server_t s, uint64_t ticket, double timeout_s,
                             aidw_status* job_status, double* latency_s) {
    const auto t_end = std::chrono::steady_clock::now() +
                       std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s);
    for (;;) {
        aidw_status st = aidw_server_poll(s, ticket, job_status, latency_s);
        if (st != AIDW_EAGAIN) return st;
        if (std::chrono::steady_clock::now() >= t_end) return AIDW_EAGAIN;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

aidw_status aidw_server_stats(aidw_server_t s, aidw_server_counters* out) {
    ErrorScope es(s ? s->h : nullptr);
    if (!s || !out) return fail(AIDW_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    const sv::Stats st = s->sched->stats();
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->failed = st.failed;
    out->ticks = st.ticks;
    out->pair_evals = st.pair_evals;
    out->arena_in_use = st.arena_in_use;
    out->queued = st.queued;
    out->admitted = st.admitted;
    return s->ex.error;
}

aidw_status aidw_submit(aidw_t h, const aidw_job* job, uint64_t* ticket) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_server* s = nullptr;
    aidw_status st = handle_server(h, true, &s);
    return st != AIDW_OK ? st : aidw_server_submit(s, job, ticket);
}

aidw_status aidw_submit_batch(aidw_t h, const aidw_job* jobs, int count, uint64_t* tickets) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_server* s = nullptr;
    aidw_status st = handle_server(h, true, &s);
    return st != AIDW_OK ? st : aidw_server_submit_batch(s, jobs, count, tickets);
}

aidw_status aidw_poll(aidw_t h, uint64_t ticket, aidw_status* job_status, double* latency_s) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_server* s = nullptr;
    (void)handle_server(h, false, &s);
    if (!s) return fail(AIDW_ENOTFOUND, "no ticket %llu", (unsigned long long)ticket);
    return aidw_server_poll(s, ticket, job_status, latency_s);
}

aidw_status aidw_wait(aidw_t h, uint64_t ticket, double timeout_s, aidw_status* job_status,
                      double* latency_s) {
    ErrorScope es(h);
    if (!h) return fail(AIDW_EINVAL, "handle is NULL");
    aidw_server* s = nullptr;
    (void)handle_server(h, false, &s);
    if (!s) return fail(AIDW_ENOTFOUND, "no ticket %llu", (unsigned long long)ticket);
    return aidw_server_wait(s, ticket, timeout_s, job_status, latency_s);
}

}  // extern "C"
