// Test-only harness: the serving scheduler driven by a fake executor and a
// fake clock, exposed through a small C API for tests/test_serve_sched.py.
// Not part of libaidw.
#include <cstdint>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "serve_sched.h"

namespace sv = aidw::serve;

namespace {

struct Launch {
    int slot;
    double start, finish, pair_evals;
    std::vector<uint64_t> jobs;
    std::vector<sv::Item> items;
};

struct Fake : sv::Executor {
    double t = 0.0;
    double rate = 1e12;  // distance evaluations per fake second
    std::vector<double> finish;
    std::vector<bool> busy;
    std::set<uint64_t> poison_admit;
    std::map<uint64_t, int> poison_launch;  // ticket -> launches that still succeed
    std::map<uint64_t, int> launched;       // ticket -> successful launches so far
    std::vector<Launch> launches;
    std::map<uint64_t, int> retired;
    std::map<std::tuple<uint64_t, int, int, int>, int> issued;

    double now() override { return t; }
    int admit(uint64_t ticket, size_t) override { return poison_admit.count(ticket) ? -3 : 0; }
    int launch(const sv::TickPlan& plan, int slot) override {
        for (uint64_t j : plan.jobs) {
            auto p = poison_launch.find(j);
            if (p != poison_launch.end() && launched[j] >= p->second) return -3;
        }
        for (uint64_t j : plan.jobs) ++launched[j];
        Launch l{slot, t, t + plan.pair_evals / rate, plan.pair_evals, plan.jobs, plan.items};
        launches.push_back(l);
        finish[(size_t)slot] = l.finish;
        busy[(size_t)slot] = true;
        for (const sv::Item& it : plan.items) ++issued[{it.ticket, it.phase, it.tile, it.seg}];
        return 0;
    }
    bool done(int slot) override {
        if (!busy[(size_t)slot]) return true;
        if (t + 1e-12 < finish[(size_t)slot]) return false;
        busy[(size_t)slot] = false;
        return true;
    }
    void retire(uint64_t ticket, int status) override { retired[ticket] = status; }
};

struct Harness {
    Fake ex;
    sv::Scheduler* s;
};

}  // namespace

extern "C" {

void* h_create(double arena, int slots, double tick_pairs, double max_wait, double rate) {
    Harness* h = new Harness;
    h->ex.rate = rate;
    h->ex.finish.assign((size_t)slots, 0.0);
    h->ex.busy.assign((size_t)slots, false);
    sv::Config c;
    c.arena_bytes = (size_t)arena;
    c.slots = slots;
    c.tick_pairs = tick_pairs;
    c.max_wait_s = max_wait;
    h->s = new sv::Scheduler(&h->ex, c);
    return h;
}

void h_destroy(void* p) {
    Harness* h = static_cast<Harness*>(p);
    delete h->s;
    delete h;
}

uint64_t h_submit(void* p, int64_t m, int64_t n, int segments, int64_t seg_len, double ws) {
    sv::JobSpec s;
    s.m = m;
    s.n = n;
    s.segments = segments;
    s.seg_len = seg_len;
    s.ws_bytes = (size_t)ws;
    return static_cast<Harness*>(p)->s->submit(s);
}

uint64_t h_submit_scaled(void* p, int64_t m, int64_t n, double cost_scale) {
    sv::JobSpec s;
    s.m = m;
    s.n = n;
    s.cost_scale = cost_scale;
    return static_cast<Harness*>(p)->s->submit(s);
}

int h_step(void* p) { return static_cast<Harness*>(p)->s->step() ? 1 : 0; }
int h_idle(void* p) { return static_cast<Harness*>(p)->s->idle() ? 1 : 0; }
void h_advance(void* p, double dt) { static_cast<Harness*>(p)->ex.t += dt; }
double h_now(void* p) { return static_cast<Harness*>(p)->ex.t; }
void h_poison_admit(void* p, uint64_t t) { static_cast<Harness*>(p)->ex.poison_admit.insert(t); }
void h_poison_launch(void* p, uint64_t t) { static_cast<Harness*>(p)->ex.poison_launch[t] = 0; }
// Launches carrying job t fail once `ok` of them have succeeded.
void h_poison_launch_after(void* p, uint64_t t, int ok) {
    static_cast<Harness*>(p)->ex.poison_launch[t] = ok;
}

// state: 0 queued, 1 admitted, 2 done, 3 failed, -1 unknown
int h_poll(void* p, uint64_t t, double* latency, int* status) {
    sv::JobState st;
    if (!static_cast<Harness*>(p)->s->poll(t, &st, latency, status)) return -1;
    return (int)st;
}

void h_stats(void* p, double* out) {
    const sv::Stats s = static_cast<Harness*>(p)->s->stats();
    out[0] = (double)s.submitted;
    out[1] = (double)s.completed;
    out[2] = (double)s.failed;
    out[3] = (double)s.ticks;
    out[4] = s.pair_evals;
    out[5] = (double)s.arena_in_use;
    out[6] = (double)s.queued;
    out[7] = (double)s.admitted;
}

int h_launches(void* p) { return (int)static_cast<Harness*>(p)->ex.launches.size(); }

// Launch i: returns its item count; fills slot, start, finish, pair evals and
// up to cap job tickets.
int h_launch(void* p, int i, int* slot, double* times, uint64_t* jobs, int cap, int* njobs) {
    const Launch& l = static_cast<Harness*>(p)->ex.launches[(size_t)i];
    *slot = l.slot;
    times[0] = l.start;
    times[1] = l.finish;
    times[2] = l.pair_evals;
    *njobs = (int)l.jobs.size();
    for (int j = 0; j < cap && j < (int)l.jobs.size(); ++j) jobs[j] = l.jobs[(size_t)j];
    return (int)l.items.size();
}

// Items of launch i as (ticket, phase, tile, seg) rows.
int h_launch_items(void* p, int i, int64_t* rows, int cap) {
    const Launch& l = static_cast<Harness*>(p)->ex.launches[(size_t)i];
    int k = 0;
    for (const sv::Item& it : l.items) {
        if (k >= cap) break;
        rows[4 * k + 0] = (int64_t)it.ticket;
        rows[4 * k + 1] = it.phase;
        rows[4 * k + 2] = it.tile;
        rows[4 * k + 3] = it.seg;
        ++k;
    }
    return k;
}

// Largest number of times any (ticket, phase, tile, seg) item was issued.
int h_max_issue(void* p) {
    int mx = 0;
    for (auto& kv : static_cast<Harness*>(p)->ex.issued) mx = kv.second > mx ? kv.second : mx;
    return mx;
}

int h_issued_count(void* p) { return (int)static_cast<Harness*>(p)->ex.issued.size(); }

int h_retired(void* p, uint64_t t, int* status) {
    auto& r = static_cast<Harness*>(p)->ex.retired;
    auto it = r.find(t);
    if (it == r.end()) return 0;
    *status = it->second;
    return 1;
}

}  // extern "C"

#ifdef SCHED_HARNESS_MAIN
// Stand-alone random stress of the scheduler for sanitizer builds.
#include <cstdio>
#include <random>

int main() {
    void* h = h_create(1 << 20, 3, 5e8, 0.01, 1e11);
    std::mt19937_64 rng(7);
    std::vector<uint64_t> tickets;
    for (int step = 0; step < 2000; ++step) {
        const int arrivals = (int)(rng() % 3);
        for (int a = 0; a < arrivals; ++a) {
            const int64_t m = 1 + (int64_t)(rng() % 300000);
            const int64_t n = (int64_t)(rng() % 3000);
            if (m > 32768 && n)
                tickets.push_back(h_submit(h, m, n, (int)((m + 32767) / 32768), 32768,
                                           (double)(1000 + rng() % 300000)));
            else
                tickets.push_back(h_submit(h, m, n, 1, m, 0.0));
        }
        h_step(h);
        h_advance(h, 1e-3 * (double)(rng() % 3));
    }
    for (int i = 0; i < 1000000 && !h_idle(h); ++i) {
        h_step(h);
        h_advance(h, 1e-3);
    }
    int bad = !h_idle(h) || h_max_issue(h) != 1;
    for (uint64_t t : tickets) {
        double lat;
        int status;
        if (h_poll(h, t, &lat, &status) != 2) bad = 1;
    }
    double st[8];
    h_stats(h, st);
    if (st[5] != 0.0) bad = 1;
    h_destroy(h);
    std::printf("%s: %zu jobs\n", bad ? "FAIL" : "ok", tickets.size());
    return bad;
}
#endif
