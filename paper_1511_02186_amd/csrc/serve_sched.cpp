// Scheduler of the AIDW serving loop (see serve_sched.h).
#include "serve_sched.h"

#include <algorithm>
#include <array>
#include <limits>

namespace aidw {
namespace serve {

// ---- Arena ----------------------------------------------------------------------

Arena::Arena(size_t size, size_t align) : size_(size), align_(align ? align : 1) {
    if (size_) free_[0] = size_;
}

bool Arena::alloc(size_t bytes, size_t* offset) {
    if (bytes == 0) bytes = 1;
    const size_t need = (bytes + align_ - 1) / align_ * align_;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < need) continue;
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > need) free_[off + need] = len - need;
        used_[off] = need;
        in_use_ += need;
        *offset = off;
        return true;
    }
    return false;
}

void Arena::free(size_t offset) {
    auto u = used_.find(offset);
    if (u == used_.end()) return;
    size_t off = u->first, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += len;
            return;
        }
    }
    free_[off] = len;
}

// ---- Scheduler --------------------------------------------------------------------

Scheduler::Scheduler(Executor* ex, const Config& cfg)
    : ex_(ex), cfg_(cfg), arena_(cfg.arena_bytes), slots_((size_t)std::max(1, cfg.slots)) {}

int64_t Scheduler::total_items(const Job& j, int phase) const {
    if (j.spec.segments <= 1) return phase == kFused ? j.tiles : 0;
    return phase == kFused ? 0 : j.tiles * j.spec.segments;
}

double Scheduler::item_cost(const Job& j, int phase) const {
    // distance evaluations of one item: 64 queries against m (both passes) or
    // against one segment (one pass), weighted by the job's relative cost
    if (phase == kFused) return 2.0 * 64.0 * (double)j.spec.m * j.spec.cost_scale;
    return 64.0 * (double)j.spec.seg_len * j.spec.cost_scale;
}

bool Scheduler::finished(const Job& j) const {
    if (j.spec.segments <= 1) return j.done[kFused] == j.tiles;
    return j.done[kSum] == total_items(j, kSum);
}

uint64_t Scheduler::submit(const JobSpec& spec) {
    const uint64_t t = next_ticket_++;
    Job& j = jobs_[t];
    j.spec = spec;
    if (j.spec.segments < 1) j.spec.segments = 1;
    if (j.spec.seg_len <= 0) j.spec.seg_len = j.spec.m;
    if (!(j.spec.cost_scale > 0.0)) j.spec.cost_scale = 1.0;
    j.tiles = (spec.n + 63) / 64;
    j.t_submit = ex_->now();
    j.remaining = 2.0 * (double)spec.m * (double)(j.tiles * 64) * j.spec.cost_scale;
    ++stats_.submitted;
    if (spec.ws_bytes > 0 && arena_.rounded(spec.ws_bytes) > arena_.size()) {
        j.state = JobState::Failed;
        j.status = -2;  // can never be admitted
        j.t_done = j.t_submit;
        ++stats_.failed;
        return t;
    }
    queue_.push_back(t);
    return t;
}

bool Scheduler::poll(uint64_t ticket, JobState* state, double* latency, int* status) const {
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return false;
    const Job& j = it->second;
    if (state) *state = j.state;
    if (j.state == JobState::Done || j.state == JobState::Failed) {
        if (latency) *latency = j.t_done - j.t_submit;
        if (status) *status = j.status;
    }
    return true;
}

void Scheduler::forget(uint64_t ticket) {
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return;
    if (it->second.state == JobState::Done || it->second.state == JobState::Failed)
        jobs_.erase(it);
}

void Scheduler::complete(uint64_t ticket, Job& j, int status) {
    if (j.state == JobState::Done || j.state == JobState::Failed) return;
    if (j.has_ws) {
        arena_.free(j.ws_offset);
        j.has_ws = false;
    }
    j.state = status == 0 ? JobState::Done : JobState::Failed;
    j.status = status;
    j.t_done = ex_->now();
    if (status == 0)
        ++stats_.completed;
    else
        ++stats_.failed;
    active_.erase(std::remove(active_.begin(), active_.end(), ticket), active_.end());
    ex_->retire(ticket, status);
}

void Scheduler::fail(uint64_t ticket, Job& j, int status) {
    if (j.state != JobState::Admitted && j.state != JobState::Queued) return;
    if (j.inflight > 0) {
        // kernels of earlier ticks may still touch its buffers and workspace
        if (!j.failing) j.fail_status = status;
        j.failing = true;
        return;
    }
    complete(ticket, j, status);
}

bool Scheduler::retire_ticks() {
    bool changed = false;
    for (size_t s = 0; s < slots_.size(); ++s) {
        InFlight& f = slots_[s];
        if (!f.busy || !ex_->done((int)s)) continue;
        f.busy = false;
        changed = true;
        stats_.pair_evals += f.pair_evals;
        for (auto& c : f.credits) {
            auto it = jobs_.find(c.first);
            if (it == jobs_.end()) continue;
            Job& j = it->second;
            if (j.inflight > 0) --j.inflight;
            if (j.state != JobState::Admitted) continue;
            if (j.failing) {
                if (j.inflight == 0) complete(c.first, j, j.fail_status);
                continue;
            }
            for (int p = 0; p < 3; ++p) j.done[p] += c.second[p];
            if (finished(j)) complete(c.first, j, 0);
        }
        f.credits.clear();
    }
    return changed;
}

bool Scheduler::admit_jobs() {
    bool changed = false;
    const double now = ex_->now();
    // The oldest queued job whose workspace does not fit blocks later
    // workspace jobs only once it has waited max_wait_s; jobs that need no
    // workspace always pass it.
    bool blocked = false, blocked_aged = false;
    for (auto it = queue_.begin(); it != queue_.end();) {
        const uint64_t t = *it;
        Job& j = jobs_[t];
        size_t off = 0;
        if (j.spec.ws_bytes > 0) {
            if (blocked && blocked_aged) {
                ++it;
                continue;
            }
            if (!arena_.alloc(j.spec.ws_bytes, &off)) {
                if (!blocked) {
                    blocked = true;
                    blocked_aged = now - j.t_submit > cfg_.max_wait_s;
                }
                ++it;
                continue;
            }
            j.has_ws = true;
            j.ws_offset = off;
        }
        it = queue_.erase(it);
        changed = true;
        j.state = JobState::Admitted;
        active_.push_back(t);
        const int rc = ex_->admit(t, off);
        if (rc != 0)
            complete(t, j, rc);
        else if (finished(j))
            complete(t, j, 0);
    }
    return changed;
}

bool Scheduler::build_tick(TickPlan* plan,
                           std::vector<std::pair<uint64_t, std::array<int64_t, 3>>>* credits) {
    const double now = ex_->now();
    struct Cand {
        uint64_t t;
        bool aged;
        double t_submit, remaining;
        int phase;
    };
    std::vector<Cand> cands;
    for (uint64_t t : active_) {
        Job& j = jobs_[t];
        if (j.failing) continue;
        int phase = -1;
        if (j.spec.segments <= 1) {
            if (j.issued[kFused] < total_items(j, kFused)) phase = kFused;
        } else if (j.issued[kKnn] < total_items(j, kKnn)) {
            phase = kKnn;
        } else if (j.done[kKnn] == total_items(j, kKnn) &&
                   j.issued[kSum] < total_items(j, kSum)) {
            phase = kSum;  // pass 2 only after every pass-1 item has completed
        }
        if (phase < 0) continue;
        cands.push_back({t, now - j.t_submit > cfg_.max_wait_s, j.t_submit, j.remaining, phase});
    }
    if (cands.empty()) return false;
    // Jobs that waited too long go first, oldest first; the rest shortest
    // remaining work first.
    std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) {
        if (a.aged != b.aged) return a.aged;
        if (a.aged) return a.t_submit < b.t_submit;
        if (a.remaining != b.remaining) return a.remaining < b.remaining;
        return a.t_submit < b.t_submit;
    });
    for (const Cand& c : cands) {
        if (!plan->items.empty() && plan->pair_evals >= cfg_.tick_pairs) break;
        Job& j = jobs_[c.t];
        const int64_t total = total_items(j, c.phase);
        const double cost = item_cost(j, c.phase);
        std::array<int64_t, 3> cnt{0, 0, 0};
        while (j.issued[c.phase] < total &&
               (plan->items.empty() || plan->pair_evals < cfg_.tick_pairs)) {
            const int64_t i = j.issued[c.phase]++;
            Item it;
            it.ticket = c.t;
            it.phase = c.phase;
            if (c.phase == kFused) {
                it.tile = (int)i;
                it.seg = 0;
            } else {
                it.seg = (int)(i / j.tiles);  // segment-major: neighbours share data
                it.tile = (int)(i % j.tiles);
            }
            plan->items.push_back(it);
            plan->pair_evals += cost;
            j.remaining -= cost;
            ++cnt[c.phase];
        }
        if (cnt[0] + cnt[1] + cnt[2] > 0) {
            plan->jobs.push_back(c.t);
            credits->push_back({c.t, cnt});
        }
    }
    return !plan->items.empty();
}

bool Scheduler::launch_ticks() {
    bool changed = false;
    for (size_t s = 0; s < slots_.size(); ++s) {
        InFlight& f = slots_[s];
        if (f.busy) continue;
        TickPlan plan;
        std::vector<std::pair<uint64_t, std::array<int64_t, 3>>> credits;
        if (!build_tick(&plan, &credits)) break;
        changed = true;
        const int rc = ex_->launch(plan, (int)s);
        if (rc != 0) {
            for (auto& c : credits) {
                auto it = jobs_.find(c.first);
                if (it != jobs_.end()) fail(c.first, it->second, rc);
            }
            continue;
        }
        for (auto& c : credits) {
            auto it = jobs_.find(c.first);
            if (it != jobs_.end()) ++it->second.inflight;
        }
        ++stats_.ticks;
        f.busy = true;
        f.credits = std::move(credits);
        f.pair_evals = plan.pair_evals;
    }
    return changed;
}

bool Scheduler::step() {
    bool changed = retire_ticks();
    changed |= admit_jobs();
    changed |= launch_ticks();
    return changed;
}

bool Scheduler::idle() const {
    if (!queue_.empty() || !active_.empty()) return false;
    for (const InFlight& f : slots_)
        if (f.busy) return false;
    return true;
}

Stats Scheduler::stats() const {
    Stats s = stats_;
    s.arena_in_use = arena_.in_use();
    s.queued = queue_.size();
    s.admitted = active_.size();
    return s;
}

}  // namespace serve
}  // namespace aidw
