"""The serving scheduler (paper_1511_02186_amd/csrc/serve_sched.cpp) on the CPU,
driven by a fake executor and a fake clock (tests/sched_harness.cpp): admission
under the workspace budget, tick quotas, ordering and aging, the pass-1 /
pass-2 dependency of split jobs, failures and a random stress run."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_02186_amd", "csrc")
QUEUED, ADMITTED, DONE, FAILED = 0, 1, 2, 3
FUSED, KNN, SUM = 0, 1, 2


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "sched_harness.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fPIC", "-shared", "-I" + CSRC,
                    os.path.join(CSRC, "serve_sched.cpp"),
                    os.path.join(ROOT, "tests", "sched_harness.cpp"), "-o", so], check=True)
    L = ctypes.CDLL(so)
    vp, u64, i64, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
    L.h_create.restype = vp
    L.h_create.argtypes = [dbl, ctypes.c_int, dbl, dbl, dbl]
    L.h_destroy.argtypes = [vp]
    L.h_submit.restype = u64
    L.h_submit.argtypes = [vp, i64, i64, ctypes.c_int, i64, dbl]
    for f in ["h_step", "h_idle", "h_launches", "h_max_issue", "h_issued_count"]:
        getattr(L, f).argtypes = [vp]
    L.h_advance.argtypes = [vp, dbl]
    L.h_now.restype = dbl
    L.h_now.argtypes = [vp]
    L.h_poison_admit.argtypes = [vp, u64]
    L.h_poison_launch.argtypes = [vp, u64]
    L.h_poison_launch_after.argtypes = [vp, u64, ctypes.c_int]
    L.h_submit_scaled.restype = u64
    L.h_submit_scaled.argtypes = [vp, i64, i64, dbl]
    L.h_poll.argtypes = [vp, u64, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int)]
    L.h_stats.argtypes = [vp, ctypes.POINTER(dbl)]
    L.h_launch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(dbl),
                           ctypes.POINTER(u64), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.h_launch_items.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64), ctypes.c_int]
    L.h_retired.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
    return L


class Sched:
    def __init__(self, L, arena=0, slots=1, tick_pairs=1e9, max_wait=10.0, rate=1e12):
        self.L = L
        self.h = L.h_create(float(arena), slots, float(tick_pairs), float(max_wait), float(rate))

    def close(self):
        self.L.h_destroy(self.h)

    def submit(self, m, n, segments=1, seg_len=0, ws=0):
        return self.L.h_submit(self.h, m, n, segments, seg_len or m, float(ws))

    def submit_scaled(self, m, n, cost_scale):
        return self.L.h_submit_scaled(self.h, m, n, float(cost_scale))

    def step(self):
        return self.L.h_step(self.h)

    def advance(self, dt):
        self.L.h_advance(self.h, dt)

    def poll(self, t):
        lat, st = ctypes.c_double(), ctypes.c_int()
        s = self.L.h_poll(self.h, t, ctypes.byref(lat), ctypes.byref(st))
        return s, lat.value, st.value

    def stats(self):
        out = (ctypes.c_double * 8)()
        self.L.h_stats(self.h, out)
        return dict(zip(["submitted", "completed", "failed", "ticks", "pair_evals", "arena",
                         "queued", "admitted"], list(out)))

    def launches(self):
        res = []
        for i in range(self.L.h_launches(self.h)):
            slot, nj = ctypes.c_int(), ctypes.c_int()
            times = (ctypes.c_double * 3)()
            jobs = (ctypes.c_uint64 * 256)()
            ni = self.L.h_launch(self.h, i, ctypes.byref(slot), times, jobs, 256, ctypes.byref(nj))
            rows = (ctypes.c_int64 * (4 * max(ni, 1)))()
            self.L.h_launch_items(self.h, i, rows, ni)
            items = np.array(rows[:4 * ni], dtype=np.int64).reshape(-1, 4)
            res.append(dict(slot=slot.value, start=times[0], finish=times[1], pairs=times[2],
                            jobs=list(jobs[:nj.value]), items=items))
        return res

    def run_until_idle(self, dt=1e-4, limit=100000):
        for _ in range(limit):
            self.step()
            if self.L.h_idle(self.h):
                return
            self.advance(dt)
        raise AssertionError("scheduler did not drain")


def test_fused_job_runs_and_reports_latency(lib):
    s = Sched(lib, rate=1e9)
    t = s.submit(m=1000, n=130)  # 3 tiles of 64 queries
    s.step()
    L = s.launches()
    assert len(L) == 1 and sorted(L[0]["items"][:, 2].tolist()) == [0, 1, 2]
    assert L[0]["pairs"] == pytest.approx(3 * 2 * 64 * 1000)
    assert s.poll(t)[0] == ADMITTED
    s.advance(L[0]["finish"] - L[0]["start"])
    s.step()
    state, lat, status = s.poll(t)
    assert state == DONE and status == 0
    assert lat == pytest.approx(3 * 2 * 64 * 1000 / 1e9)
    s.close()


def test_empty_job_completes_at_admission(lib):
    s = Sched(lib)
    t = s.submit(m=10, n=0)
    s.step()
    assert s.poll(t)[0] == DONE and not s.launches()
    s.close()


def test_fifo_admission_under_workspace_budget(lib):
    s = Sched(lib, arena=1000, rate=1e9)
    a = s.submit(m=100000, n=64, segments=4, seg_len=25000, ws=600)
    b = s.submit(m=100000, n=64, segments=4, seg_len=25000, ws=600)
    c = s.submit(m=100, n=64)  # needs no workspace: passes the blocked b
    s.step()
    assert [s.poll(x)[0] for x in (a, b, c)] == [ADMITTED, QUEUED, ADMITTED]
    assert s.stats()["arena"] == 768  # 600 rounded up to 256-byte blocks
    s.run_until_idle()
    assert all(s.poll(x)[0] == DONE for x in (a, b, c))
    assert s.stats()["arena"] == 0
    s.close()


def test_blocked_head_is_passed_only_until_it_has_aged(lib):
    # arena 1024: a holds 768; b (768) cannot fit; c (256) fits beside a
    s = Sched(lib, arena=1024, max_wait=1.0, rate=1e3)
    a = s.submit(m=100000, n=64, segments=4, seg_len=25000, ws=700)
    b = s.submit(m=100000, n=64, segments=4, seg_len=25000, ws=700)
    c = s.submit(m=100000, n=64, segments=4, seg_len=25000, ws=200)
    s.step()
    assert [s.poll(x)[0] for x in (a, b, c)] == [ADMITTED, QUEUED, ADMITTED]
    # once b has waited longer than max_wait, a small workspace job stays
    # behind it, while a job without workspace still passes
    s.advance(1.5)
    d = s.submit(m=100000, n=64, segments=4, seg_len=25000, ws=10)
    e = s.submit(m=100, n=64)
    s.step()
    assert [s.poll(x)[0] for x in (b, d, e)] == [QUEUED, QUEUED, ADMITTED]
    s.run_until_idle(dt=1.0)
    assert all(s.poll(x)[0] == DONE for x in (a, b, c, d, e))
    # d did not start before b
    L = s.launches()
    first = {t: min(i for i, x in enumerate(L) if t in x["jobs"]) for t in (b, d)}
    assert first[b] <= first[d]
    assert s.stats()["arena"] == 0
    s.close()


def test_cost_scale_weights_the_tick_quota(lib):
    quota = 4 * 2 * 64 * 1000
    s = Sched(lib, tick_pairs=quota, rate=1e9)
    t = s.submit_scaled(m=1000, n=64 * 8, cost_scale=2.0)  # each item costs twice
    s.run_until_idle()
    assert [len(x["items"]) for x in s.launches()] == [2, 2, 2, 2]
    assert s.poll(t)[0] == DONE
    s.close()


def test_failed_launch_completes_after_in_flight_ticks(lib):
    # the job's first tick runs on slot 0; its second launch (slot 1) fails
    # while the first is still in flight: the job is reported only after the
    # first tick has finished, and its workspace is held until then
    q = 64 * 1000
    s = Sched(lib, arena=1 << 20, slots=2, tick_pairs=q, rate=1e3)
    t = s.submit(m=4000, n=64 * 2, segments=4, seg_len=1000, ws=4096)
    lib.h_poison_launch_after(s.h, t, 1)
    s.step()
    assert len(s.launches()) == 1
    assert s.poll(t)[0] == ADMITTED and s.stats()["arena"] == 4096
    s.advance(0.5 * q / 1e3)
    s.step()
    assert s.poll(t)[0] == ADMITTED and s.stats()["arena"] == 4096
    s.advance(q / 1e3)
    s.step()
    state, _, status = s.poll(t)
    assert state == FAILED and status == -3 and s.stats()["arena"] == 0
    retired = ctypes.c_int()
    assert lib.h_retired(s.h, t, ctypes.byref(retired)) == 1 and retired.value == -3
    s.close()


def test_job_that_never_fits_fails_at_once(lib):
    s = Sched(lib, arena=1000)
    t = s.submit(m=10 ** 6, n=64, segments=10, seg_len=10 ** 5, ws=5000)
    state, _, status = s.poll(t)
    assert state == FAILED and status == -2
    other = s.submit(m=100, n=64)
    s.run_until_idle()
    assert s.poll(other)[0] == DONE
    s.close()


def test_tick_quota_is_soft_by_at_most_one_item(lib):
    quota = 5 * 2 * 64 * 1000
    s = Sched(lib, tick_pairs=quota, rate=1e9)
    t = s.submit(m=1000, n=64 * 23)
    s.run_until_idle()
    L = s.launches()
    assert sum(len(x["items"]) for x in L) == 23
    for x in L:
        assert x["pairs"] < quota + 2 * 64 * 1000
    assert [len(x["items"]) for x in L] == [5, 5, 5, 5, 3]
    assert s.poll(t)[0] == DONE
    s.close()


def test_shortest_remaining_first_and_aging(lib):
    s = Sched(lib, tick_pairs=2 * 64 * 10 ** 6, max_wait=1.0, rate=1e9)
    big = s.submit(m=10 ** 6, n=64 * 50)  # 50 items, one per tick
    s.step()  # first tick: big's first item
    small = s.submit(m=10 ** 6, n=64)
    s.advance(0.2)
    s.step()  # second tick: the small job jumps ahead
    L = s.launches()
    assert L[1]["jobs"] == [small]
    # an old job is served before newer, smaller ones
    s.advance(2.0)
    s.step()
    late_small = s.submit(m=10 ** 6, n=64)
    s.advance(0.2)
    s.step()
    L = s.launches()
    assert L[-1]["jobs"] == [big]
    s.run_until_idle(dt=0.05)
    assert all(s.poll(x)[0] == DONE for x in (big, small, late_small))
    s.close()


def test_split_job_runs_pass2_after_all_of_pass1(lib):
    s = Sched(lib, arena=10 ** 6, slots=2, tick_pairs=64 * 1000 * 3, rate=1e9)
    t = s.submit(m=4000, n=64 * 2, segments=4, seg_len=1000, ws=1000)
    s.run_until_idle()
    L = s.launches()
    phases = [set(x["items"][:, 1].tolist()) for x in L]
    first_sum = next(i for i, p in enumerate(phases) if SUM in p)
    knn_launches = [x for x in L if KNN in set(x["items"][:, 1].tolist())]
    # every pass-1 tick finished before the first pass-2 tick started
    assert max(x["finish"] for x in knn_launches) <= L[first_sum]["start"] + 1e-12
    items = np.concatenate([x["items"] for x in L])
    assert sorted(map(tuple, items[items[:, 1] == KNN][:, 2:].tolist())) == \
        [(tile, seg) for tile in range(2) for seg in range(4)]
    assert (items[:, 1] == SUM).sum() == 8
    assert s.poll(t)[0] == DONE
    s.close()


def test_failures_are_contained(lib):
    s = Sched(lib, rate=1e9)
    a = s.submit(m=1000, n=64)
    b = s.submit(m=1000, n=64)
    c = s.submit(m=1000, n=64)
    lib.h_poison_admit(s.h, b)
    s.run_until_idle()
    assert s.poll(a)[0] == DONE and s.poll(c)[0] == DONE
    state, _, status = s.poll(b)
    assert state == FAILED and status == -3
    st = s.stats()
    assert st["completed"] == 2 and st["failed"] == 1
    s.close()


def test_launch_failure_fails_only_that_ticks_jobs(lib):
    s = Sched(lib, tick_pairs=2 * 64 * 1000, rate=1e9)
    a = s.submit(m=1000, n=64)
    b = s.submit(m=1000, n=64)
    lib.h_poison_launch(s.h, a)
    s.run_until_idle()
    assert s.poll(a)[0] == FAILED and s.poll(b)[0] == DONE
    s.close()


def test_two_slots_overlap(lib):
    s = Sched(lib, slots=2, tick_pairs=2 * 64 * 1000, rate=1e9)
    s.submit(m=1000, n=64 * 4)
    s.step()
    L = s.launches()
    assert len(L) == 2 and {x["slot"] for x in L} == {0, 1}
    s.run_until_idle()
    s.close()


def test_random_stress_every_item_once_and_budget_returns(lib):
    rng = np.random.default_rng(0)
    s = Sched(lib, arena=1 << 20, slots=3, tick_pairs=5e8, max_wait=0.01, rate=1e11)
    tickets = []
    expect_items = 0
    for step in range(400):
        for _ in range(rng.poisson(0.7)):
            m = int(rng.integers(1, 300000))
            n = int(rng.integers(0, 3000))
            tiles = (n + 63) // 64
            if m > 32768 and n:
                seg = 32768
                segs = (m + seg - 1) // seg
                ws = int(rng.integers(1000, 300000))
                tickets.append(s.submit(m, n, segs, seg, ws))
                expect_items += 2 * tiles * segs
            else:
                tickets.append(s.submit(m, n))
                expect_items += tiles
        s.step()
        s.advance(float(rng.exponential(1e-3)))
    s.run_until_idle(dt=1e-3)
    assert all(s.poll(t)[0] == DONE for t in tickets)
    assert lib.h_max_issue(s.h) == 1
    assert lib.h_issued_count(s.h) == expect_items
    st = s.stats()
    assert st["arena"] == 0 and st["completed"] == len(tickets)
    s.close()


def test_scheduler_under_address_and_undefined_sanitizers():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "sched_stress")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-DSCHED_HARNESS_MAIN", "-I" + CSRC,
                    os.path.join(CSRC, "serve_sched.cpp"),
                    os.path.join(ROOT, "tests", "sched_harness.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
