"""The serving loop on the GPU: jobs of mixed sizes submitted while others run,
registered data sets, admission under the workspace budget, concurrent
submitters.  Every job's result equals the same problem run alone (bitwise for
unsplit jobs, to rounding for split ones) and matches the FP64 oracle."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1511_02186_amd import aidw, workloads

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-4
SEG = 8192  # points per segment in these tests, so that mid-size jobs split


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = aidw.Context(0)
    yield c
    c.close()


def rel_err(got, want, scale):
    diff = np.abs(np.asarray(got, dtype=np.float64) - want)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(scale > 0, diff / scale, np.where(diff == 0, 0.0, np.inf))


def ref(inst, idx):
    a = (inst.data_x, inst.data_y)
    kw = dict(alpha_levels=inst.levels, R_min=inst.R_min, R_max=inst.R_max, area=inst.area)
    out = oracle.run(*a, inst.data_z, inst.query_x[idx], inst.query_y[idx], inst.k, **kw)
    scale = oracle.run(*a, np.abs(inst.data_z), inst.query_x[idx], inst.query_y[idx], inst.k,
                       **kw)
    return out, scale


def alone(ctx, torch, inst, split):
    data_xy, data_z, query_xy = aidw.to_device(inst)
    ctx.set_tuning(q_per_lane=1, split_segments=0 if split else 1)
    try:
        r = ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min,
                            inst.R_max, inst.area)
    finally:
        ctx.set_tuning()
    torch.cuda.synchronize()
    return r.cpu().numpy()


class Job:
    def __init__(self, torch, inst, dataset=0):
        self.inst = inst
        self.data_xy, self.data_z, self.query_xy = aidw.to_device(inst)
        self.out = torch.full((inst.n,), float("nan"), device="cuda")
        self.dataset = dataset

    def spec(self):
        i = self.inst
        if self.dataset:
            return aidw.make_job(self.query_xy, i.k, self.out, i.levels, i.R_min, i.R_max,
                                 dataset=self.dataset)
        return aidw.make_job(self.query_xy, i.k, self.out, i.levels, i.R_min, i.R_max,
                             data_xy=self.data_xy, data_z=self.data_z, area=i.area)


def mixed(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(np.exp(rng.uniform(np.log(50), np.log(60000))))
        n = int(np.exp(rng.uniform(np.log(1), np.log(3000)))) if i % 9 else 0
        k = min(m, int(rng.choice([1, 8, 10, 15, 32])))
        if rng.uniform() < 0.5:
            inst = workloads.uniform_unit(m, n, 500 + i, k)
        else:
            inst = workloads.clustered(m, n, 500 + i, k, on_point=0.05)
        if inst.area <= 0:
            inst.area = 1.0
        out.append(inst)
    return out


def test_jobs_in_a_mix_equal_jobs_alone(ctx, torch):
    insts = mixed(1, 40)
    jobs = [Job(torch, i) for i in insts]
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=256 << 20, streams=2,
                                  tick_pair_evals=2e8, segment_points=SEG)
    try:
        tickets = []
        for j in jobs:  # arrivals spread while earlier jobs run
            tickets.append(aidw.aidw_submit(srv, j.spec()))
            time.sleep(0.0005)
        lat = []
        for t in tickets:
            st, js, l = aidw.aidw_wait(srv, t, 60.0)
            assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
            lat.append(l)
        st, stats = aidw.aidw_server_stats(srv)
        assert st == aidw.AIDW_OK and stats["completed"] == len(jobs) and stats["failed"] == 0
        assert stats["arena_in_use"] == 0
        print("serve mix: %d jobs, %d ticks, p50 %.2f ms, max %.2f ms"
              % (len(jobs), stats["ticks"], 1e3 * np.median(lat), 1e3 * max(lat)), flush=True)
    finally:
        aidw.aidw_server_destroy(srv)
    torch.cuda.synchronize()
    for j in jobs:
        i = j.inst
        if i.n == 0:
            continue
        got = j.out.cpu().numpy()
        idx = np.unique(np.linspace(0, i.n - 1, 7).astype(int))
        o, scale = ref(i, idx)
        assert rel_err(got[idx], o, scale).max() <= TOL_F32, i.name
        split = i.m > SEG
        solo = alone(ctx, torch, i, split)
        if split:  # other segment boundaries: the same up to rounding of the FP64 sums
            assert rel_err(got, solo, np.abs(solo) + 1e-30).max() <= 1e-6, i.name
        else:
            assert np.array_equal(got, solo), i.name


def test_registered_datasets(ctx, torch):
    base = workloads.uniform_unit(30000, 10, 9, 10)
    data_xy, data_z, _ = aidw.to_device(base)
    ds = aidw.aidw_dataset_register(ctx.h, data_xy.data_ptr(), data_z.data_ptr(), base.m,
                                    base.area)
    del data_xy, data_z  # the library keeps its own copy
    torch.cuda.empty_cache()
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=64 << 20, segment_points=SEG)
    try:
        jobs = []
        for s in range(4):
            inst = workloads.uniform_unit(30000, 200 + 50 * s, 9, 10)  # same data, other queries
            rng = np.random.default_rng(s)
            inst.query_x[:] = rng.uniform(0, 1, inst.n).astype(np.float32)
            inst.query_y[:] = rng.uniform(0, 1, inst.n).astype(np.float32)
            jobs.append(Job(torch, inst, dataset=ds))
        tickets = [aidw.aidw_submit(srv, j.spec()) for j in jobs]
        for t in tickets:
            st, js, _ = aidw.aidw_wait(srv, t, 60.0)
            assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
        assert aidw.aidw_poll(srv, tickets[0])[0] == aidw.AIDW_ENOTFOUND  # forgotten once done
    finally:
        aidw.aidw_server_destroy(srv)
    for j in jobs:
        o, scale = ref(j.inst, np.arange(j.inst.n))
        assert rel_err(j.out.cpu().numpy(), o, scale).max() <= TOL_F32
    assert aidw.aidw_dataset_release(ctx.h, ds) == aidw.AIDW_OK
    assert aidw.aidw_dataset_release(ctx.h, ds) == aidw.AIDW_ENOTFOUND
    bad = aidw.aidw_job()
    bad.dataset = ds
    srv = aidw.aidw_server_create(ctx.h)
    try:
        with pytest.raises(aidw.AidwError) as ei:
            aidw.aidw_submit(srv, bad)
        assert ei.value.status == aidw.AIDW_ENOTFOUND
    finally:
        aidw.aidw_server_destroy(srv)


def test_workspace_budget(ctx, torch):
    small = workloads.uniform_unit(20000, 100, 3, 8)      # split: needs a little workspace
    big = workloads.uniform_unit(20000, 60000, 4, 8)      # split: needs more than the arena
    fused = workloads.uniform_unit(3000, 500, 5, 8)        # no workspace
    jobs = [Job(torch, small), Job(torch, big), Job(torch, fused)]
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=1 << 20, segment_points=SEG)
    try:
        res = [aidw.aidw_wait(srv, aidw.aidw_submit(srv, j.spec()), 60.0) for j in jobs]
    finally:
        aidw.aidw_server_destroy(srv)
    assert res[0][:2] == (aidw.AIDW_OK, aidw.AIDW_OK)
    assert res[1][:2] == (aidw.AIDW_OK, aidw.AIDW_ENOMEM)
    assert res[2][:2] == (aidw.AIDW_OK, aidw.AIDW_OK)
    assert np.all(np.isnan(jobs[1].out.cpu().numpy()))  # a failed job writes nothing
    for j in (jobs[0], jobs[2]):
        o, scale = ref(j.inst, np.arange(0, j.inst.n, 5))
        assert rel_err(j.out.cpu().numpy()[::5], o, scale).max() <= TOL_F32


def test_invalid_job_is_rejected_at_submit(ctx, torch):
    inst = workloads.uniform_unit(100, 10, 1, 5)
    j = Job(torch, inst)
    spec = j.spec()
    spec.k = 200
    srv = aidw.aidw_server_create(ctx.h)
    try:
        with pytest.raises(aidw.AidwError) as ei:
            aidw.aidw_submit(srv, spec)
        assert ei.value.status == aidw.AIDW_EINVAL
    finally:
        aidw.aidw_server_destroy(srv)


def test_submit_batch_all_or_nothing(ctx, torch):
    insts = mixed(11, 12)
    jobs = [Job(torch, i) for i in insts]
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=256 << 20, segment_points=SEG)
    try:
        bad = [j.spec() for j in jobs]
        bad[5].k = 0  # invalid: nothing may be enqueued
        with pytest.raises(aidw.AidwError) as ei:
            aidw.aidw_submit_batch(srv, bad)
        assert ei.value.status == aidw.AIDW_EINVAL
        assert "job 5" in aidw.last_error()
        st, stats = aidw.aidw_server_stats(srv)
        assert stats["submitted"] == 0
        tickets = aidw.aidw_submit_batch(srv, [j.spec() for j in jobs])
        assert len(set(tickets)) == len(jobs) and 0 not in tickets
        for t in tickets:
            st, js, _ = aidw.aidw_wait(srv, t, 60.0)
            assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
    finally:
        aidw.aidw_server_destroy(srv)
    torch.cuda.synchronize()
    for j in jobs:
        i = j.inst
        if i.n == 0:
            continue
        solo = alone(ctx, torch, i, i.m > SEG)
        got = j.out.cpu().numpy()
        if i.m > SEG:
            assert rel_err(got, solo, np.abs(solo) + 1e-30).max() <= 1e-6, i.name
        else:
            assert np.array_equal(got, solo), i.name


def test_concurrent_submitters(ctx, torch):
    insts = mixed(7, 24)
    jobs = [Job(torch, i) for i in insts]
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=256 << 20, segment_points=SEG)
    errors = []

    def client(part):
        try:
            for j in part:
                t = aidw.aidw_submit(srv, j.spec())
                st, js, _ = aidw.aidw_wait(srv, t, 60.0)
                if st != aidw.AIDW_OK or js != aidw.AIDW_OK:
                    errors.append((st, js))
        except Exception as e:  # pragma: no cover
            errors.append(e)

    threads = [threading.Thread(target=client, args=(jobs[i::4],)) for i in range(4)]
    try:
        for t in threads:
            t.start()
        for t in threads:
            t.join()
    finally:
        aidw.aidw_server_destroy(srv)
    assert not errors
    for j in jobs:
        if j.inst.n:
            idx = np.unique(np.linspace(0, j.inst.n - 1, 5).astype(int))
            o, scale = ref(j.inst, idx)
            assert rel_err(j.out.cpu().numpy()[idx], o, scale).max() <= TOL_F32


def test_poisson_stream_latency(ctx, torch):
    reqs, specs = workloads.serving_stream(count=120, rate=2000.0, seed=4,
                                           m_range=(4096, 1 << 17), n_range=(256, 1 << 14))
    gen = torch.Generator(device="cuda").manual_seed(4)
    datasets = {}
    for i, (m, _, _) in enumerate(specs):
        xy = torch.rand((2, m), device="cuda", generator=gen)
        z = torch.sin(4 * xy[0]) * torch.cos(3 * xy[1])
        datasets[i] = (xy, z.contiguous())
    jobs = []
    for r in reqs:
        xy, z = datasets[r.dataset]
        q = torch.rand((2, r.n), device="cuda", generator=gen)
        out = torch.full((r.n,), float("nan"), device="cuda")
        jobs.append((r, q, out, aidw.make_job(q, r.k, out, data_xy=xy, data_z=z, area=1.0)))
    torch.cuda.synchronize()
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=2 << 30)
    try:
        t0 = time.perf_counter()
        tickets = []
        for r, _, _, spec in jobs:
            delay = r.t_arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(aidw.aidw_submit(srv, spec))
        lat = [aidw.aidw_wait(srv, t, 120.0) for t in tickets]
        wall = time.perf_counter() - t0
    finally:
        aidw.aidw_server_destroy(srv)
    assert all(st == aidw.AIDW_OK and js == aidw.AIDW_OK for st, js, _ in lat)
    ms = np.array([l for _, _, l in lat]) * 1e3
    pairs = sum(2.0 * specs[r.dataset][0] * r.n for r in reqs)
    print("poisson: %d jobs in %.2f s, p50 %.2f ms, p99 %.2f ms, %.3e pair-evals/s"
          % (len(reqs), wall, np.percentile(ms, 50), np.percentile(ms, 99), pairs / wall),
          flush=True)
    for (r, q, out, _) in jobs[::15]:
        xy, z = datasets[r.dataset]
        idx = np.arange(0, r.n, max(1, r.n // 5))
        X, Z, Q = xy.cpu().numpy(), z.cpu().numpy(), q.cpu().numpy()
        o = oracle.run(X[0], X[1], Z, Q[0][idx], Q[1][idx], r.k, area=1.0)
        s = oracle.run(X[0], X[1], np.abs(Z), Q[0][idx], Q[1][idx], r.k, area=1.0)
        assert rel_err(out.cpu().numpy()[idx], o, s).max() <= TOL_F32
