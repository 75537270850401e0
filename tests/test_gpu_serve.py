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
    # serving orders each job's queries as a single launch does (the
    # automatic choice), so a fused job's tiles are the same; a fused job is
    # the two-pass kernel's arithmetic (not the speculative single pass)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    ctx.set_tuning(q_per_lane=1, split_segments=0 if split else 1, speculate=0 if split else 1)
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
            tickets.append(aidw.aidw_server_submit(srv, j.spec()))
            time.sleep(0.0005)
        lat = []
        for t in tickets:
            st, js, l = aidw.aidw_server_wait(srv, t, 60.0)
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
        tickets = [aidw.aidw_server_submit(srv, j.spec()) for j in jobs]
        for t in tickets:
            st, js, _ = aidw.aidw_server_wait(srv, t, 60.0)
            assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
        # forgotten once done
        assert aidw.aidw_server_poll(srv, tickets[0])[0] == aidw.AIDW_ENOTFOUND
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
            aidw.aidw_server_submit(srv, bad)
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
        res = [aidw.aidw_server_wait(srv, aidw.aidw_server_submit(srv, j.spec()), 60.0)
               for j in jobs]
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
            aidw.aidw_server_submit(srv, spec)
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
            aidw.aidw_server_submit_batch(srv, bad)
        assert ei.value.status == aidw.AIDW_EINVAL
        assert "job 5" in aidw.last_error()
        st, stats = aidw.aidw_server_stats(srv)
        assert stats["submitted"] == 0
        tickets = aidw.aidw_server_submit_batch(srv, [j.spec() for j in jobs])
        assert len(set(tickets)) == len(jobs) and 0 not in tickets
        for t in tickets:
            st, js, _ = aidw.aidw_server_wait(srv, t, 60.0)
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
                t = aidw.aidw_server_submit(srv, j.spec())
                st, js, _ = aidw.aidw_server_wait(srv, t, 60.0)
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
            tickets.append(aidw.aidw_server_submit(srv, spec))
        lat = [aidw.aidw_server_wait(srv, t, 120.0) for t in tickets]
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


def _stream_data(spec):
    """Host arrays and device tensors of a serving data set spec (m, kind, seed)."""
    import torch

    x, y, z, area = workloads.dataset_arrays(spec)
    xy = torch.from_numpy(np.stack([x, y])).cuda()
    return (x, y, z, area), xy, torch.from_numpy(z.copy()).cuda()


def test_c5_sizes_two_streams_against_oracle(ctx, torch):
    """Serving at the full ranges of the serving workload (m log-uniform up to
    2^20, n up to 2^18, default segment length, tick quota and two streams):
    large split jobs span several ticks on both streams.  Sampled queries of
    every job match the oracle; a subset equals the same jobs served alone,
    bit for bit."""
    reqs, specs = workloads.serving_stream(count=48, rate=2000.0, seed=44)
    data = {}
    for r in reqs:
        if r.dataset not in data:
            data[r.dataset] = _stream_data(specs[r.dataset])
    jobs = []
    for r in reqs:
        qx, qy = workloads.request_queries(r)
        q = torch.from_numpy(np.stack([qx, qy])).cuda()
        out = torch.full((r.n,), float("nan"), device="cuda")
        (_, _, _, area), xy, z = data[r.dataset]
        jobs.append((r, qx, qy, q, out, aidw.make_job(q, r.k, out, data_xy=xy, data_z=z,
                                                       area=area)))
    torch.cuda.synchronize()
    print("c5: %d jobs, largest m %d, largest n %d" % (len(reqs), max(s[0] for s in specs),
                                                      max(r.n for r in reqs)), flush=True)
    srv = aidw.aidw_server_create(ctx.h, streams=2)
    try:
        t0 = time.perf_counter()
        tickets = []
        for r, *_, spec in jobs:
            delay = r.t_arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(aidw.aidw_server_submit(srv, spec))
        res = [aidw.aidw_server_wait(srv, t, 120.0) for t in tickets]
        st, stats = aidw.aidw_server_stats(srv)
    finally:
        aidw.aidw_server_destroy(srv)
    assert all(s == aidw.AIDW_OK and js == aidw.AIDW_OK for s, js, _ in res)
    assert st == aidw.AIDW_OK and stats["arena_in_use"] == 0
    n_split = sum(1 for r in reqs if specs[r.dataset][0] > 32768)
    print("c5: %d split jobs, %d ticks" % (n_split, stats["ticks"]), flush=True)
    assert n_split >= 10
    worst = 0.0
    for r, qx, qy, q, out, _ in jobs:
        (x, y, z, area), _, _ = data[r.dataset]
        idx = np.unique(np.linspace(0, r.n - 1, 3).astype(int))
        o = oracle.run(x, y, z, qx[idx], qy[idx], r.k, area=area)
        s = oracle.run(x, y, np.abs(z), qx[idx], qy[idx], r.k, area=area)
        e = rel_err(out.cpu().numpy()[idx], o, s).max()
        worst = max(worst, e)
        assert e <= TOL_F32, (r, e)
    print("c5: max rel err %.3e over sampled queries of every job" % worst, flush=True)
    # a subset, each job alone on a fresh server with the same options
    for r, qx, qy, q, out, spec in jobs[::8]:
        solo = torch.full((r.n,), float("nan"), device="cuda")
        spec.out = solo.data_ptr()
        srv = aidw.aidw_server_create(ctx.h, streams=2)
        try:
            st, js, _ = aidw.aidw_server_wait(srv, aidw.aidw_server_submit(srv, spec), 120.0)
        finally:
            aidw.aidw_server_destroy(srv)
        assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
        assert np.array_equal(solo.cpu().numpy(), out.cpu().numpy()), r


def test_fp64_and_knn_jobs_through_submit_and_poll(ctx, torch):
    """FP64 jobs (the plain FP64 kernel) and FP32-scaled jobs that ask for the
    neighbour indices go through the serving loop beside ordinary jobs: FP64
    within 1e-12 of the oracle with exact neighbour sets, FP32 equal to the
    same problem run alone."""
    insts64 = [workloads.uniform_small(m, n, 60 + i, k) for i, (m, n, k) in
               enumerate([(1024, 1024, 10), (3000, 200, 15), (20000, 130, 8), (64, 64, 32)])]
    insts32 = [workloads.uniform_unit(m, n, 70 + i, k) for i, (m, n, k) in
               enumerate([(5000, 300, 10), (50000, 700, 15), (40000, 90, 8)])]
    srv = aidw.aidw_server_create(ctx.h, arena_bytes=256 << 20, segment_points=SEG,
                                  tick_pair_evals=1e8)
    runs = []
    try:
        specs = []
        for inst in insts64 + insts32:
            d = aidw.to_device(inst)
            out = torch.full((inst.n,), float("nan"), dtype=d[0].dtype, device="cuda")
            r_obs = torch.empty(inst.n, dtype=torch.float64, device="cuda")
            al = torch.empty(inst.n, dtype=torch.float64, device="cuda")
            knn = torch.full((inst.n, inst.k), -1, dtype=torch.int32, device="cuda")
            specs.append(aidw.make_job(d[2], inst.k, out, inst.levels, inst.R_min, inst.R_max,
                                       data_xy=d[0], data_z=d[1], area=inst.area, r_obs=r_obs,
                                       alpha=al, knn_idx=knn))
            runs.append((inst, d, out, r_obs, al, knn))
        # ordinary split jobs in the same ticks
        extra = [Job(torch, workloads.clustered(30000, 500, 80 + i, 10)) for i in range(3)]
        tickets = aidw.aidw_server_submit_batch(srv, specs + [j.spec() for j in extra])
        for t in tickets:
            st, js, _ = aidw.aidw_server_wait(srv, t, 120.0)
            assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
    finally:
        aidw.aidw_server_destroy(srv)
    torch.cuda.synchronize()
    for inst, d, out, r_obs, al, knn in runs:
        want, w_robs, w_al, w_knn = oracle.run(inst.data_x, inst.data_y, inst.data_z,
                                               inst.query_x, inst.query_y, inst.k, inst.levels,
                                               inst.R_min, inst.R_max, inst.area, diag=True)
        if inst.dtype == np.float64:
            got = out.cpu().numpy()
            assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-12, inst.name
            assert np.array_equal(knn.cpu().numpy(), w_knn), inst.name
            assert np.allclose(r_obs.cpu().numpy(), w_robs, rtol=1e-14, atol=0)
        else:
            got, g_robs, g_al, g_knn = ctx.interpolate(*d, inst.k, inst.levels, inst.R_min,
                                                       inst.R_max, inst.area, diag=True)
            assert np.array_equal(out.cpu().numpy(), got.cpu().numpy()), inst.name
            assert np.array_equal(knn.cpu().numpy(), g_knn.cpu().numpy()), inst.name
            assert np.array_equal(r_obs.cpu().numpy(), g_robs.cpu().numpy()), inst.name
            assert np.array_equal(al.cpu().numpy(), g_al.cpu().numpy()), inst.name
    for j in extra:
        o, scale = ref(j.inst, np.arange(0, j.inst.n, 7))
        assert rel_err(j.out.cpu().numpy()[::7], o, scale).max() <= TOL_F32


def test_fp64_job_on_registered_dataset_is_rejected(ctx, torch):
    base = workloads.uniform_unit(1000, 10, 9, 10)
    data_xy, data_z, q = aidw.to_device(base)
    ds = aidw.aidw_dataset_register(ctx.h, data_xy.data_ptr(), data_z.data_ptr(), base.m,
                                    base.area)
    try:
        out = torch.empty(base.n, dtype=torch.float64, device="cuda")
        spec = aidw.make_job(q.double(), base.k, out, dataset=ds)
        with pytest.raises(aidw.AidwError) as ei:
            aidw.aidw_submit(ctx.h, spec)
        assert ei.value.status == aidw.AIDW_EINVAL
    finally:
        assert aidw.aidw_dataset_release(ctx.h, ds) == aidw.AIDW_OK


def test_handle_level_submit_poll_wait(torch):
    """aidw_submit / aidw_poll / aidw_wait on the handle's own serving loop,
    which aidw_destroy finishes."""
    insts = mixed(21, 10)
    c = aidw.Context(0)
    try:
        jobs = [Job(torch, i) for i in insts]
        tickets = aidw.aidw_submit_batch(c.h, [j.spec() for j in jobs[:5]])
        tickets += [aidw.aidw_submit(c.h, j.spec()) for j in jobs[5:]]
        for t in tickets[:-1]:
            st, js, _ = aidw.aidw_wait(c.h, t, 60.0)
            assert st == aidw.AIDW_OK and js == aidw.AIDW_OK
        while True:
            st, js, lat = aidw.aidw_poll(c.h, tickets[-1])
            if st != aidw.AIDW_EAGAIN:
                break
            time.sleep(0.001)
        assert st == aidw.AIDW_OK and js == aidw.AIDW_OK and lat > 0
        assert aidw.aidw_poll(c.h, tickets[0])[0] == aidw.AIDW_ENOTFOUND
        # a job left unpolled is finished by aidw_destroy
        late = Job(torch, insts[3])
        aidw.aidw_submit(c.h, late.spec())
    finally:
        c.close()
    torch.cuda.synchronize()
    for j in jobs + [late]:
        if j.inst.n:
            idx = np.unique(np.linspace(0, j.inst.n - 1, 5).astype(int))
            o, scale = ref(j.inst, idx)
            assert rel_err(j.out.cpu().numpy()[idx], o, scale).max() <= TOL_F32


def test_last_error_is_per_handle(torch):
    a, b = aidw.Context(0), aidw.Context(0)
    try:
        inst = workloads.uniform_unit(100, 10, 1, 5)
        d = aidw.to_device(inst)
        out = torch.empty(inst.n, device="cuda")
        p = a.problem(*d, inst.k, out, area=inst.area)
        p.k = 0
        assert aidw.aidw_interpolate_ex(a.h, p) == aidw.AIDW_EINVAL
        assert "k = 0" in aidw.last_error(a.h)
        assert aidw.last_error(b.h) == ""
        assert "k = 0" in aidw.last_error(None)
    finally:
        a.close()
        b.close()
