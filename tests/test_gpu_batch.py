"""Batched launches (many independent problems, one launch, graph
replay) and the split-m path for problems with few queries.  All results are
checked against the FP64 oracle, and batched results against the same
problems run alone."""
import numpy as np
import pytest

import oracle
from paper_1511_02186_amd import aidw, workloads

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = aidw.Context(0)
    yield c
    c.close()


def say(msg):
    print(msg, flush=True)


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


class Dev:
    """Device copies of one instance plus its output buffer."""

    def __init__(self, torch, inst):
        self.inst = inst
        self.data_xy, self.data_z, self.query_xy = aidw.to_device(inst)
        self.out = torch.full((inst.n,), float("nan"), device="cuda")

    def problem(self, ctx):
        i = self.inst
        return ctx.problem(self.data_xy, self.data_z, self.query_xy, i.k, self.out, i.levels,
                           i.R_min, i.R_max, i.area)


def mixed_instances(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rng.integers(1, 9000))
        n = int(rng.integers(0, 700))
        k = int(rng.choice([1, 8, 10, 15, 32]))
        k = min(k, m)
        if rng.uniform() < 0.5:
            inst = workloads.uniform_unit(m, n, 1000 + i, k)
        else:
            inst = workloads.clustered(m, n, 1000 + i, k, on_point=0.05)
        if inst.area <= 0:
            inst.area = 1.0
        out.append(inst)
    return out


def run_alone(ctx, torch, dev):
    # the unsplit two-pass kernel (a batch item's arithmetic; the speculative
    # single pass agrees with it to rounding)
    ctx.set_tuning(q_per_lane=1, split_segments=1, speculate=1)
    try:
        i = dev.inst
        r = ctx.interpolate(dev.data_xy, dev.data_z, dev.query_xy, i.k, i.levels, i.R_min,
                            i.R_max, i.area)
    finally:
        ctx.set_tuning()
    torch.cuda.synchronize()
    return r.cpu().numpy()


def test_batch_is_bitwise_equal_to_problems_alone(ctx, torch):
    insts = mixed_instances(24, 1)
    devs = [Dev(torch, i) for i in insts]
    ctx.bind_current_stream()
    aidw.check(aidw.aidw_interpolate_batch(ctx.h, [d.problem(ctx) for d in devs]))
    torch.cuda.synchronize()
    for d in devs:
        got = d.out.cpu().numpy()
        alone = run_alone(ctx, torch, d)
        assert np.array_equal(got, alone), d.inst.name
        if d.inst.n:
            idx = np.unique(np.linspace(0, d.inst.n - 1, 9).astype(int))
            o, scale = ref(d.inst, idx)
            assert rel_err(got[idx], o, scale).max() <= TOL_F32, d.inst.name


def test_graph_replays_follow_input_changes(ctx, torch):
    insts = mixed_instances(10, 2)
    devs = [Dev(torch, i) for i in insts]
    ctx.bind_current_stream()
    b = aidw.aidw_batch_create(ctx.h, [d.problem(ctx) for d in devs])
    try:
        rng = np.random.default_rng(0)
        for replay in range(3):
            # eager work between replays: new query positions in place
            for d in devs:
                if d.inst.n:
                    d.inst.query_x[:] = rng.uniform(0, 1, d.inst.n).astype(np.float32)
                    d.inst.query_y[:] = rng.uniform(0, 1, d.inst.n).astype(np.float32)
                    d.query_xy.copy_(torch.from_numpy(d.inst.query_xy()))
                d.out.fill_(float("nan"))
            torch.cuda.synchronize()
            aidw.check(aidw.aidw_batch_launch(b))
            for d in devs:
                got = d.out.cpu().numpy()
                assert np.array_equal(got, run_alone(ctx, torch, d)), (replay, d.inst.name)
    finally:
        aidw.aidw_batch_destroy(b)


def test_batch_argument_errors(ctx, torch):
    inst = workloads.uniform_unit(500, 100, 3, 8)
    d = Dev(torch, inst)
    good = d.problem(ctx)
    bad = d.problem(ctx)
    bad.k = 0
    st = aidw.aidw_interpolate_batch(ctx.h, [good, good, bad])
    assert st == aidw.AIDW_EINVAL and "problem 2" in aidw.last_error()
    knn = torch.empty((inst.n, inst.k), dtype=torch.int32, device="cuda")
    with_knn = d.problem(ctx)
    with_knn.knn_idx = knn.data_ptr()
    assert aidw.aidw_interpolate_batch(ctx.h, [with_knn]) == aidw.AIDW_EINVAL
    inst64 = workloads.uniform_unit(500, 100, 3, 8, dtype=np.float64)
    d64 = Dev(torch, inst64)
    d64.out = torch.empty(inst64.n, dtype=torch.float64, device="cuda")
    assert aidw.aidw_interpolate_batch(ctx.h, [d64.problem(ctx)]) == aidw.AIDW_EINVAL
    assert aidw.aidw_interpolate_batch(ctx.h, []) == aidw.AIDW_OK


def test_batched_config_512_instances(ctx, torch):
    insts = workloads.batched()  # 512 problems, m in [1024, 65536], n in [1024, 32768]
    pairs = sum(i.pair_evals() for i in insts)
    say("batched: %d problems, %.3e pair evaluations" % (len(insts), pairs))
    devs = [Dev(torch, i) for i in insts]
    ctx.bind_current_stream()
    b = aidw.aidw_batch_create(ctx.h, [d.problem(ctx) for d in devs])
    try:
        aidw.check(aidw.aidw_batch_launch(b))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        aidw.check(aidw.aidw_batch_launch(b, aidw.AIDW_FLAG_ASYNC))
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        say("batched: %.2f ms, %.3e pair-evals/s" % (ms, pairs / (ms * 1e-3)))
    finally:
        aidw.aidw_batch_destroy(b)
    rng = np.random.default_rng(5)
    worst = 0.0
    for d in devs:
        got = d.out.cpu().numpy()
        assert not np.isnan(got).any(), d.inst.name  # every query written (NaN before)
        idx = np.sort(rng.choice(d.inst.n, 3, replace=False))
        o, scale = ref(d.inst, idx)
        worst = max(worst, rel_err(got[idx], o, scale).max())
    say("batched: max err %.3e over %d sampled queries" % (worst, 3 * len(devs)))
    assert worst <= TOL_F32
    for d in devs[::64]:
        assert np.array_equal(d.out.cpu().numpy(), run_alone(ctx, torch, d)), d.inst.name


# ---- split-m ---------------------------------------------------------------

def _run(ctx, torch, inst, segments=0, diag=False, query_order=0, speculate=0):
    data_xy, data_z, query_xy = aidw.to_device(inst)
    ctx.set_tuning(split_segments=segments, speculate=speculate, query_order=query_order)
    try:
        # no knn_idx: asking for the indices would keep m unsplit
        r = ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min,
                            inst.R_max, inst.area, diag=diag, knn=False)
    finally:
        ctx.set_tuning()
    torch.cuda.synchronize()
    return tuple(None if t is None else t.cpu().numpy() for t in r) if diag else r.cpu().numpy()


@pytest.mark.parametrize("segments", [2, 7, 64, 1000])
@pytest.mark.parametrize("k", [1, 10, 15, 32])
def test_split_matches_unsplit_and_oracle(ctx, torch, segments, k):
    inst = workloads.clustered(m=50003, n=700, seed=segments + k, k=k, on_point=0.03)
    # in the caller's order, where split pass 2 keeps the pass-1 tiles (and a
    # query its wave mates, so its pass-2 loop), against the two-pass kernel
    # (in the speculative single pass a query that ends at alpha_5 keeps its
    # whole-power sums whatever its wave mates do)
    whole, r0, a0, _ = _run(ctx, torch, inst, segments=1, diag=True, query_order=1, speculate=1)
    split, r1, a1, _ = _run(ctx, torch, inst, segments=segments, diag=True, query_order=1,
                            speculate=1)
    assert np.array_equal(r0, r1)  # same k nearest distances, same order of summation
    assert np.array_equal(a0, a1)
    assert np.allclose(split, whole, rtol=2e-7, atol=0)
    idx = np.arange(0, inst.n, 11)
    o, scale = ref(inst, idx)
    assert rel_err(split[idx], o, scale).max() <= TOL_F32


@pytest.mark.parametrize("levels", [(1, 2, 3, 4, 5), (1, 2, 3, 4, 4.5), (2, 2, 2, 2, 2)])
def test_split_pass2_regrouped_by_loop(ctx, torch, levels):
    # split pass 2 regroups the positions by the loop they take (whole power,
    # unscaled or not; exp2/log2; on a data point): every query is computed
    # once, r_obs and alpha are untouched, and the outputs agree with the
    # pass-1 tiles' (query_order = 1) to rounding and with the oracle
    inst = workloads.clustered(m=60013, n=3001, seed=71, k=10, on_point=0.02)
    inst.levels = levels
    o1, r1, a1, _ = _run(ctx, torch, inst, segments=6, diag=True)
    o0, r0, a0, _ = _run(ctx, torch, inst, segments=6, diag=True, query_order=1)
    assert not np.isnan(o1).any()
    assert np.array_equal(r0, r1) and np.array_equal(a0, a1)
    assert np.allclose(o1, o0, rtol=1e-5, atol=1e-6 * np.abs(o0).max())
    idx = np.unique(np.linspace(0, inst.n - 1, 40).astype(int))
    o, scale = ref(inst, idx)
    assert rel_err(o1[idx], o, scale).max() <= TOL_F32
    on = np.asarray(inst.meta["on_point_queries"][:20])
    o, scale = ref(inst, on)
    assert rel_err(o1[on], o, scale).max() <= TOL_F32
    for qo, named in ((0, True), (1, False)):
        ctx.set_tuning(split_segments=6, query_order=qo)
        try:
            plan = _plan(ctx, torch, inst, inst.n, levels)
        finally:
            ctx.set_tuning()
        assert ("pass 2 regrouped by loop" in plan) == named, plan
        assert "aidw_f32_wsum_part" in plan


@pytest.mark.parametrize("m,n", [(4096, 1), (300000, 64), (1 << 20, 256), (65536, 5000)])
def test_automatic_split_for_few_queries(ctx, torch, m, n):
    inst = workloads.paper_scale(m=m, n=n, seed=m % 97 + n, k=15)
    out = _run(ctx, torch, inst)
    idx = np.unique(np.linspace(0, n - 1, min(n, 24)).astype(int))
    o, scale = ref(inst, idx)
    assert rel_err(out[idx], o, scale).max() <= TOL_F32


def _plan(ctx, torch, inst, n, levels):
    data_xy, data_z, query_xy = aidw.to_device(inst)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    p = ctx.problem(data_xy, data_z, query_xy[:, :n].contiguous(), inst.k, out, levels,
                    inst.R_min, inst.R_max, inst.area)
    return aidw.aidw_describe_launch(ctx.h, p)


def split_boundary(torch, levels):
    """Queries at which the automatic plan stops splitting m: 1.5 rounds of
    64-query tiles (8 waves per SIMD) when alpha_5 is whole (the speculative
    single pass), two rounds otherwise (the two-pass kernel)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rnd = cus * 4 * 8 * 64  # queries in one round of tiles
    return 3 * rnd // 2 if levels[4] == int(levels[4]) else 2 * rnd


def test_automatic_split_boundaries(ctx, torch):
    """Above the boundary the unsplit launch is the speculative single pass
    when alpha_5 is whole and the two-pass kernel otherwise; below it the
    split kernels run."""
    whole5, frac5 = (1, 2, 3, 4, 5), (1, 2, 3, 4, 4.5)
    nw, nf = split_boundary(torch, whole5), split_boundary(torch, frac5)
    inst = workloads.paper_scale(m=1 << 14, n=max(nw, nf), seed=78, k=15)
    assert "aidw_f32_fused_spec<16>" in _plan(ctx, torch, inst, nw, whole5)
    assert "aidw_f32_knn_part<16>" in _plan(ctx, torch, inst, nw - 64, whole5)
    assert "aidw_f32_fused<16, 1, false>" in _plan(ctx, torch, inst, nf, frac5)
    assert "aidw_f32_knn_part<16>" in _plan(ctx, torch, inst, nf - 64, frac5)


@pytest.mark.parametrize("levels", [(1, 2, 3, 4, 5), (1, 2, 3, 4, 4.5)])
def test_automatic_split_boundary(ctx, torch, levels):
    """The same queries run on both sides of the automatic split boundary:
    identical k-nearest statistics, outputs equal to FP64 summation order, and
    both within the bar on sampled queries."""
    import copy

    n = split_boundary(torch, levels)
    inst = workloads.paper_scale(m=1 << 16, n=n, seed=77, k=15)
    inst.levels = levels
    below = copy.copy(inst)
    below.query_x = np.ascontiguousarray(inst.query_x[: n - 64])
    below.query_y = np.ascontiguousarray(inst.query_y[: n - 64])
    # in the caller's order, so that a query has the same wave mates on both
    # sides (the spatial order of n - 64 queries groups them differently)
    whole, r0, a0, _ = _run(ctx, torch, inst, diag=True, query_order=1)
    split, r1, a1, _ = _run(ctx, torch, below, diag=True, query_order=1)
    assert np.array_equal(r0[: n - 64], r1)
    assert np.array_equal(a0[: n - 64], a1)
    # Above the boundary a whole alpha_5 runs the speculative single pass, in
    # which a query that ends at alpha_5 keeps its whole-power sums even when
    # a wave mate leaves alpha_5; the split kernels then take the general
    # loop for the whole wave.  Such tiles agree to the loops' rounding, the
    # others to FP64 summation order.
    mixed = np.zeros(n - 64, dtype=bool)
    if levels[4] == int(levels[4]):
        mixed = np.repeat((a1.reshape(-1, 64) != levels[4]).any(axis=1), 64)
    w = whole[: n - 64]
    diff = np.abs(split.astype(np.float64) - w)
    say("tiles with a query off alpha_5: %d of %d; max rel diff there %.2e" % (
        mixed.sum() // 64, (n - 64) // 64,
        (diff[mixed] / np.abs(w[mixed])).max() if mixed.any() else 0.0))
    assert np.allclose(split[~mixed], w[~mixed], rtol=2e-7, atol=0)
    assert np.allclose(split, w, rtol=1e-5, atol=1e-6 * np.abs(w).max())
    # the queries of such tiles that kept their sums, against the oracle
    kept = np.flatnonzero(mixed & (a1 == levels[4]))
    if kept.size:
        idx = kept[np.linspace(0, kept.size - 1, min(16, kept.size)).astype(int)]
        o, scale = ref(inst, idx)
        assert rel_err(whole[idx], o, scale).max() <= TOL_F32
    idx = np.unique(np.linspace(0, n - 65, 48).astype(int))
    o, scale = ref(inst, idx)
    assert rel_err(whole[idx], o, scale).max() <= TOL_F32
    assert rel_err(split[idx], o, scale).max() <= TOL_F32


def test_split_with_alpha_zero_and_coincident_queries(ctx, torch):
    inst = workloads.uniform_unit(40000, 300, 7, 10)
    inst.query_x[:30] = inst.data_x[:30]
    inst.query_y[:30] = inst.data_y[:30]
    for levels in [(1, 2, 3, 4, 5), (0, 0, 0, 0, 0)]:
        inst.levels = levels
        out = _run(ctx, torch, inst, segments=16)
        o, scale = ref(inst, np.arange(inst.n))
        assert rel_err(out, o, scale).max() <= TOL_F32
        if levels[0] > 0:
            assert np.array_equal(out[:30], inst.data_z[:30])


def test_deterministic_handle_ignores_launch_shape(ctx, torch):
    """With aidw_options.deterministic the FP32-scaled result does not depend
    on the launch shape (tuning, automatic split for few queries): it is the
    unsplit one-query-per-lane kernel's, which is also what a batched launch
    computes."""
    inst = workloads.clustered(20000, 3000, 5, 10, on_point=0.02)  # few queries: auto split
    dev = Dev(torch, inst)
    det = aidw.Context(0, deterministic=1)
    outs = []
    try:
        for t in [dict(), dict(q_per_lane=2), dict(q_per_lane=4, max_waves_per_simd=4),
                  dict(split_segments=4), dict(q_per_lane=1, split_segments=1)]:
            det.set_tuning(**t)
            outs.append(det.interpolate(dev.data_xy, dev.data_z, dev.query_xy, inst.k,
                                        inst.levels, inst.R_min, inst.R_max,
                                        inst.area).cpu().numpy())
        g = det.interpolate(dev.data_xy, dev.data_z, dev.query_xy, inst.k, inst.levels,
                            inst.R_min, inst.R_max, inst.area,
                            flags=aidw.AIDW_FLAG_GRID_KNN).cpu().numpy()
    finally:
        det.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(outs[0], run_alone(ctx, torch, dev))
    ctx.bind_current_stream()
    aidw.check(aidw.aidw_interpolate_batch(ctx.h, [dev.problem(ctx)]))
    torch.cuda.synchronize()
    assert np.array_equal(dev.out.cpu().numpy(), outs[0])
    # the automatic (non-deterministic) choice splits this problem: it agrees
    # to rounding only
    auto = ctx.interpolate(dev.data_xy, dev.data_z, dev.query_xy, inst.k, inst.levels,
                           inst.R_min, inst.R_max, inst.area).cpu().numpy()
    assert rel_err(auto, outs[0], np.abs(outs[0]) + 1e-30).max() <= 1e-6
    assert rel_err(g, outs[0], np.abs(outs[0]) + 1e-30).max() <= 1e-6
