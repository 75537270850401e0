"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Error metric (primary): |z_gpu - z_ref| / (sum w|z| / sum w), the oracle's own
weighted mean of |z| (obtained by running the oracle on |z|, since the weights
do not depend on z).  Bars: FP32-scaled <= 1e-4; plain FP64 <= 1e-12 with
kNN index sets identical to the oracle's (ties broken by data index).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1511_02186_amd import aidw, workloads

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4
TOL_F64 = 1e-12


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


def gpu_run(ctx, torch, inst, diag=False, q_per_lane=0, query_index=None, split=0, cap=0):
    inst_q = inst if query_index is None else _subset(inst, query_index)
    data_xy, data_z, query_xy = aidw.to_device(inst_q)
    ctx.set_tuning(q_per_lane, cap, split)
    try:
        res = ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min,
                              inst.R_max, inst.area, diag=diag)
    finally:
        ctx.set_tuning(0)
    torch.cuda.synchronize()
    if diag:
        return tuple(t.cpu().numpy() for t in res)
    return res.cpu().numpy()


def _subset(inst, idx):
    import copy

    s = copy.copy(inst)
    s.query_x = np.ascontiguousarray(inst.query_x[idx])
    s.query_y = np.ascontiguousarray(inst.query_y[idx])
    return s


def ref(inst, idx=None, diag=False, levels=None):
    qx = inst.query_x if idx is None else inst.query_x[idx]
    qy = inst.query_y if idx is None else inst.query_y[idx]
    lv = inst.levels if levels is None else levels
    args = (inst.data_x, inst.data_y)
    res = oracle.run(*args, inst.data_z, qx, qy, inst.k, lv, inst.R_min, inst.R_max, inst.area,
                     diag=diag)
    scale = oracle.run(*args, np.abs(inst.data_z), qx, qy, inst.k, lv, inst.R_min, inst.R_max,
                       inst.area)
    return res, scale


def rel_err(got, want, scale):
    diff = np.abs(np.asarray(got, dtype=np.float64) - want)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(scale > 0, diff / scale, np.where(diff == 0, 0.0, np.inf))
    return e


# ---- small single instance in FP64 and FP32 ------------------------------------

def test_small_fp64_exact_knn_and_1e12(ctx, torch):
    inst = workloads.uniform_small()  # m = n = 1024, k = 10, FP64, seed 0
    out, r_obs, alpha, knn = gpu_run(ctx, torch, inst, diag=True)
    (o_out, o_r, o_a, o_knn), scale = ref(inst, diag=True)
    assert np.array_equal(knn.astype(np.int64), o_knn)
    assert np.max(np.abs(r_obs - o_r) / o_r) <= 1e-14
    assert np.max(np.abs(alpha - o_a)) <= 1e-13
    err = rel_err(out, o_out, scale)
    say("fp64 small: max err %.3e" % err.max())
    assert err.max() <= TOL_F64


def test_small_fp32_scaled(ctx, torch):
    inst = workloads.uniform_small(dtype=np.float32)
    out, r_obs, alpha, _ = gpu_run(ctx, torch, inst, diag=True)
    (o_out, o_r, o_a, _), scale = ref(inst, diag=True)
    err = rel_err(out, o_out, scale)
    say("fp32 small: max err %.3e (vs |z|: %.3e)" % (err.max(),
        np.max(np.abs(out - o_out) / np.maximum(np.abs(o_out), 1e-300))))
    assert err.max() <= TOL_F32
    assert np.max(np.abs(r_obs - o_r) / o_r) <= 1e-6
    assert np.max(np.abs(alpha - o_a)) <= 1e-5


@pytest.mark.parametrize("q,cap", [(1, 0), (2, 0), (4, 0), (1, 2), (2, 4)])
def test_fp32_launch_shapes_agree(ctx, torch, q, cap):
    # one fused launch (no split of m), so the queries-per-lane and
    # occupancy-cap variants of the kernel really run
    inst = workloads.paper_scale(m=3001, n=2 * 4 * 256 + 77, seed=21)
    inst.query_x[::41] = inst.data_x[:len(inst.query_x[::41])]  # some queries on data points
    inst.query_y[::41] = inst.data_y[:len(inst.query_y[::41])]
    out = gpu_run(ctx, torch, inst, q_per_lane=q, split=1, cap=cap)
    base = gpu_run(ctx, torch, inst, q_per_lane=1, split=1)
    # one query per lane may take the one-transcendental pass 2 for waves of
    # a common whole power; the shapes agree to rounding
    assert np.allclose(out, base, rtol=2e-6, atol=1e-6 * np.abs(base).max())
    assert np.array_equal(out[::41], inst.data_z[:len(out[::41])])  # z_i of the point hit
    o, scale = ref(inst, idx=np.arange(0, inst.n, 7))
    assert rel_err(out[::7], o, scale).max() <= TOL_F32


# ---- every register bucket, ragged sizes --------------------------------------

KS = [1, 2, 3, 4, 5, 8, 9, 10, 11, 12, 15, 16, 17, 20, 23, 24, 25, 31, 32]


@pytest.mark.parametrize("k", KS)
def test_ragged_sizes_all_k_fp64(ctx, torch, k):
    inst = workloads.uniform_small(m=700 + 13 * k, n=333, seed=100 + k, k=k)
    out, r_obs, alpha, knn = gpu_run(ctx, torch, inst, diag=True)
    (o_out, o_r, o_a, o_knn), scale = ref(inst, diag=True)
    assert np.array_equal(knn.astype(np.int64), o_knn)
    assert rel_err(out, o_out, scale).max() <= TOL_F64


@pytest.mark.parametrize("k", KS)
def test_ragged_sizes_all_k_fp32(ctx, torch, k):
    inst = workloads.paper_scale(m=900 + 17 * k, n=555, seed=200 + k, k=k)
    out, _, alpha, knn = gpu_run(ctx, torch, inst, diag=True)
    (o_out, _, o_a, o_knn), scale = ref(inst, diag=True)
    assert rel_err(out, o_out, scale).max() <= TOL_F32
    # FP32 squared distances may order near-ties differently from FP64: the
    # selected sets must be valid k-nearest sets up to FP32 rounding.
    for q in range(0, inst.n, 37):
        assert len(set(knn[q])) == k and knn[q].min() >= 0 and knn[q].max() < inst.m
        d_gpu = np.sort(np.hypot(inst.query_x[q] - inst.data_x[knn[q]].astype(np.float64),
                                 inst.query_y[q] - inst.data_y[knn[q]].astype(np.float64)))
        d_ref = np.sort(np.hypot(inst.query_x[q] - inst.data_x[o_knn[q]].astype(np.float64),
                                 inst.query_y[q] - inst.data_y[o_knn[q]].astype(np.float64)))
        assert np.allclose(d_gpu, d_ref, rtol=1e-6, atol=1e-9)


# ---- edge cases -----------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("m,k", [(1, 1), (5, 5), (16, 3), (17, 16), (33, 32)])
def test_minimal_data_sets(ctx, torch, dtype, m, k):
    inst = workloads.uniform_small(m=m, n=70, seed=m + k, k=k, dtype=dtype)
    inst.area = 1.0  # the unit square (one point has a zero-area bounding box)
    out = gpu_run(ctx, torch, inst)
    o, scale = ref(inst)
    assert rel_err(out, o, scale).max() <= (TOL_F64 if dtype == np.float64 else TOL_F32)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_queries_on_data_points_return_their_values(ctx, torch, dtype):
    inst = workloads.uniform_small(m=1000, n=300, seed=3, dtype=dtype)
    idx = np.random.default_rng(0).choice(inst.m, 100, replace=False)
    inst.query_x[:100] = inst.data_x[idx]
    inst.query_y[:100] = inst.data_y[idx]
    out = gpu_run(ctx, torch, inst)
    assert np.array_equal(out[:100], inst.data_z[idx])
    o, scale = ref(inst)
    assert rel_err(out, o, scale).max() <= (TOL_F64 if dtype == np.float64 else TOL_F32)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_duplicate_data_points(ctx, torch, dtype):
    inst = workloads.uniform_small(m=400, n=100, seed=4, dtype=dtype)
    inst.data_x[200:300] = inst.data_x[:100]
    inst.data_y[200:300] = inst.data_y[:100]
    inst.query_x[:50] = inst.data_x[:50]
    inst.query_y[:50] = inst.data_y[:50]
    out = gpu_run(ctx, torch, inst)
    want = (inst.data_z[:50].astype(np.float64) + inst.data_z[200:250]) / 2
    assert np.allclose(out[:50], want, rtol=0, atol=1e-6 if dtype == np.float32 else 1e-15)
    o, scale = ref(inst)
    assert rel_err(out, o, scale).max() <= (TOL_F64 if dtype == np.float64 else TOL_F32)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_constant_power_of_two_field_is_exact(ctx, torch, dtype):
    inst = workloads.uniform_small(m=777, n=250, seed=5, dtype=dtype)
    inst.data_z[:] = 4.0
    out = gpu_run(ctx, torch, inst)
    assert np.all(out == 4.0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("levels", [(0, 0, 0, 0, 0), (2, 2, 2, 2, 2), (0.5, 1.5, 2.5, 4, 6),
                                    (6, 4, 2.5, 1.5, 0.5)])
def test_other_alpha_levels(ctx, torch, dtype, levels):
    inst = workloads.clustered(m=3000, n=500, seed=6, k=8, dtype=dtype)
    inst.levels = levels
    out, _, alpha, _ = gpu_run(ctx, torch, inst, diag=True)
    (o, _, o_a, _), scale = ref(inst, diag=True)
    assert np.max(np.abs(alpha - o_a)) <= (1e-12 if dtype == np.float64 else 1e-5)
    assert rel_err(out, o, scale).max() <= (TOL_F64 if dtype == np.float64 else TOL_F32)
    if len(set(levels)) == 1:
        idw = oracle.idw(inst.data_x, inst.data_y, inst.data_z, inst.query_x, inst.query_y,
                         levels[0])
        assert rel_err(out, idw, scale).max() <= (TOL_F64 if dtype == np.float64 else TOL_F32)


# m around multiples of the 16-point pass-2 batch: the software-pipelined
# loops need two whole batches, end on the last whole one and leave the rest
# to the point-by-point tail; whole levels take the rsq loop, the others the
# log2/exp2 loop, and queries on data points its clamped variant
@pytest.mark.parametrize("m", [31, 32, 33, 47, 48, 49, 64, 95])
@pytest.mark.parametrize("levels", [(5, 5, 5, 5, 5), (0.5, 1.5, 2.5, 4, 6)])
@pytest.mark.parametrize("on_point", [0.0, 0.05])
def test_pass2_batch_boundaries(ctx, torch, m, levels, on_point):
    inst = workloads.clustered(m=m, n=300, seed=40 + m, k=min(8, m), on_point=on_point)
    inst.levels = levels
    out = gpu_run(ctx, torch, inst)
    o, scale = ref(inst)
    err = rel_err(out, o, scale).max()
    say("m=%d levels=%s on_point=%g: max err %.3e" % (m, levels, on_point, err))
    assert err <= TOL_F32


def test_empty_query_set_is_a_no_op(ctx, torch):
    d = torch.rand(2, 10, device="cuda")
    z = torch.rand(10, device="cuda")
    q = torch.empty(2, 0, device="cuda")
    out = torch.empty(0, device="cuda")
    res = ctx.interpolate(d, z, q, 3, area=1.0, out=out)
    assert res.numel() == 0


@pytest.mark.parametrize("bad", [
    dict(k=0), dict(k=11), dict(k=33), dict(area=0.0), dict(area=float("nan")),
    dict(R_min=2.0, R_max=1.0), dict(R_min=-1.0, R_max=0.0),
    dict(alpha_levels=(1, 2, -3, 4, 5)), dict(alpha_levels=(1, 2, float("inf"), 4, 5)),
])
def test_invalid_arguments_leave_output_untouched(ctx, torch, bad):
    d = torch.rand(2, 10, device="cuda")
    z = torch.rand(10, device="cuda")
    q = torch.rand(2, 7, device="cuda")
    out = torch.full((7,), 123.0, device="cuda")
    kw = dict(k=3, alpha_levels=(1, 2, 3, 4, 5), R_min=0.0, R_max=2.0, area=1.0)
    kw.update(bad)
    with pytest.raises(aidw.AidwError) as ei:
        ctx.interpolate(d, z, q, kw.pop("k"), out=out, **kw)
    assert ei.value.status == aidw.AIDW_EINVAL
    torch.cuda.synchronize()
    assert torch.all(out == 123.0)


def test_plain_c_entry_point(ctx, torch):
    inst = workloads.uniform_small(m=500, n=64, seed=8, dtype=np.float32)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    out = torch.empty(inst.n, device="cuda")
    ctx.bind_current_stream()
    aidw.check(aidw.aidw_interpolate(ctx.h, data_xy.data_ptr(), data_z.data_ptr(), inst.m,
                                     query_xy.data_ptr(), inst.n, inst.k, inst.levels,
                                     inst.R_min, inst.R_max, inst.area, out.data_ptr()))
    o, scale = ref(inst)
    assert rel_err(out.cpu().numpy(), o, scale).max() <= TOL_F32


# ---- determinism and invariance ------------------------------------------------

def test_repeat_runs_are_bitwise_identical(ctx, torch):
    inst = workloads.clustered(m=20000, n=5000, seed=9)
    a = gpu_run(ctx, torch, inst)
    for _ in range(3):
        assert np.array_equal(a, gpu_run(ctx, torch, inst))


def test_query_permutation_permutes_output(ctx, torch):
    inst = workloads.paper_scale(m=5000, n=3000, seed=10)
    a = gpu_run(ctx, torch, inst)
    perm = np.random.default_rng(1).permutation(inst.n)
    b = gpu_run(ctx, torch, inst, query_index=perm)
    assert np.array_equal(a[perm], b)


def test_async_on_side_stream(ctx, torch):
    inst = workloads.paper_scale(m=4000, n=4000, seed=11)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = ctx.interpolate(data_xy, data_z, query_xy, inst.k, area=inst.area,
                              flags=aidw.AIDW_FLAG_ASYNC)
    s.synchronize()
    o, scale = ref(inst, idx=np.arange(0, inst.n, 50))
    assert rel_err(out.cpu().numpy()[::50], o, scale).max() <= TOL_F32


# ---- full sizes, sampled ----------------------------------------------------

def test_paper_scale_full_size_sampled(ctx, torch):
    # the production launch (speculative single pass, spatial tile order) at
    # full size: random queries, the ends, and every query whose alpha left
    # alpha_5 (their tiles run the deferred pass 2, the exp2/log2 loop for
    # general alpha; about 0.03 % of the queries here)
    inst = workloads.paper_scale()  # m = n = 2^20, k = 15, FP32
    say("paper scale: m=%d n=%d" % (inst.m, inst.n))
    data_xy, data_z, query_xy = aidw.to_device(inst)
    res = ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min,
                          inst.R_max, inst.area, diag=True, knn=False)
    torch.cuda.synchronize()
    out, r_obs, alpha = (t.cpu().numpy() for t in res[:3])
    off = np.nonzero(alpha != inst.levels[4])[0]
    say("paper scale: %d queries off alpha_5" % off.size)
    assert 0 < off.size < 2000
    idx = np.sort(np.random.default_rng(12).choice(inst.n, 160, replace=False))
    idx = np.unique(np.concatenate([idx, [0, inst.n - 1], off]))
    want, w_robs, w_alpha, _ = oracle.run(inst.data_x, inst.data_y, inst.data_z,
                                          inst.query_x[idx], inst.query_y[idx], inst.k,
                                          inst.levels, inst.R_min, inst.R_max, inst.area,
                                          diag=True)
    scale = oracle.run(inst.data_x, inst.data_y, np.abs(inst.data_z), inst.query_x[idx],
                       inst.query_y[idx], inst.k, inst.levels, inst.R_min, inst.R_max, inst.area)
    err = rel_err(out[idx], want, scale)
    say("paper scale fp32: max err %.3e over %d queries (%d off alpha_5)"
        % (err.max(), len(idx), off.size))
    assert err.max() <= TOL_F32
    assert np.allclose(r_obs[idx], w_robs, rtol=1e-6, atol=0)
    assert np.allclose(alpha[idx], w_alpha, rtol=1e-5, atol=1e-6)


def test_paper_scale_fp64_kernel_subset(ctx, torch):
    inst = workloads.paper_scale(dtype=np.float64)
    idx = np.arange(0, inst.n, 256)  # 4096 queries against all 2^20 data points
    out, r_obs, alpha, knn = gpu_run(ctx, torch, inst, diag=True, query_index=idx)
    sub = np.arange(0, len(idx), 64)
    (o, o_r, o_a, o_knn), scale = ref(inst, idx=idx[sub], diag=True)
    assert np.array_equal(knn[sub].astype(np.int64), o_knn)
    assert rel_err(out[sub], o, scale).max() <= TOL_F64


def test_clustered_full_size_sampled(ctx, torch):
    inst = workloads.clustered()  # m = n = 2^18, k = 10, FP32, 1% on-point queries
    out = gpu_run(ctx, torch, inst)
    on = inst.meta["on_point_queries"]
    idx = np.sort(np.concatenate([np.random.default_rng(13).choice(inst.n, 120, replace=False),
                                  on[:40]]))
    o, scale = ref(inst, idx=idx)
    err = rel_err(out[idx], o, scale)
    say("clustered fp32: max err %.3e over %d sampled queries" % (err.max(), len(idx)))
    assert err.max() <= TOL_F32
    # an on-point query with a unique location returns that point's value
    xs = inst.data_x[inst.meta["on_point_data"][:40]]
    ys = inst.data_y[inst.meta["on_point_data"][:40]]
    for q, x, y, d in zip(on[:40], xs, ys, inst.meta["on_point_data"][:40]):
        if np.count_nonzero((inst.data_x == x) & (inst.data_y == y)) == 1:
            assert out[q] == inst.data_z[d]


# ---- standard IDW (constant power) ------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("power", [0.0, 1.0, 2.0, 3.3])
def test_standard_idw_matches_oracle(ctx, torch, dtype, power):
    inst = workloads.clustered(m=20000, n=700, seed=31, k=1, dtype=dtype, on_point=0.02)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    out = aidw.idw(ctx, data_xy, data_z, query_xy, power).cpu().numpy()
    want = oracle.idw(inst.data_x, inst.data_y, inst.data_z, inst.query_x, inst.query_y, power)
    scale = oracle.idw(inst.data_x, inst.data_y, np.abs(inst.data_z), inst.query_x,
                       inst.query_y, power)
    assert rel_err(out, want, scale).max() <= (TOL_F64 if dtype == np.float64 else TOL_F32)


def test_standard_idw_rejects_negative_power(ctx, torch):
    d = torch.rand(2, 10, device="cuda")
    z = torch.rand(10, device="cuda")
    q = torch.rand(2, 4, device="cuda")
    with pytest.raises(aidw.AidwError) as ei:
        aidw.idw(ctx, d, z, q, -1.0)
    assert ei.value.status == aidw.AIDW_EINVAL


# ---- data-access variants (the paper's naive / tiled designs, SoA / AoaS) ----------

@pytest.mark.parametrize("access", [aidw.AIDW_ACCESS_SCALAR, aidw.AIDW_ACCESS_TILED,
                                    aidw.AIDW_ACCESS_NAIVE])
@pytest.mark.parametrize("layout", [aidw.AIDW_LAYOUT_SOA, aidw.AIDW_LAYOUT_AOAS])
@pytest.mark.parametrize("m,n,k", [(1, 3, 1), (255, 257, 8), (5003, 1001, 15)])
def test_access_variants_match_oracle(ctx, torch, access, layout, m, n, k):
    inst = workloads.clustered(m=m, n=n, seed=m + n + access, k=k, on_point=0.05)
    inst.area = max(inst.area, 1e-6) if m > 1 else 1.0
    data_xy, data_z, query_xy = aidw.to_device(inst)
    out = torch.full((inst.n,), float("nan"), device="cuda")
    alpha = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    ctx.bind_current_stream()
    p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min, inst.R_max,
                    inst.area, alpha=alpha)
    aidw.check(aidw.aidw_interpolate_variant(ctx.h, p, access, layout))
    (o, _, o_a, _), scale = ref(inst, diag=True)
    assert rel_err(out.cpu().numpy(), o, scale).max() <= TOL_F32
    assert np.max(np.abs(alpha.cpu().numpy() - o_a)) <= 1e-5


@pytest.mark.parametrize("access,layout", [(0, 1), (1, 0), (1, 1), (2, 0), (2, 1)])
@pytest.mark.parametrize("m,n,k", [(700, 300, 10), (1537, 257, 15), (3, 65, 3)])
def test_fp64_access_variants_equal_plain_kernel(ctx, torch, access, layout, m, n, k):
    # the FP64 designs do the plain kernel's arithmetic in its order: equal
    # to it bit for bit, to the oracle within 1e-12, with exact k-nearest sets
    inst = workloads.clustered(m=m, n=n, seed=m + n + access, k=k, on_point=0.05,
                               dtype=np.float64)
    inst.area = max(inst.area, 1e-6) if m > 1 else 1.0
    data_xy, data_z, query_xy = aidw.to_device(inst)
    outs, knns = [], []
    for acc, lay in ((0, 0), (access, layout)):
        out = torch.full((inst.n,), float("nan"), dtype=torch.float64, device="cuda")
        knn = torch.full((inst.n, inst.k), -7, dtype=torch.int32, device="cuda")
        ctx.bind_current_stream()
        p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min,
                        inst.R_max, inst.area, knn_idx=knn)
        aidw.check(aidw.aidw_interpolate_variant(ctx.h, p, acc, lay))
        outs.append(out.cpu().numpy())
        knns.append(knn.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(knns[0], knns[1])
    (o, _, _, o_knn), _ = ref(inst, diag=True)
    assert np.max(np.abs(outs[1] - o) / np.maximum(np.abs(o), 1e-300)) <= TOL_F64
    assert np.array_equal(np.sort(knns[1], axis=1), np.sort(o_knn, axis=1))


# ---- whole powers: the unscaled weights only where FP32 holds them -----------------

@pytest.mark.parametrize("coord_scale", [1e-7, 1.0, 1e3, 1e7])
@pytest.mark.parametrize("z_scale", [1.0, 1e30])
@pytest.mark.parametrize("power", [1.0, 2.0, 5.0, 8.0])
def test_whole_power_weights_in_range(ctx, torch, coord_scale, z_scale, power):
    # every level equal: alpha is the whole number `power` for every query, so
    # every wave takes the one-transcendental path; the range of d^-power and of
    # max|z| decides whether the d_min rescaling may be skipped
    inst = workloads.clustered(m=6000, n=900, seed=int(power) + 3, k=8, on_point=0.0)
    inst.data_x = (inst.data_x * coord_scale).astype(np.float32)
    inst.data_y = (inst.data_y * coord_scale).astype(np.float32)
    inst.query_x = (inst.query_x * coord_scale).astype(np.float32)
    inst.query_y = (inst.query_y * coord_scale).astype(np.float32)
    inst.data_z = (inst.data_z * z_scale).astype(np.float32)
    inst.area = workloads.bbox_area(inst.data_x, inst.data_y)
    inst.levels = (power,) * 5
    out = gpu_run(ctx, torch, inst)
    assert np.all(np.isfinite(out))
    o, scale = ref(inst)
    err = rel_err(out, o, scale)
    say("power %g coords x%g z x%g: max err %.3e" % (power, coord_scale, z_scale, err.max()))
    assert err.max() <= TOL_F32


# ---- tracked and untracked pass 1 keep the same k nearest ----------------------------

def _r_obs_alpha(ctx, torch, inst, track):
    data_xy, data_z, query_xy = aidw.to_device(inst)
    n = inst.n
    out = torch.empty(n, device="cuda")
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    knn = torch.empty((n, inst.k), dtype=torch.int32, device="cuda") if track else None
    ctx.bind_current_stream()
    p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min, inst.R_max,
                    inst.area, r_obs=r, alpha=a, knn_idx=knn)
    # the caller's order: a split pass 2 keeps the pass-1 tiles, so both runs
    # give each query the same pass-2 loop
    ctx.set_tuning(query_order=1)
    try:
        aidw.check(aidw.aidw_interpolate_ex(ctx.h, p))
    finally:
        ctx.set_tuning()
    torch.cuda.synchronize()
    return r.cpu().numpy(), a.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("case", ["offset", "tiny", "clustered", "duplicates", "line"])
@pytest.mark.parametrize("k", [1, 7, 32])
def test_untracked_pass1_equals_tracked_scan(ctx, torch, case, k):
    # kNN-index tracking runs the (d^2, index) list and never splits m; without
    # it the list holds distances only and m may be split into segments
    rng = np.random.default_rng(k * 31 + len(case))
    m, n = 9000, 1500
    if case == "offset":  # large coordinates, small spread: strong cancellation
        dx, dy = 1e5 + rng.random(m), -3e4 + rng.random(m)
    elif case == "tiny":
        dx, dy = 1e-6 * rng.random(m), 1e-6 * rng.random(m)
    elif case == "clustered":
        c = rng.random((8, 2))
        pick = rng.integers(0, 8, m)
        dx = c[pick, 0] + 1e-4 * rng.standard_normal(m)
        dy = c[pick, 1] + 1e-4 * rng.standard_normal(m)
    elif case == "duplicates":
        bx, by = rng.random(m // 3), rng.random(m // 3)
        dx, dy = np.tile(bx, 3), np.tile(by, 3)
    else:  # all on one line
        dx, dy = rng.random(m), np.full(m, 0.5)
    lo_x, hi_x, lo_y, hi_y = dx.min(), dx.max(), dy.min(), dy.max()
    qx = rng.uniform(lo_x - 0.1 * (hi_x - lo_x), hi_x + 0.1 * (hi_x - lo_x), n)
    qy = rng.uniform(lo_y - 0.1 * (hi_y - lo_y) - 1e-7, hi_y + 0.1 * (hi_y - lo_y) + 1e-7, n)
    qx[:50], qy[:50] = dx[:50], dy[:50]  # on-point queries
    inst = workloads.uniform_unit(m=m, n=n, k=k, seed=1, dtype=np.float32)
    inst.data_x, inst.data_y = dx.astype(np.float32), dy.astype(np.float32)
    inst.query_x, inst.query_y = qx.astype(np.float32), qy.astype(np.float32)
    inst.data_z = rng.standard_normal(m).astype(np.float32)
    inst.area = max(workloads.bbox_area(inst.data_x, inst.data_y), 1e-12)
    r0, a0, o0 = _r_obs_alpha(ctx, torch, inst, track=True)
    r1, a1, o1 = _r_obs_alpha(ctx, torch, inst, track=False)
    assert np.array_equal(r0, r1)
    assert np.array_equal(a0, a1)
    # the untracked run may split m into segments: same sums up to FP64 order
    assert np.allclose(o1, o0, rtol=1e-6, atol=1e-30)


def test_issue_cost_probe_is_plausible(ctx, torch):
    c = aidw.aidw_probe_issue_costs(ctx.h)
    say("issue costs: %s" % c)
    assert c["compute_units"] >= 1 and c["clock_ghz"] > 0.5
    # a wave64 FMA takes at least one pass of a 32-lane pipe and a transcendental more
    assert 1.5 < c["fma_cycles"] < 8.0
    assert c["fma_cycles"] < c["exp_cycles"] < 64.0
    assert 0.0 <= c["exp_cycles_beside_fma"] < 64.0
    # an SGPR-operand instruction costs at least what a plain one does, and
    # interleaving VGPR-only work can only lower the cost per instruction
    assert c["fma_cycles"] * 0.8 < c["sgpr_operand_cycles"] < 16.0
    assert 1.0 < c["sgpr_beside_vgpr_cycles"] <= c["sgpr_operand_cycles"] * 1.05


# ---- size limits and malformed pointers (host validation, nothing launched) ----------

@pytest.mark.parametrize("field,value", [("m", 1 << 31), ("m", aidw.AIDW_MAX_POINTS + 1),
                                         ("m", 0), ("n", 1 << 31),
                                         ("n", aidw.AIDW_MAX_POINTS + 1), ("n", -1),
                                         ("misaligned", 1), ("null_out", 0)])
def test_size_limits_and_pointers_are_validated(ctx, torch, field, value):
    d = torch.rand(2, 64, device="cuda")
    z = torch.rand(64, device="cuda")
    q = torch.rand(2, 8, device="cuda")
    out = torch.full((8,), 7.0, device="cuda")
    ctx.bind_current_stream()
    p = ctx.problem(d, z, q, 4, out, area=1.0)
    if field == "m":
        p.m = value
    elif field == "n":
        p.n = value
    elif field == "misaligned":
        p.data_z = z.data_ptr() + value
    else:
        p.out = None
    assert aidw.aidw_interpolate_ex(ctx.h, p) == aidw.AIDW_EINVAL
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)


def test_sixteen_million_points_k32(ctx, torch):
    # m = 2^24 (the data alone 192 MiB), few queries (split into data segments),
    # the largest k; sampled queries against the oracle
    inst = workloads.paper_scale(m=1 << 24, n=3000, seed=17, k=32)
    out = gpu_run(ctx, torch, inst)
    idx = np.concatenate([np.arange(0, 3000, 97), [2999]])
    o, scale = ref(inst, idx=idx)
    err = rel_err(out[idx], o, scale)
    say("m=2^24 k=32: max err %.3e over %d sampled queries" % (err.max(), len(idx)))
    assert err.max() <= TOL_F32
