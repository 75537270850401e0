"""The spatial tile order (which 64 queries share a wave).

The order is a performance device: every query's result is its own whatever
its wave mates.  These tests check the order itself against its definition
(a stable sort by Morton cell code, recomputed here in FP32 with numpy), and
that ordered launches give the oracle's results, the same k-nearest lists,
r_obs and alpha as launches in the caller's order, and outputs equal to
rounding.
"""
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


def spread(v):
    v = v.astype(np.uint64) & np.uint64(0xFFFF)
    out = np.zeros_like(v)
    for b in range(16):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
    return out


def expected_order(qx, qy):
    """The definition in aidw_query_order: b the least b >= 1 with
    16 * 4^b >= n (at most 11); cells floor((v - min) * (2^b / extent)) in
    FP32, clamped; a stable sort of the interleaved codes (x in the even
    bits)."""
    n = qx.size
    b = 1
    while b < 11 and 16 * 4 ** b < n:
        b += 1
    cells = np.float32(2 ** b)
    top = np.float32(2 ** b - 1)

    def cell(v):
        lo, hi = v.min(), v.max()
        scale = cells / (hi - lo) if hi > lo else np.float32(0)
        if not np.isfinite(scale):
            scale = np.float32(0)
        t = np.minimum(np.maximum((v - lo) * np.float32(scale), np.float32(0)), top)
        return t.astype(np.uint32)

    with np.errstate(over="ignore", invalid="ignore"):
        key = spread(cell(qx)) | (spread(cell(qy)) << np.uint64(1))
    return np.argsort(key, kind="stable"), key, b


def device_order(ctx, torch, qx, qy):
    q = torch.from_numpy(np.stack([qx, qy]).astype(np.float32)).cuda()
    order = torch.full((qx.size,), -1, dtype=torch.int32, device="cuda")
    ctx.bind_current_stream()
    aidw.check(aidw.aidw_query_order(ctx.h, q, qx.size, order))
    return order.cpu().numpy()


def _queries(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(0, 1, n).astype(np.float32), rng.uniform(0, 1, n).astype(np.float32)
    if kind == "clustered":
        c = rng.uniform(0, 1, (8, 2))
        pick = rng.integers(0, 8, n)
        pts = c[pick] + rng.normal(0, 1e-3, (n, 2))
        return pts[:, 0].astype(np.float32), pts[:, 1].astype(np.float32)
    if kind == "duplicates":  # many equal keys: stability decides the order
        v = rng.integers(0, 5, (2, n)).astype(np.float32)
        return v[0], v[1]
    if kind == "line":  # zero extent in y
        return rng.uniform(-1e6, 1e6, n).astype(np.float32), np.full(n, 3.5, np.float32)
    if kind == "offset":  # large offset, small extent
        return (1e6 + rng.uniform(0, 1, n)).astype(np.float32), \
            (-2e5 + rng.uniform(0, 1, n)).astype(np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 4095, 4096, 4097, 70001])
@pytest.mark.parametrize("kind", ["uniform", "clustered", "duplicates", "line", "offset"])
def test_order_is_the_stable_morton_sort(ctx, torch, kind, n):
    qx, qy = _queries(kind, n, 7 + n)
    got = device_order(ctx, torch, qx, qy)
    want, key, b = expected_order(qx, qy)
    assert np.array_equal(np.sort(got), np.arange(n))  # a permutation
    assert np.array_equal(got, want), (kind, n, b)


def test_order_three_radix_passes(ctx, torch):
    # n > 16 * 4^8: 9 bits per axis, 18-bit codes, three 8-bit digit passes
    n = (1 << 20) + 4099
    qx, qy = _queries("uniform", n, 11)
    got = device_order(ctx, torch, qx, qy)
    want, _, b = expected_order(qx, qy)
    assert b == 9
    assert np.array_equal(got, want)


def test_order_is_deterministic(ctx, torch):
    qx, qy = _queries("duplicates", 300001, 12)
    a = device_order(ctx, torch, qx, qy)
    b = device_order(ctx, torch, qx, qy)
    assert np.array_equal(a, b)


def test_order_argument_errors(ctx, torch):
    q = torch.zeros((2, 10), dtype=torch.float32, device="cuda")
    order = torch.empty(10, dtype=torch.int32, device="cuda")
    assert aidw.aidw_query_order(ctx.h, q, -1, order) == aidw.AIDW_EINVAL
    assert aidw.aidw_query_order(ctx.h, None, 10, order) == aidw.AIDW_EINVAL
    assert aidw.aidw_query_order(ctx.h, q, 0, None) == aidw.AIDW_OK


def _run(ctx, torch, inst, query_order, split=0, knn=False):
    d = aidw.to_device(inst)
    ctx.set_tuning(split_segments=split, query_order=query_order)
    try:
        r = ctx.interpolate(*d, inst.k, inst.levels, inst.R_min, inst.R_max, inst.area,
                            diag=True, knn=knn)
    finally:
        ctx.set_tuning()
    torch.cuda.synchronize()
    return [None if t is None else t.cpu().numpy() for t in r]


def _oracle_err(inst, out, idx):
    a = (inst.data_x, inst.data_y)
    kw = dict(alpha_levels=inst.levels, R_min=inst.R_min, R_max=inst.R_max, area=inst.area)
    want = oracle.run(*a, inst.data_z, inst.query_x[idx], inst.query_y[idx], inst.k, **kw)
    scale = oracle.run(*a, np.abs(inst.data_z), inst.query_x[idx], inst.query_y[idx], inst.k,
                       **kw)
    return float(np.max(np.abs(out[idx].astype(np.float64) - want) / scale))


@pytest.mark.parametrize("split", [1, 5])
@pytest.mark.parametrize("levels", [(1, 2, 3, 4, 5), (1, 2, 3, 4, 4.5)])
def test_ordered_launch_matches_caller_order(ctx, torch, split, levels):
    # clustered data: alpha varies; forced unsplit (speculative single pass or
    # two-pass kernel) and forced split launches
    inst = workloads.clustered(m=30011, n=3001, seed=40 + split, k=10, on_point=0.02)
    inst.levels = levels
    o1, r1, a1, _ = _run(ctx, torch, inst, 2, split)
    o0, r0, a0, _ = _run(ctx, torch, inst, 1, split)
    assert not np.isnan(o1).any()
    assert np.array_equal(r0, r1) and np.array_equal(a0, a1)
    assert np.allclose(o1, o0, rtol=1e-5, atol=1e-6 * np.abs(o0).max())
    idx = np.unique(np.linspace(0, inst.n - 1, 40).astype(int))
    err = _oracle_err(inst, o1, idx)
    say("split %d levels %s: err %.3e" % (split, levels, err))
    assert err <= TOL_F32


def test_ordered_launch_with_knn_indices(ctx, torch):
    # the k-nearest indices go to each query's own row
    inst = workloads.clustered(m=9000, n=700, seed=45, k=15, on_point=0.05)
    o1, r1, a1, k1 = _run(ctx, torch, inst, 2, knn=True)
    o0, r0, a0, k0 = _run(ctx, torch, inst, 1, knn=True)
    assert np.array_equal(k0, k1)
    assert np.array_equal(r0, r1) and np.array_equal(a0, a1)
    assert np.allclose(o1, o0, rtol=1e-5, atol=1e-6 * np.abs(o0).max())


def test_ordering_groups_neighbours(ctx, torch):
    # the point of the order: a tile's queries are neighbours
    qx, qy = _queries("uniform", 1 << 16, 13)
    order = device_order(ctx, torch, qx, qy)
    t = order.reshape(-1, 64)
    area = (qx[t].max(1) - qx[t].min(1)) * (qy[t].max(1) - qy[t].min(1))
    say("mean tile bounding box: %.2e of the square" % area.mean())
    assert area.mean() < 64 * 16 / qx.size


def test_automatic_order_threshold(ctx, torch):
    inst = workloads.uniform_unit(2000, 300, 3, 8)
    d = aidw.to_device(inst)
    out = torch.empty(inst.n, device="cuda")
    p = ctx.problem(*d, inst.k, out, inst.levels, inst.R_min, inst.R_max, inst.area)
    assert aidw.aidw_describe_launch(ctx.h, p).startswith("aidw_order_box_part")
    small = workloads.uniform_unit(1000, 300, 3, 8)  # fewer than 1024 points
    ds = aidw.to_device(small)
    ps = ctx.problem(*ds, small.k, out, small.levels, small.R_min, small.R_max, small.area)
    # (the Morton order starts with aidw_order_box_part; a split problem's
    # pass-2 regroup uses the sort kernels alone)
    assert "aidw_order_box_part" not in aidw.aidw_describe_launch(ctx.h, ps)
    one_tile = ctx.problem(d[0], d[1], d[2][:, :64].contiguous(), inst.k, out[:64], inst.levels,
                           inst.R_min, inst.R_max, inst.area)
    assert "aidw_order_box_part" not in aidw.aidw_describe_launch(ctx.h, one_tile)
    ctx.set_tuning(query_order=1)
    try:
        assert "aidw_order" not in aidw.aidw_describe_launch(ctx.h, p)  # nor the regroup
    finally:
        ctx.set_tuning()


def test_order_with_non_finite_queries(ctx, torch):
    # NaN and infinite coordinates land in edge cells: the order stays a
    # permutation, and an ordered launch still gives every finite query the
    # oracle's result (the others come out NaN, as in the caller's order)
    inst = workloads.uniform_unit(5000, 700, 46, 10)
    qx, qy = inst.query_x.copy(), inst.query_y.copy()
    bad = np.arange(0, 700, 37)
    qx[bad[::3]] = np.nan
    qy[bad[1::3]] = np.inf
    qx[bad[2::3]] = -np.inf
    order = device_order(ctx, torch, qx, qy)
    assert np.array_equal(np.sort(order), np.arange(qx.size))
    inst.query_x, inst.query_y = qx, qy
    o1, r1, a1, _ = _run(ctx, torch, inst, 2)
    o0, r0, a0, _ = _run(ctx, torch, inst, 1)
    good = np.setdiff1d(np.arange(inst.n), bad)
    assert np.array_equal(r0[good], r1[good]) and np.array_equal(a0[good], a1[good])
    assert np.allclose(o1[good], o0[good], rtol=1e-5, atol=1e-6 * np.abs(o0[good]).max())
    assert np.array_equal(np.isnan(o1), np.isnan(o0))
    err = _oracle_err(inst, o1, good[::20])
    assert err <= TOL_F32


def test_order_left_out_under_a_tight_budget(torch):
    # two rounds of tiles and a non-whole alpha_5: the unsplit two-pass kernel,
    # whose workspace is a few bytes; the order's ~20 n bytes do not fit a
    # 4 MiB budget, so the call runs in the caller's order instead of failing
    inst = workloads.paper_scale(m=2048, n=(1 << 20) + 64, seed=47, k=10)
    inst.levels = (1, 2, 3, 4, 4.5)
    d = aidw.to_device(inst)
    tight = aidw.Context(0, hbm_budget_bytes=4 << 20)
    plain = aidw.Context(0)
    try:
        out = tight.interpolate(*d, inst.k, inst.levels, inst.R_min, inst.R_max, inst.area)
        plain.set_tuning(query_order=1)
        ref_out = plain.interpolate(*d, inst.k, inst.levels, inst.R_min, inst.R_max, inst.area)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref_out.cpu().numpy())
    finally:
        tight.close()
        plain.close()
