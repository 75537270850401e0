"""The grid k-nearest search (AIDW_FLAG_GRID_KNN) against the full scan and the
FP64 oracle.

The grid only replaces how pass 1 finds the k nearest squared distances, so
r_obs and alpha must equal the full scan's bit for bit (same FP32 distance
formula, same FP64 alpha arithmetic); the output is held to the FP32-scaled
bar against the oracle.
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


def run(ctx, torch, inst, flags):
    data_xy, data_z, query_xy = aidw.to_device(inst)
    n = inst.n
    out = torch.full((n,), float("nan"), device="cuda")
    r_obs = torch.empty(n, dtype=torch.float64, device="cuda")
    alpha = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.bind_current_stream()
    p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min, inst.R_max,
                    inst.area, r_obs=r_obs, alpha=alpha, flags=flags)
    aidw.check(aidw.aidw_interpolate_ex(ctx.h, p))
    torch.cuda.synchronize()
    return out.cpu().numpy(), r_obs.cpu().numpy(), alpha.cpu().numpy()


def ref(inst, idx=None):
    qx = inst.query_x if idx is None else inst.query_x[idx]
    qy = inst.query_y if idx is None else inst.query_y[idx]
    args = (inst.data_x, inst.data_y)
    o = oracle.run(*args, inst.data_z, qx, qy, inst.k, inst.levels, inst.R_min, inst.R_max,
                   inst.area)
    s = oracle.run(*args, np.abs(inst.data_z), qx, qy, inst.k, inst.levels, inst.R_min,
                   inst.R_max, inst.area)
    return o, s


def rel_err(got, want, scale):
    diff = np.abs(np.asarray(got, dtype=np.float64) - want)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(scale > 0, diff / scale, np.where(diff == 0, 0.0, np.inf))


def check_against_scan(ctx, torch, inst, idx=None):
    g_out, g_r, g_a = run(ctx, torch, inst, aidw.AIDW_FLAG_GRID_KNN)
    s_out, s_r, s_a = run(ctx, torch, inst, 0)
    assert np.array_equal(g_r, s_r), "r_obs differs from the full scan"
    assert np.array_equal(g_a, s_a), "alpha differs from the full scan"
    o, scale = ref(inst, idx)
    got = g_out if idx is None else g_out[idx]
    err = rel_err(got, o, scale)
    assert err.max() <= TOL_F32
    return g_out, s_out, err.max()


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
@pytest.mark.parametrize("m,n,k", [(1, 5, 1), (3, 70, 2), (257, 300, 8), (5003, 1001, 15),
                                   (20000, 4099, 32)])
def test_grid_matches_full_scan_and_oracle(ctx, torch, kind, m, n, k):
    if kind == "uniform":
        inst = workloads.uniform_unit(m=m, n=n, k=k, seed=m + 7 * n, dtype=np.float32)
    else:
        inst = workloads.clustered(m=m, n=n, seed=m + n, k=k, on_point=0.05)
    if m == 1:
        inst.area = 1.0
    _, _, e = check_against_scan(ctx, torch, inst)
    say("grid %s m=%d n=%d k=%d: max err %.3e" % (kind, m, n, k, e))


def _custom(data_x, data_y, query_x, query_y, k, area=None, seed=0):
    inst = workloads.uniform_unit(m=len(data_x), n=len(query_x), k=k, seed=seed,
                                  dtype=np.float32)
    inst.data_x = np.ascontiguousarray(data_x, dtype=np.float32)
    inst.data_y = np.ascontiguousarray(data_y, dtype=np.float32)
    rng = np.random.default_rng(seed)
    inst.data_z = rng.standard_normal(len(data_x)).astype(np.float32)
    inst.query_x = np.ascontiguousarray(query_x, dtype=np.float32)
    inst.query_y = np.ascontiguousarray(query_y, dtype=np.float32)
    inst.area = area if area is not None else max(workloads.bbox_area(inst.data_x, inst.data_y),
                                                  1e-6)
    return inst


def test_grid_queries_far_outside_the_data(ctx, torch):
    rng = np.random.default_rng(41)
    dx, dy = rng.random(3000), rng.random(3000)
    qx = np.concatenate([rng.uniform(-50, 50, 500), [1e4, -1e4, 0.5, 0.5, 1e-3]])
    qy = np.concatenate([rng.uniform(-50, 50, 500), [0.5, 0.5, 1e4, -1e4, -1e3]])
    check_against_scan(ctx, torch, _custom(dx, dy, qx, qy, 10))


@pytest.mark.parametrize("shape", ["vertical", "horizontal", "point", "thin"])
def test_grid_degenerate_extents(ctx, torch, shape):
    rng = np.random.default_rng(43)
    m = 4000
    t = rng.random(m)
    if shape == "vertical":  # every point at x = 0.25
        dx, dy = np.full(m, 0.25), t
    elif shape == "horizontal":
        dx, dy = t, np.full(m, -3.0)
    elif shape == "point":  # all coincident
        dx, dy = np.full(m, 0.5), np.full(m, 0.5)
    else:  # a 1000:1 strip
        dx, dy = t * 1000.0, rng.random(m)
    qx = np.concatenate([rng.uniform(-2, 2, 300), dx[:20]])
    qy = np.concatenate([rng.uniform(-2, 2, 300), dy[:20]])
    check_against_scan(ctx, torch, _custom(dx, dy, qx, qy, 12, area=1.0))


def test_grid_duplicates_and_on_point_queries(ctx, torch):
    rng = np.random.default_rng(47)
    base_x, base_y = rng.random(800), rng.random(800)
    dx = np.concatenate([base_x, base_x[:300], base_x[:50]])  # points repeated up to 3 times
    dy = np.concatenate([base_y, base_y[:300], base_y[:50]])
    qx = np.concatenate([rng.random(200), base_x[::7]])
    qy = np.concatenate([rng.random(200), base_y[::7]])
    check_against_scan(ctx, torch, _custom(dx, dy, qx, qy, 8))


def test_grid_rejects_knn_idx(ctx, torch):
    inst = workloads.uniform_unit(m=100, n=10, k=4, seed=5, dtype=np.float32)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    out = torch.zeros(inst.n, device="cuda")
    knn = torch.empty((inst.n, inst.k), dtype=torch.int32, device="cuda")
    ctx.bind_current_stream()
    p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, area=inst.area, knn_idx=knn,
                    flags=aidw.AIDW_FLAG_GRID_KNN)
    assert aidw.aidw_interpolate_ex(ctx.h, p) == aidw.AIDW_EINVAL


def test_grid_paper_scale_full_size(ctx, torch):
    inst = workloads.paper_scale()  # m = n = 2^20, k = 15
    idx = np.sort(np.random.default_rng(14).choice(inst.n, 120, replace=False))
    _, _, e = check_against_scan(ctx, torch, inst, idx)
    say("grid paper scale: max err %.3e over %d sampled queries" % (e, len(idx)))


def test_grid_clustered_full_size(ctx, torch):
    inst = workloads.clustered()  # m = n = 2^18, k = 10, Gaussian mixture
    on = inst.meta["on_point_queries"]
    idx = np.sort(np.concatenate([np.random.default_rng(15).choice(inst.n, 100, replace=False),
                                  on[:30]]))
    _, _, e = check_against_scan(ctx, torch, inst, idx)
    say("grid clustered: max err %.3e over %d sampled queries" % (e, len(idx)))
