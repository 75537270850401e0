"""The speculative single pass of the unsplit FP32-scaled kernel.

When alpha_5 is a whole power, pass 1 also forms the unscaled pass-2 sums of
that power; queries that end at alpha_5 are done after one scan, the others
get pass 2 afterwards in data segments.  These tests force the
unsplit launch (split_segments = 1) so that small problems take that path, and
check it against the FP64 oracle and against the two-pass kernel (the
deterministic handle runs that one), with tiles that keep the speculation,
tiles that lose it, and problems where it is never tried.
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


@pytest.fixture(scope="module")
def ctx_det(torch):
    c = aidw.Context(0, deterministic=1)
    yield c
    c.close()


def say(msg):
    print(msg, flush=True)


def run(c, inst, split=1, levels=None):
    """(out, r_obs, alpha) of an unsplit launch on handle c."""
    data_xy, data_z, query_xy = aidw.to_device(inst)
    c.set_tuning(0, 0, split)
    try:
        out, r_obs, alpha, _ = c.interpolate(data_xy, data_z, query_xy, inst.k,
                                             levels or inst.levels, inst.R_min, inst.R_max,
                                             inst.area, diag=True, knn=False)
    finally:
        c.set_tuning(0)
    return out.cpu().numpy(), r_obs.cpu().numpy(), alpha.cpu().numpy()


def oracle_check(inst, out, idx=None, levels=None):
    idx = np.arange(inst.n) if idx is None else idx
    lv = levels or inst.levels
    args = (inst.data_x, inst.data_y)
    want, _, a_ref, _ = oracle.run(*args, inst.data_z, inst.query_x[idx], inst.query_y[idx], inst.k,
                                   lv, inst.R_min, inst.R_max, inst.area, diag=True)
    scale = oracle.run(*args, np.abs(inst.data_z), inst.query_x[idx], inst.query_y[idx], inst.k,
                       lv, inst.R_min, inst.R_max, inst.area)
    err = float(np.max(np.abs(out[idx].astype(np.float64) - want) / scale))
    return err, a_ref


def tile_order(c, inst):
    """The queries' tile order in these launches: the spatial order (as
    aidw_query_order gives it) when there is more than one tile and at least
    1024 data points, else the caller's order."""
    import torch

    if inst.m < 1024 or inst.n <= 64:
        return np.arange(inst.n)
    q = torch.from_numpy(inst.query_xy()).cuda()
    order = torch.empty(inst.n, dtype=torch.int32, device="cuda")
    c.bind_current_stream()
    aidw.check(aidw.aidw_query_order(c.h, q, inst.n, order))
    return order.cpu().numpy()


def tile_flags(alpha, order, power=5.0):
    """Per tile (64 consecutive positions of the order): some query off the power."""
    a = alpha[order]
    pad = (-a.size) % 64
    a = np.concatenate([a, np.full(pad, power)])
    return (a.reshape(-1, 64) != power).any(axis=1)


def failing_tiles(alpha, order, power=5.0):
    return int(np.sum(tile_flags(alpha, order, power)))


def test_mixed_tiles_match_oracle_and_two_pass(ctx, ctx_det):
    # a dense patch: 21 of 32 tiles leave the alpha_5 range, 11 keep it
    inst = workloads.dense_patch()
    say("speculative pass: dense patch m=%d n=%d k=%d" % (inst.m, inst.n, inst.k))
    out, r_obs, alpha = run(ctx, inst)
    err, a_ref = oracle_check(inst, out)
    order = tile_order(ctx, inst)
    fails = failing_tiles(a_ref, order)
    say("  tiles off alpha_5: %d of %d, max rel err vs oracle %.3e" % (fails, -(-inst.n // 64), err))
    assert 0 < fails < -(-inst.n // 64)  # both kinds of tile are exercised
    assert err <= TOL_F32
    # pass 1 is the same multiset scan: r_obs and alpha are bit-identical
    out2, r2, a2 = run(ctx_det, inst)
    assert np.array_equal(r_obs, r2) and np.array_equal(alpha, a2)
    # tiles whose queries all kept the speculation reproduce the two-pass
    # sums bit for bit; in the other tiles a query that kept it has the sums
    # of a whole-power wave, and a deferred one adds its data segments in
    # another grouping
    keep = np.zeros(inst.n, dtype=bool)
    keep[order] = np.repeat(~tile_flags(alpha, order), 64)[: inst.n]
    assert keep.any()
    assert np.array_equal(out[keep], out2[keep])
    scale = np.max(np.abs(out2))
    assert np.max(np.abs(out.astype(np.float64) - out2)) <= 1e-6 * scale


def test_kept_queries_of_failed_tiles(ctx, ctx_det):
    # In a tile where one query ends just below alpha_5, the other 63 keep
    # their speculative sums: bit for bit what the two-pass kernel gives them
    # in waves of alpha_5 queries only (a problem of those queries alone),
    # where the two-pass kernel on the mixed tiles takes the general loop.
    # A tile whose early check gives the speculation up (on 1/32 of the
    # points, so now and then for a near miss) runs pass 2 deferred instead.
    # R_max = 3.5 puts R_90 (mu_R = 0.9) in the bulk of the R distribution of
    # uniform data, so near misses abound; the other queries are taken well
    # above it, and tiles are laid out in the caller's order.
    import copy

    base = workloads.uniform_unit(1 << 16, 20000, seed=33, k=15)
    base.R_max = 3.5
    _, r_all, a_all = run(ctx, base)
    r90 = r_all[a_all == 5.0].min()
    on = np.flatnonzero((a_all == 5.0) & (r_all >= 1.3 * r90))
    near = np.flatnonzero((a_all >= 4.95) & (a_all < 5.0))
    tiles = 16
    assert on.size >= 63 * tiles and near.size >= tiles
    pick = []
    for t in range(tiles):
        lanes = list(on[63 * t: 63 * (t + 1)])
        lanes.insert(17, near[t])
        pick.extend(lanes)
    pick = np.asarray(pick)
    inst = copy.copy(base)
    inst.query_x = np.ascontiguousarray(base.query_x[pick])
    inst.query_y = np.ascontiguousarray(base.query_y[pick])
    data_xy, data_z, query_xy = aidw.to_device(inst)
    res = []
    for speculate in (0, 1):  # unsplit, caller's order: speculative, two-pass
        ctx.set_tuning(0, 0, 1, speculate, 1)
        try:
            o, _, a, _ = ctx.interpolate(data_xy, data_z, query_xy, inst.k, inst.levels,
                                         inst.R_min, inst.R_max, inst.area, diag=True,
                                         knn=False)
        finally:
            ctx.set_tuning(0)
        res.append((o.cpu().numpy(), a.cpu().numpy()))
    (out, alpha), (two, alpha2) = res
    assert np.array_equal(alpha, alpha2)
    kept = alpha == 5.0
    assert kept.sum() == 63 * tiles and np.all(~kept[17::64])
    sub = copy.copy(inst)
    sub.query_x = np.ascontiguousarray(inst.query_x[kept])
    sub.query_y = np.ascontiguousarray(inst.query_y[kept])
    out_sub, _, alpha_sub = run(ctx_det, sub)
    assert np.all(alpha_sub == 5.0)
    alone = np.full(inst.n, np.nan, dtype=np.float32)
    alone[kept] = out_sub
    same = ((out == alone) | ~kept).reshape(tiles, 64).all(axis=1)
    differs = ((out != two) & kept).reshape(tiles, 64).any(axis=1)
    say("tiles whose alpha_5 queries kept their sums: %d of %d" % ((same & differs).sum(), tiles))
    assert (same & differs).sum() >= tiles // 2
    assert np.allclose(out, two, rtol=1e-5, atol=1e-6 * np.abs(two).max())
    err, _ = oracle_check(inst, out, np.arange(17, inst.n, 64))  # the near misses
    assert err <= TOL_F32
    err, _ = oracle_check(inst, out, np.arange(0, inst.n, 37))
    assert err <= TOL_F32


def test_deferred_queries_repeat_bit_for_bit(ctx):
    # the deferred queries are listed in position order, so which of them
    # share a deferred wave (and the pass-2 loop the wave takes) does not
    # depend on the order in which tiles finish: runs repeat bit for bit
    inst = workloads.dense_patch(m=20000, n=3000, seed=34, k=15)
    outs = [run(ctx, inst)[0] for _ in range(3)]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_every_tile_deferred(ctx):
    # clustered data with k = 8: few tiles keep alpha_5 everywhere
    inst = workloads.clustered(m=8192, n=1000, seed=21, k=8)
    out, _, alpha = run(ctx, inst)
    err, a_ref = oracle_check(inst, out)
    say("clustered k=8: tiles off alpha_5 %d of %d, err %.3e" % (
        failing_tiles(a_ref, tile_order(ctx, inst)), -(-inst.n // 64), err))
    assert err <= TOL_F32


def test_many_deferred_tiles_in_l2_segments(ctx, torch):
    # More failed tiles than target / 7 (target: one round of waves) over
    # m = 2^20, where the deferred pass 2 cuts the data into eight L2-sized
    # segments: count * 8 (tile, segment) items, more than target + count.
    # Every item must run, and every deferred query come out right.
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    target = cus * 4 * 8
    n = 64 * (target // 7 + 256)
    inst = workloads.dense_patch(m=1 << 20, n=n, seed=32, k=15, patch_queries=1.0)
    say("speculative pass: every query in the dense patch, m=%d n=%d" % (inst.m, inst.n))
    out, _, alpha = run(ctx, inst)
    fails = failing_tiles(alpha, tile_order(ctx, inst))
    say("  tiles off alpha_5: %d of %d (deferred items %d, one round %d)"
        % (fails, -(-inst.n // 64), 8 * fails, target))
    assert 8 * fails > target + fails
    assert not np.isnan(out).any()
    idx = np.unique(np.linspace(0, inst.n - 1, 48).astype(np.int64))
    err, _ = oracle_check(inst, out, idx)
    say("  max rel err vs oracle %.3e" % err)
    assert err <= TOL_F32


def test_no_tile_deferred(ctx):
    inst = workloads.uniform_unit(1 << 16, 1 << 12, seed=22, k=15)
    out, _, alpha = run(ctx, inst)
    idx = np.linspace(0, inst.n - 1, 128).astype(np.int64)
    err, _ = oracle_check(inst, out, idx)
    say("uniform k=15: queries off alpha_5 %d, err %.3e" % (int(np.sum(alpha != 5.0)), err))
    assert err <= TOL_F32


@pytest.mark.parametrize("levels", [(1, 2, 3, 4, 2.5), (0.5, 1, 1.5, 2, 2)])
def test_other_powers(ctx, ctx_det, levels):
    # alpha_5 = 2.5 is not whole: no speculation, the two-pass kernel runs;
    # alpha_5 = 2 is: speculation with A = 2
    inst = workloads.dense_patch(m=8192, n=1500, seed=23, k=10)
    out, _, alpha = run(ctx, inst, levels=levels)
    out2, _, _ = run(ctx_det, inst, levels=levels)
    err, _ = oracle_check(inst, out, levels=levels)
    assert err <= TOL_F32
    if levels[4] != int(levels[4]):
        assert np.array_equal(out, out2)


def test_ragged_and_small(ctx):
    # m just above the speculation threshold, n not a multiple of 64, and a
    # data count that leaves a ragged batch tail
    for m, n in ((1024, 65), (1037, 1), (3001, 777)):
        inst = workloads.uniform_unit(m, n, seed=24 + m, k=15)
        out, _, _ = run(ctx, inst)
        err, _ = oracle_check(inst, out)
        say("m=%d n=%d err %.3e" % (m, n, err))
        assert err <= TOL_F32


def test_noalloc_takes_the_same_path(ctx, torch):
    inst = workloads.dense_patch(m=8192, n=1200, seed=25, k=15)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    outs = []
    for entry in (aidw.aidw_interpolate_ex, aidw.aidw_interpolate_noalloc):
        out = torch.full((inst.n,), np.nan, dtype=torch.float32, device="cuda")
        ctx.set_tuning(0, 0, 1)
        try:
            ctx.bind_current_stream()
            p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min,
                            inst.R_max, inst.area)
            assert entry(ctx.h, p) == aidw.AIDW_OK, aidw.last_error(ctx.h)
        finally:
            ctx.set_tuning(0)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("segments", [3, 8])
def test_split_speculation_is_bit_identical(ctx, segments):
    # in the split kernels (speculate = 2) a pass-1 item's speculative sums
    # are the sums its pass-2 item would write, so the output does not depend
    # on which tiles kept the speculation.  Both runs in the caller's order:
    # without speculation split pass 2 would otherwise regroup its waves by
    # loop, which changes rounding
    inst = workloads.dense_patch(m=20000, n=2500, seed=26 + segments, k=15)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    res = []
    for speculate in (2, 1):
        ctx.set_tuning(0, 0, segments, speculate, 1)
        try:
            res.append(tuple(t.cpu().numpy() for t in ctx.interpolate(
                data_xy, data_z, query_xy, inst.k, inst.levels, inst.R_min, inst.R_max, inst.area,
                diag=True, knn=False)[:3]))
        finally:
            ctx.set_tuning(0)
    (o0, r0, a0), (o1, r1, a1) = res
    assert np.array_equal(r0, r1) and np.array_equal(a0, a1)
    assert np.array_equal(o0, o1)
    err, a_ref = oracle_check(inst, o0)
    fails = failing_tiles(a_ref, np.arange(inst.n))
    say("split %d: tiles off alpha_5 %d of %d, err %.3e" % (segments, fails, -(-inst.n // 64), err))
    assert 0 < fails < -(-inst.n // 64)
    assert err <= TOL_F32


def test_speculate_off_gives_the_two_pass_kernel(ctx, ctx_det, torch):
    inst = workloads.dense_patch(m=8192, n=1500, seed=31, k=15)
    data_xy, data_z, query_xy = aidw.to_device(inst)
    out = torch.empty(inst.n, dtype=torch.float32, device="cuda")
    ctx.set_tuning(0, 0, 1, 1)
    try:
        p = ctx.problem(data_xy, data_z, query_xy, inst.k, out, inst.levels, inst.R_min,
                        inst.R_max, inst.area)
        assert "aidw_f32_fused<16, 1, false>" in aidw.aidw_describe_launch(ctx.h, p)
        ctx.bind_current_stream()
        aidw.check(aidw.aidw_interpolate_ex(ctx.h, p))
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning(0)
    two_pass, _, _ = run(ctx_det, inst)
    assert np.array_equal(out.cpu().numpy(), two_pass)
