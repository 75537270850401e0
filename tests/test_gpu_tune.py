"""The autotuner: it measures launch shapes for a size class, later calls in
that class use the winner (results unchanged up to the split's rounding), and
its table survives a save/load round trip."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1511_02186_amd import aidw, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


def test_tune_save_load_and_use(torch, tmp_path):
    ctx = aidw.Context(0)
    try:
        best = aidw.aidw_tune(ctx.h, 20000, 300, 10, budget_s=2.0)
        assert best["q_per_lane"] in (1, 2, 4) and best["split_segments"] >= 1
        assert best["speculate"] in (0, 2)
        assert best["speculate"] == 0 or best["split_segments"] > 1
        path = tmp_path / "tune.json"
        aidw.check(aidw.aidw_tune_save(ctx.h, path))
        table = json.loads(path.read_text())
        assert table["format"] == "libaidw-tuning-1" and len(table["entries"]) == 1
        e = table["entries"][0]
        assert (e["m_log2"], e["n_log2"], e["K"]) == (14, 8, 10)
    finally:
        ctx.close()
    ctx2 = aidw.Context(0)
    try:
        aidw.check(aidw.aidw_tune_load(ctx2.h, path))
        inst = workloads.uniform_unit(20000, 300, 8, 10)
        d = aidw.to_device(inst)
        out = ctx2.interpolate(*d, inst.k, area=inst.area).cpu().numpy()
        want = oracle.run(inst.data_x, inst.data_y, inst.data_z, inst.query_x, inst.query_y,
                          inst.k, area=inst.area)
        scale = oracle.run(inst.data_x, inst.data_y, np.abs(inst.data_z), inst.query_x,
                           inst.query_y, inst.k, area=inst.area)
        assert np.max(np.abs(out - want) / scale) <= 1e-4
        assert aidw.aidw_tune_load(ctx2.h, tmp_path / "missing.json") == aidw.AIDW_ENOTFOUND
        bad = tmp_path / "bad.json"
        bad.write_text('{"format": "libaidw-tuning-1", "entries": [\n'
                       '  {"m_log2": 3, "n_log2": 3, "K": 11, "q_per_lane": 1, '
                       '"max_waves_per_simd": 0, "split_segments": 1, "ms": 1.0}\n]}\n')
        assert aidw.aidw_tune_load(ctx2.h, bad) == aidw.AIDW_EINVAL
        other = tmp_path / "other.json"
        other.write_text("{}\n")
        assert aidw.aidw_tune_load(ctx2.h, other) == aidw.AIDW_EINVAL
        bad_spec = tmp_path / "bad_spec.json"
        bad_spec.write_text('{"format": "libaidw-tuning-1", "entries": [\n'
                            '  {"m_log2": 3, "n_log2": 3, "K": 10, "q_per_lane": 1, '
                            '"max_waves_per_simd": 0, "split_segments": 4, "speculate": 1, '
                            '"ms": 1.0}\n]}\n')
        assert aidw.aidw_tune_load(ctx2.h, bad_spec) == aidw.AIDW_EINVAL
        # an entry written without the speculate field still loads (as 0)
        old = tmp_path / "old.json"
        old.write_text('{"format": "libaidw-tuning-1", "entries": [\n'
                       '  {"m_log2": 3, "n_log2": 3, "K": 10, "q_per_lane": 1, '
                       '"max_waves_per_simd": 0, "split_segments": 1, "ms": 1.0}\n]}\n')
        aidw.check(aidw.aidw_tune_load(ctx2.h, old))
        again = tmp_path / "old_again.json"
        aidw.check(aidw.aidw_tune_save(ctx2.h, again))
        assert json.loads(again.read_text())["entries"][0]["speculate"] == 0
        aidw.check(aidw.aidw_tune_load(ctx2.h, path))
    finally:
        ctx2.close()
    # the same table through aidw_options.tune_path at creation
    ctx3 = aidw.Context(0, tune_path=path)
    try:
        p2 = tmp_path / "again.json"
        aidw.check(aidw.aidw_tune_save(ctx3.h, p2))
        assert json.loads(p2.read_text())["entries"] == table["entries"]
    finally:
        ctx3.close()
    aidw.Context(0, tune_path=tmp_path / "missing.json").close()  # a missing file is ignored
    with pytest.raises(aidw.AidwError) as ei:
        aidw.Context(0, tune_path=bad)
    assert ei.value.status == aidw.AIDW_EINVAL


def test_tune_rejects_bad_sizes(torch):
    ctx = aidw.Context(0)
    try:
        for m, n, k in [(0, 10, 1), (10, 0, 1), (10, 10, 0), (10, 10, 11), (100, 10, 33)]:
            with pytest.raises(aidw.AidwError) as ei:
                aidw.aidw_tune(ctx.h, m, n, k, 1.0)
            assert ei.value.status == aidw.AIDW_EINVAL
    finally:
        ctx.close()


def test_tuned_split_speculation_is_used(torch, tmp_path):
    # a tuned entry may ask for the speculative sums in the split kernels;
    # calls of that size class then run them (the result is bit-identical to
    # the split without them, in the same tiles) and stay within the bar
    inst = workloads.paper_scale(m=20000, n=300, seed=9, k=10)
    d = aidw.to_device(inst)
    outs = []
    for spec in (2, 0):
        path = tmp_path / ("t%d.json" % spec)
        path.write_text('{"format": "libaidw-tuning-1", "entries": [\n'
                        '  {"m_log2": 14, "n_log2": 8, "K": 10, "q_per_lane": 1, '
                        '"max_waves_per_simd": 0, "split_segments": 4, "speculate": %d, '
                        '"ms": 1.0}\n]}\n' % spec)
        ctx = aidw.Context(0, tune_path=path)
        # the caller's order: without speculation split pass 2 would regroup
        # its waves by loop, which changes rounding
        ctx.set_tuning(query_order=1)
        try:
            out = torch.empty(inst.n, device="cuda")
            p = ctx.problem(*d, inst.k, out, inst.levels, inst.R_min, inst.R_max, inst.area)
            assert "4 data segments" in aidw.aidw_describe_launch(ctx.h, p)
            outs.append(ctx.interpolate(*d, inst.k, inst.levels, inst.R_min, inst.R_max,
                                        inst.area).cpu().numpy())
        finally:
            ctx.close()
    assert np.array_equal(outs[0], outs[1])
    want = oracle.run(inst.data_x, inst.data_y, inst.data_z, inst.query_x, inst.query_y, inst.k,
                      area=inst.area)
    scale = oracle.run(inst.data_x, inst.data_y, np.abs(inst.data_z), inst.query_x,
                       inst.query_y, inst.k, area=inst.area)
    assert np.max(np.abs(outs[0] - want) / scale) <= 1e-4
