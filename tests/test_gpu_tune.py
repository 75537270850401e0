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
