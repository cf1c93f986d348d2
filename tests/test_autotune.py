"""The autotuner's cache logic (host only) and, on the GPU, that every update plan it
chooses among gives the oracle's counters and that a tuned plan round-trips."""
import json

import numpy as np
import pytest

import oracle
import paper_1711_00975_amd as csk
from paper_1711_00975_amd import autotune


def test_cache_round_trip_and_classes(tmp_path):
    path = str(tmp_path / "tune.json")
    t = autotune.Tuner(path, device="dev-A")
    assert autotune.size_class(1 << 16, 70_000) == "w16_n16"
    assert autotune.size_class(1 << 20, 1) == "w20_n0"
    t.record("w16_n16", {"mode": csk.CSK_UPDATE_DIRECT, "max_wg": 0, "ms": 0.1})
    t.save()
    t2 = autotune.Tuner(path, device="dev-A")
    assert t2.lookup("w16_n16")["mode"] == csk.CSK_UPDATE_DIRECT
    assert autotune.Tuner(path, device="dev-B").lookup("w16_n16") is None   # keyed by device
    assert json.load(open(path))["dev-A"]["w16_n16"]["max_wg"] == 0


@pytest.mark.gpu
@pytest.mark.parametrize("plan", autotune.UPDATE_CANDIDATES + [autotune._plan(csk.CSK_UPDATE_AUTO)],
                         ids=autotune.plan_key)
def test_every_update_plan_matches_oracle(plan):
    # the plans differ only in speed: the counters are the same +-1 sums (Sec. 2.2 Add)
    from test_gpu_parity import clustered, dev
    for w in (1 << 16, 1 << 20):
        pos = clustered(120_000, 100.0, 5)
        s = csk.Sketch(5, w, 3)
        autotune.set_plan(s, plan)
        s.update(dev(pos), 0.1, 100.0)
        Mo, _ = oracle.sketch(pos, 5, w, 3, 0.1, 100.0, threads=8)
        assert np.array_equal(s.counters().cpu().numpy(), Mo), w
        s.close()


def test_old_cache_entries_still_apply(tmp_path):
    # a plan cached before the tiling axes (mode and max_wg only) keys and applies as before
    t = autotune.Tuner(str(tmp_path / "tune.json"), device="dev-A")
    t.record("w14_n16", {"mode": csk.CSK_UPDATE_BINNED, "max_wg": 64, "ms": 0.2})
    assert autotune.plan_key(autotune._plan(csk.CSK_UPDATE_BINNED, 64)) == "1:64:0:0:0:0"
    assert t.lookup("w14_n16")["max_wg"] == 64


@pytest.mark.gpu
def test_tuner_end_to_end(tmp_path):
    t = autotune.Tuner(str(tmp_path / "tune.json"))
    plan = t.tune_update(5, 1 << 20, 300_000, reps=2)
    keys = [autotune.plan_key(p) for p in autotune.UPDATE_CANDIDATES]
    assert autotune.plan_key(plan) in keys
    assert set(plan["all_ms"]) <= set(keys) and len(plan["all_ms"]) >= 5
    t.save()
    s = csk.Sketch(5, 1 << 20, 9)
    assert autotune.Tuner(str(tmp_path / "tune.json")).apply(s, 300_000)
    s.close()
