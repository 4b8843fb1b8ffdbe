"""Launch-shape autotuner (host logic, synthetic timer; no GPU)."""
import json

import pytest

from paper_1709_04488_amd import serve as S
from paper_1709_04488_amd import tune as T
from paper_1709_04488_amd import workloads as W


def _req(rid, side, precision=0, kind="evaluate"):
    w = W.jittered_lattice(side, seed=rid)
    return S.Request(rid, 0.0, kind, w.arrays, w.setup, precision=precision, nsteps=2)


def test_class_keys_group_by_kind_precision_boundary_and_size():
    assert T.request_class("evaluate", 0, True, 4096) == T.request_class("evaluate", 0, True, 5000)
    assert T.request_class("evaluate", 0, True, 4096) != T.request_class("evaluate", 1, True, 4096)
    assert T.request_class("evaluate", 0, True, 4096) != T.request_class("integrate", 0, True, 4096)
    assert T.request_class("evaluate", 0, True, 4096) != T.request_class("evaluate", 0, False, 4096)
    assert T.request_class("evaluate", 0, True, 4096) != T.request_class("evaluate", 0, True, 32768)


def _separable_timer(calls, leaf_cost, stage_cost, claim_cost):
    """A synthetic time that is a sum of one term per knob."""
    def timer(arrays, setup, precision, shape):
        calls.append((arrays["x"].size, precision, T.shape_key(shape)))
        return (leaf_cost[precision][shape["leaf"]] + stage_cost[shape["stage"]]
                + claim_cost[shape["claim"]])
    return timer


def test_coordinate_descent_finds_each_knob(tmp_path):
    calls = []
    timer = _separable_timer(calls, {0: {8: 1.0, 16: 1.2, 32: 3.0}, 1: {8: 1.1, 16: 1.0, 32: 2.5}},
                             {"full": 0.3, "half": 0.1}, {1: 0.05, 4: 0.0})
    path = tmp_path / "tune.json"
    t = T.LaunchTuner(timer=timer, path=str(path))
    assert t.shape(_req(1, 16, 0)) == {"leaf": 8, "stage": "half", "claim": 4}
    assert t.shape(_req(2, 16, 1)) == {"leaf": 16, "stage": "half", "claim": 4}
    # per class: 3 leaf sizes, then 1 more stage, then 1 more claim
    assert len(calls) == 10
    # same classes again: no new measurement
    assert t.choose(_req(3, 16, 0)) == 8
    assert t.choose(_req(4, 16, 1)) == 16
    assert len(calls) == 10
    # the table persists and is reused by a new tuner
    data = json.loads(path.read_text())
    assert {v["leaf"] for v in data.values()} == {8, 16}
    assert {v["stage"] for v in data.values()} == {"half"}
    t2 = T.LaunchTuner(timer=lambda *a: 1 / 0, path=str(path))
    assert t2.shape(_req(5, 16, 0)) == {"leaf": 8, "stage": "half", "claim": 4}


def test_knobs_are_chosen_independently():
    # the best stage and claim differ from their defaults while the leaf stays
    calls = []
    timer = _separable_timer(calls, {0: {8: 2.0, 16: 1.0, 32: 1.5}},
                             {"full": 0.0, "half": 0.2}, {1: 0.1, 4: 0.0})
    t = T.LaunchTuner(timer=timer)
    assert t.shape(_req(1, 12)) == {"leaf": 16, "stage": "full", "claim": 4}
    entry = t.table[t.key(_req(1, 12))]
    assert set(entry["seconds"]) == {"g8/full/c1", "g16/full/c1", "g32/full/c1", "g16/half/c1",
                                     "g16/full/c4"}


def test_ties_go_to_the_defaults():
    t = T.LaunchTuner(timer=lambda a, s, p, sh: 1.0)
    assert t.shape(_req(1, 8)) == {"leaf": 8, "stage": "full", "claim": 1}


def test_stage_and_params_mapping():
    assert T.stage_leaves(8, "full") == 0 and T.stage_leaves(8, "half") == 8
    assert T.stage_leaves(16, "half") == 4 and T.stage_leaves(32, "half") == 2
    assert T.params_kw({"leaf": 32, "stage": "half", "claim": 4}) == \
        {"leaf_size": 32, "stage_leaves": 2, "claim_leaves": 4}
    with pytest.raises(ValueError):
        T.stage_leaves(16, "deep")


def test_stale_table_entries_are_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"evaluate/p0/per/n2^12": {"leaf": 12, "stage": "full",
                                                          "claim": 1}}))
    calls = []
    timer = _separable_timer(calls, {0: {8: 1.0, 16: 2.0, 32: 3.0}}, {"full": 0.0, "half": 0.1},
                             {1: 0.0, 4: 0.1})
    t = T.LaunchTuner(timer=timer, path=str(path))
    assert t.choose(_req(1, 16)) == 8 and len(calls) == 5


def test_objectives_keep_separate_table_entries(tmp_path):
    path = tmp_path / "tune.json"
    calls = []
    timer = _separable_timer(calls, {0: {8: 1.0, 16: 2.0, 32: 3.0}}, {"full": 0.0, "half": 0.1},
                             {1: 0.0, 4: 0.1})
    lat = T.LaunchTuner(timer=timer, path=str(path))
    thr = T.LaunchTuner(timer=timer, path=str(path), objective="throughput")
    r = _req(1, 16)
    assert lat.key(r) != thr.key(r) and thr.key(r).endswith("/throughput")
    lat.choose(r)
    thr.load(str(path))
    assert thr.key(r) not in thr.table        # a latency entry is not reused
    thr.choose(r)
    assert len(calls) == 10
    with pytest.raises(ValueError):
        T.LaunchTuner(timer=timer, objective="fastest")


def test_serving_tuner_keeps_the_leaf_sizes_that_fit_a_slot_share():
    # C3-like: the largest set is 58^3; one slot in three of 1 GiB holds its
    # G = 8 and G = 16 footprints but not G = 32's (twice the candidate-list
    # scratch of G = 16); a 16 GiB budget holds all three
    reqs = [_req(1, 20), _req(2, 58)]
    t = S.serving_tuner(reqs, 1 << 30, 3)
    assert t.sizes == (8, 16) and t.objective == "throughput"
    assert S.serving_tuner(reqs, 16 << 30, 3).sizes == T.LEAF_SIZES
    # nothing fits: the smallest leaf size is still tried
    assert S.serving_tuner(reqs, 1 << 20, 3).sizes == (8,)
