"""Leaf-size autotuner (host logic, synthetic timer; no GPU)."""
import json

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


def test_measures_once_per_class_and_keeps_the_fastest(tmp_path):
    calls = []

    def timer(arrays, setup, precision, leaf):
        calls.append((arrays["x"].size, precision, leaf))
        # FP64 favours small leaves, FP32 the middle one
        return {0: {8: 1.0, 16: 1.2, 32: 3.0}, 1: {8: 1.1, 16: 1.0, 32: 2.5}}[precision][leaf]

    path = tmp_path / "tune.json"
    t = T.LeafTuner(timer=timer, path=str(path))
    assert t.choose(_req(1, 16, 0)) == 8
    assert t.choose(_req(2, 16, 1)) == 16
    assert len(calls) == 6
    # same classes again: no new measurement
    assert t.choose(_req(3, 16, 0)) == 8
    assert t.choose(_req(4, 16, 1)) == 16
    assert len(calls) == 6
    # the table persists and is reused by a new tuner
    data = json.loads(path.read_text())
    assert {v["leaf"] for v in data.values()} == {8, 16}
    t2 = T.LeafTuner(timer=lambda *a: 1 / 0, path=str(path))
    assert t2.choose(_req(5, 16, 0)) == 8


def test_ties_go_to_the_smaller_leaf():
    t = T.LeafTuner(timer=lambda a, s, p, g: 1.0)
    assert t.choose(_req(1, 8)) == 8
