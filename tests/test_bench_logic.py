"""Host logic of bench.py (no GPU): the roofline figures it derives and the
committed counter records it quotes, which must be dropped once the pair-loop
source has changed since they were taken."""
import hashlib
import importlib.util
import json
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_peaks_are_the_published_vector_rates():
    b = _bench()
    assert b.PEAK_TFLOPS["fp64"] == 78.6
    assert b.PEAK_TFLOPS["fp32"] == 157.3


def test_roofline_uses_the_longest_pair_loop():
    b = _bench()
    res = {"info": {"dens_pair_evals": 1_000_000, "force_pair_evals": 3_000_000},
           "kernel_ms": {"density": 2.0, "force": 1.0, "build": 0.1}}
    r = b.roofline(res, "fp64")
    flops = 1_000_000 * b.DENS_FLOPS_PER_PAIR_ITER
    assert r["kernel"] == "density" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["flops_per_launch"] == flops
    assert r["achieved"] == pytest.approx(flops / 2e-3 / 1e12, abs=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, abs=1e-4)
    assert r["traffic"] is None and r["valu_issue_frac"] is None
    other = r["other_kernel"]["force"]
    assert other["flops_per_launch"] == 3_000_000 * b.FORCE_FLOPS_PER_PAIR
    res["kernel_ms"] = {"density": 1.0, "force": 2.0, "build": 0.1}
    assert b.roofline(res, "fp32")["kernel"] == "force"


PAIR_SOURCES = ("pairs.hpp", "pairs_args.hpp")


def _sources():
    return {f: open(os.path.join(ROOT, "paper_1709_04488_amd", "csrc", f), "rb").read()
            for f in PAIR_SOURCES}


def _tree(tmp_path, texts):
    d = tmp_path / "tree"
    (d / "profiles").mkdir(parents=True)
    (d / "paper_1709_04488_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "traffic.json"), d / "profiles" / "traffic.json")
    for f, t in texts.items():
        (d / "paper_1709_04488_amd" / "csrc" / f).write_bytes(t)
    return str(d)


def test_counter_records_follow_the_pair_loop_source(tmp_path):
    b = _bench()
    recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    src = _sources()
    digest = hashlib.sha256(b"".join(src[f] for f in PAIR_SOURCES)).hexdigest()
    tag = next(iter(recs))
    want = recs[tag]["bytes_per_launch"]["density_cold"]
    # a tree whose pair-kernel sources are the ones the record names: quoted
    if recs[tag]["pairs_source_sha256"] == digest:
        b.ROOT = _tree(tmp_path / "same", src)
        assert b.measured_traffic(tag, "density_cold") == int(round(want["read"] + want["written"]))
        assert b.measured_valu_insts(tag, "density_cold") is not None
    # any edit of either file, a comment included: dropped
    for f in PAIR_SOURCES:
        b.ROOT = _tree(tmp_path / ("edited_" + f), {**src, f: src[f] + b"\n// edited\n"})
        assert b.measured_traffic(tag, "density_cold") is None
        assert b.measured_valu_insts(tag, "density_cold") is None
    # unknown workload, precision or leaf size: nothing
    b.ROOT = _tree(tmp_path / "none", src)
    assert b.measured_traffic("c9_fp64_g16", "density_cold") is None


def test_counter_record_key_names_workload_precision_leaf_and_conductivity():
    import argparse
    b = _bench()
    a = argparse.Namespace(config="c1", alpha_ac=0.0, ac_signal="wadsley",
                           leaf_used={"fp64": {"leaf": 16, "stage": "full", "claim": 1},
                                      "fp32": {"leaf": 32, "stage": "half", "claim": 4}})
    assert b.prof_tag(a, "fp64") == "c1_fp64_g16"
    assert b.prof_tag(a, "fp32") == "c1_fp32_g32"
    a.alpha_ac = 1.0
    assert b.prof_tag(a, "fp64") == "c1_fp64_g16_ac1wadsley"


def test_flops_per_pair_counts_the_kernel_and_conductivity():
    b = _bench()
    assert b.flops_per_pair({}) == (b.DENS_FLOPS_PER_PAIR_ITER, b.FORCE_FLOPS_PER_PAIR)
    assert b.flops_per_pair({"kernel": 1}) == (36, 78)
    assert b.flops_per_pair({"alpha_ac": 1.0, "ac_signal": 0}) == (26, 74)
    assert b.flops_per_pair({"alpha_ac": 1.0, "ac_signal": 1, "kernel": 1}) == (36, 94)
    assert b.flops_per_pair({"alpha_ac": 0.0, "ac_signal": 1}) == (26, 64)
