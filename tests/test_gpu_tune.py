"""The launch-shape autotuner on the GPU.

* It times the leaf sizes, then the other stage depth, then the other claim
  size (coordinate descent), and serving runs the shape it picks: results
  identical to a plain call with that shape.
* Every launch shape computes the same thing: the claim size never changes a
  bit; the stage depth leaves the density results unchanged and moves the
  force sums only in their last bits (the split of a particle's terms over
  its lanes); all shapes match the oracle within the FP64 tolerance.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1709_04488_amd import serve as S  # noqa: E402
from paper_1709_04488_amd import tune as T  # noqa: E402
from paper_1709_04488_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04488_amd import sph as s
    s.load()
    return s


def _eval(sph, w, precision, shape):
    params = sph.Params.from_setup(w.setup, precision=precision, **T.params_kw(shape))
    with sph.Context(params) as ctx:
        p = sph.Particles.from_host(w.arrays)
        ctx.evaluate(p)
        ctx.sync()
        return p.host(*S.GpuExecutor.OUT_EVAL)


def test_tuner_measures_the_knobs_and_serving_uses_its_choice(sph, tmp_path):
    w = W.blob_in_lattice(14, seed=9)
    req = S.Request(0, 0.0, "evaluate", w.arrays, w.setup, precision=0)
    tuner = T.LaunchTuner(path=str(tmp_path / "t.json"), reps=1)
    print("case: tune N=%d" % w.n, flush=True)
    shape = tuner.shape(req)
    entry = tuner.table[tuner.key(req)]
    assert shape["leaf"] in T.LEAF_SIZES and shape["stage"] in T.STAGES
    assert shape["claim"] in T.CLAIMS
    assert len(entry["seconds"]) == 5 and all(v > 0 for v in entry["seconds"].values())
    assert {f"g{g}/full/c1" for g in T.LEAF_SIZES} <= set(entry["seconds"])
    recs, _ = S.serve([req], 1 << 30, 1, "streams", leaf_for=tuner, keep_outputs=True)
    ref = _eval(sph, w, 0, shape)
    for f in S.GpuExecutor.OUT_EVAL:
        assert np.array_equal(recs[0].outputs[f], ref[f]), f


def test_throughput_tuner_times_batched_pair_loops(sph):
    w = W.jittered_lattice(12, seed=19)
    req = S.Request(0, 0.0, "evaluate", w.arrays, w.setup, precision=1)
    tuner = T.LaunchTuner(reps=1, objective="throughput")
    print("case: throughput tuning N=%d" % w.n, flush=True)
    shape = tuner.shape(req)
    entry = tuner.table[tuner.key(req)]
    assert tuner.key(req).endswith("/throughput")
    assert shape["leaf"] in T.LEAF_SIZES and len(entry["seconds"]) == 5
    assert all(v > 0 for v in entry["seconds"].values())
    # serving through the native executor with that choice: results are
    # those of a plain call with the same shape
    recs, _ = S.serve([req], 1 << 30, 3, "native", leaf_for=tuner, keep_outputs=True)
    ref = _eval(sph, w, 1, shape)
    for f in S.GpuExecutor.OUT_EVAL:
        assert np.array_equal(recs[0].outputs[f], ref[f]), f


@pytest.mark.parametrize("leaf", [8, 16, 32])
def test_every_launch_shape_computes_the_same(sph, orc, leaf):
    w = W.blob_in_lattice(13, seed=31)
    a = w.arrays
    ref = orc.evaluate(orc.Params(**w.setup), a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                       a["m"], a["u"], a["h"])
    print(f"case: launch shapes leaf={leaf} N={w.n}", flush=True)
    base = _eval(sph, w, 0, {"leaf": leaf, "stage": "full", "claim": 1})
    for stage in T.STAGES:
        for claim in (1, 3, 4):
            out = _eval(sph, w, 0, {"leaf": leaf, "stage": stage, "claim": claim})
            for k in ("h", "rho", "omega", "pressure", "cs", "nngb", "nforce"):
                assert np.array_equal(out[k], base[k]), (stage, claim, k)
            for k, sk in (("ax", "scale_a"), ("ay", "scale_a"), ("az", "scale_a"),
                          ("dudt", "scale_u")):
                if stage == "full":
                    assert np.array_equal(out[k], base[k]), (stage, claim, k)
                assert np.max(np.abs(out[k] - base[k]) / ref[sk]) < 1e-13, (stage, claim, k)
                assert np.max(np.abs(out[k] - ref[k]) / ref[sk]) < 1e-10, (stage, claim, k)
            assert np.array_equal(out["nforce"], ref["nforce"])


def test_fp32_launch_shapes_agree(sph):
    w = W.plummer(3000, seed=32)
    print("case: fp32 launch shapes", flush=True)
    base = _eval(sph, w, 1, {"leaf": 16, "stage": "full", "claim": 1})
    out = _eval(sph, w, 1, {"leaf": 16, "stage": "half", "claim": 4})
    for k in ("h", "rho", "omega", "nngb"):
        assert np.array_equal(out[k], base[k]), k
    scale = np.sqrt(base["ax"] ** 2 + base["ay"] ** 2 + base["az"] ** 2).max()
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(out[k] - base[k])) < 1e-5 * scale, k


def test_bad_launch_shapes_are_rejected(sph):
    for bad in ({"leaf_size": 32, "stage_leaves": 5}, {"stage_leaves": -1},
                {"claim_leaves": 65}, {"claim_leaves": -2}):
        with pytest.raises(sph.SphError) as e:
            sph.Context(sph.Params(**bad))
        assert e.value.code == sph.SPH_EINVAL, bad
