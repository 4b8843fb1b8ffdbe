"""The autotuner on the GPU: it measures every leaf size on a request and the
leaf it picks gives results identical to a plain call at that leaf size."""
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


def test_tuner_measures_all_leaf_sizes_and_serving_uses_its_choice(sph, tmp_path):
    w = W.blob_in_lattice(14, seed=9)
    req = S.Request(0, 0.0, "evaluate", w.arrays, w.setup, precision=0)
    tuner = T.LeafTuner(path=str(tmp_path / "t.json"), reps=1)
    print("case: tune N=%d" % w.n, flush=True)
    g = tuner.choose(req)
    entry = tuner.table[tuner.key(req)]
    assert g in T.LEAF_SIZES and set(entry["seconds"]) == {"8", "16", "32"}
    assert all(v > 0 for v in entry["seconds"].values())
    recs, _ = S.serve([req], 1 << 30, 1, "streams", leaf_for=tuner, keep_outputs=True)
    with sph.Context(sph.Params.from_setup(w.setup, precision=0, leaf_size=g)) as ctx:
        p = sph.Particles.from_host(w.arrays)
        ctx.evaluate(p)
        ctx.sync()
        ref = p.host(*S.GpuExecutor.OUT_EVAL)
    for f in S.GpuExecutor.OUT_EVAL:
        assert np.array_equal(recs[0].outputs[f], ref[f]), f
