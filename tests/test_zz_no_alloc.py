"""sph_evaluate_noalloc (the entry point for callers that cannot allocate
device memory) against sph_evaluate, through the C ABI: two calls in a row
on one context, the second with a smaller set, each compared field by field
with sph_evaluate of the same set on a separate context.  The static array
is shared state, so the second call also shows that nothing of the first
call's contents leaks into it.  Results must be the same bits: the same
kernels run, only the persistent pair grid is capped by the static
candidate-list slices, and no result depends on which wave takes a leaf.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1709_04488_amd import workloads as W  # noqa: E402

FIELDS = ("h", "rho", "omega", "pressure", "cs", "ax", "ay", "az", "dudt", "vsig", "dt",
          "nngb", "nforce")


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04488_amd import sph as s
    s.load()
    return s


def _reference(sph, params, arrays):
    with sph.Context(params) as ctx:
        p = sph.Particles.from_host(arrays)
        ctx.evaluate(p)
        ctx.sync()
        return p.host()


@pytest.mark.parametrize("precision,leaf", [(0, 16), (1, 32), (0, 8)])
def test_noalloc_equals_evaluate_twice(sph, precision, leaf):
    big = W.blob_in_lattice(30, seed=41)        # 27,000 particles, blob in a periodic box
    small = W.plummer(3000, seed=42)            # open boundary, smaller
    assert big.n <= sph.load().sph_noalloc_max_n()
    params_big = sph.Params.from_setup(big.setup, precision=precision, leaf_size=leaf)
    params_small = sph.Params.from_setup(small.setup, precision=precision, leaf_size=leaf)
    ref_big = _reference(sph, params_big, big.arrays)
    ref_small = _reference(sph, params_small, small.arrays)
    with sph.Context(params_big) as ctx:
        for w, params, ref in ((big, params_big, ref_big), (small, params_small, ref_small)):
            print(f"case: noalloc {w.name} N={w.n} precision={precision} leaf={leaf}", flush=True)
            ctx.set_params(params)
            p = sph.Particles.from_host(w.arrays)
            ctx.evaluate_noalloc(p)
            ctx.sync()
            out = p.host()
            for k in FIELDS:
                assert np.array_equal(out[k], ref[k]), (w.name, k)
        # the context allocated nothing of its own for these calls
        assert ctx.device_bytes() <= 4096


def test_noalloc_rejects_sets_above_its_maximum(sph):
    nmax = sph.load().sph_noalloc_max_n()
    rng = np.random.default_rng(0)
    n = nmax + 1
    a = {k: rng.uniform(0, 1, n) for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
    a.update(m=np.full(n, 1.0 / n), h=np.full(n, 0.02))
    with sph.Context(sph.Params()) as ctx:
        p = sph.Particles.from_host(a)
        with pytest.raises(sph.SphError) as e:
            ctx.evaluate_noalloc(p)
        assert e.value.code == sph.SPH_ECAP
        assert "exceeds" in ctx.last_error()
