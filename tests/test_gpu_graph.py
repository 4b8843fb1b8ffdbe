"""Captured resident steps (HIP graph) equal eager sph_step calls bit for
bit, replay after replay, with unrelated eager work between replays."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1709_04488_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04488_amd import sph as s
    s.load()
    return s


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_equal_eager_steps(sph, prec):
    w = W.blob_in_lattice(12, seed=31)
    stream = torch.cuda.Stream()
    params = sph.Params.from_setup(w.setup, precision=prec)
    eager = sph.Context(params, stream=stream)
    graph = sph.Context(params, stream=stream)
    with torch.cuda.stream(stream):
        pe = sph.Particles.from_host(w.arrays)
        pg = sph.Particles.from_host(w.arrays)
    eager.upload_state(pe)
    graph.upload_state(pg)
    graph.capture_steps(0.0)
    print("case: graph replays prec=%d" % prec, flush=True)
    for rep in range(4):
        eager.step(0.0)
        eager.step(0.0)
        graph.replay_steps()
        stream.synchronize()
        # unrelated eager work between replays
        junk = torch.ones(1 << 16, device="cuda") * (rep + 1)
        torch.cuda.synchronize()
        del junk
        with torch.cuda.stream(stream):
            qe = sph.Particles.from_host(w.arrays)
            qg = sph.Particles.from_host(w.arrays)
        eager.download_state(qe)
        graph.download_state(qg)
        eager.sync()
        graph.sync()
        a, b = qe.host(), qg.host()
        for f in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho", "ax", "dudt", "dt"):
            assert np.array_equal(a[f], b[f]), (rep, f)
    ie, ig = eager.state_info(), graph.state_info()
    assert ie["steps"] == ig["steps"] == 8
    assert ie["time"] == ig["time"]
    eager.close()
    graph.close()


def test_capture_needs_resident_state(sph):
    stream = torch.cuda.Stream()
    with sph.Context(sph.Params(), stream=stream) as ctx:
        with pytest.raises(sph.SphError) as e:
            ctx.capture_steps(0.0)
        assert e.value.code == sph.SPH_ESTATE
        with pytest.raises(sph.SphError) as e:
            ctx.replay_steps()
        assert e.value.code == sph.SPH_ESTATE


def test_set_params_drops_captured_steps(sph):
    """Captured steps carry the parameters of their capture: sph_set_params
    drops them, and steps captured again (after a new upload, whose initial
    forces use the new parameters) with artificial conductivity on equal
    eager steps with it on."""
    w = W.blob_in_lattice(12, seed=32)
    stream = torch.cuda.Stream()
    p0 = sph.Params.from_setup(w.setup)
    p1 = sph.Params.from_setup({**w.setup, "alpha_ac": 1.0, "ac_signal": sph.SPH_AC_PRICE})
    eager = sph.Context(p1, stream=stream)
    graph = sph.Context(p0, stream=stream)
    with torch.cuda.stream(stream):
        pe = sph.Particles.from_host(w.arrays)
        pg = sph.Particles.from_host(w.arrays)
    eager.upload_state(pe)
    graph.upload_state(pg)
    graph.capture_steps(0.0)
    print("case: set_params after capture", flush=True)
    graph.set_params(p1)
    with pytest.raises(sph.SphError) as e:
        graph.replay_steps()
    assert e.value.code == sph.SPH_ESTATE
    # the initial forces of the upload used the old parameters: upload again
    with torch.cuda.stream(stream):
        pg = sph.Particles.from_host(w.arrays)
    graph.upload_state(pg)
    graph.capture_steps(0.0)
    for _ in range(2):
        eager.step(0.0)
        eager.step(0.0)
        graph.replay_steps()
    stream.synchronize()
    with torch.cuda.stream(stream):
        qe = sph.Particles.from_host(w.arrays)
        qg = sph.Particles.from_host(w.arrays)
    eager.download_state(qe)
    graph.download_state(qg)
    eager.sync()
    graph.sync()
    a, b = qe.host(), qg.host()
    for f in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho", "ax", "dudt", "dt"):
        assert np.array_equal(a[f], b[f]), f
    eager.close()
    graph.close()
