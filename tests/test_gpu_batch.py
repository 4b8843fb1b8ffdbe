"""Batched persistent launches: every set's result inside a mix equals its
result alone, bit for bit (FP64 and FP32-pair), and matches the oracle."""
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


def _mix():
    return [
        (W.jittered_lattice(7, seed=1), 0, 16),
        (W.jittered_lattice(11, seed=2), 1, 16),
        (W.plummer(1500, seed=3), 0, 16),
        (W.blob_in_lattice(13, seed=4), 0, 8),
        (W.jittered_lattice(9, seed=5), 1, 32),
        (W.plummer(900, seed=6), 1, 16),
        (W.jittered_lattice(6, seed=7), 0, 16),
    ]


def _fields():
    return ("h", "rho", "omega", "pressure", "cs", "ax", "ay", "az", "dudt", "vsig", "dt",
            "nngb", "nforce")


@pytest.mark.parametrize("two_calls", [False, True])
def test_batch_equals_alone_bitwise(sph, two_calls):
    """sph_batch_evaluate against sph_evaluate per set, and sph_batch_density
    + sph_batch_forces against sph_density + sph_forces per set."""
    mix = _mix()
    alone = []
    for w, prec, leaf in mix:
        with sph.Context(sph.Params.from_setup(w.setup, precision=prec, leaf_size=leaf)) as ctx:
            p = sph.Particles.from_host(w.arrays)
            if two_calls:
                ctx.density_then_forces(p)
            else:
                ctx.evaluate(p)
            ctx.sync()
            alone.append(p.host())
    stream = torch.cuda.current_stream()
    ctxs = [sph.Context(sph.Params.from_setup(w.setup, precision=prec, leaf_size=leaf), stream=stream)
            for w, prec, leaf in mix]
    parts = [sph.Particles.from_host(w.arrays) for w, _, _ in mix]
    print("case: batch of %d sets, two_calls=%s" % (len(mix), two_calls), flush=True)
    if two_calls:
        sph.batch_density(ctxs, parts)
        sph.batch_forces(ctxs, parts)
    else:
        sph.batch_evaluate(ctxs, parts)
    for c in ctxs:
        c.sync()
    for k, (a, p) in enumerate(zip(alone, parts)):
        out = p.host()
        for f in _fields():
            assert np.array_equal(out[f], a[f]), (k, f)
    for c in ctxs:
        c.close()


def test_batch_matches_oracle(sph, orc):
    mix = _mix()[:3]
    stream = torch.cuda.current_stream()
    ctxs = [sph.Context(sph.Params.from_setup(w.setup, precision=0), stream=stream) for w, _, _ in mix]
    parts = [sph.Particles.from_host(w.arrays) for w, _, _ in mix]
    sph.batch_evaluate(ctxs, parts)
    for c in ctxs:
        c.sync()
    for (w, _, _), p in zip(mix, parts):
        a = w.arrays
        ref = orc.evaluate(orc.Params(**w.setup), a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                           a["m"], a["u"], a["h"])
        out = p.host()
        for k in ("h", "rho", "omega"):
            assert np.max(np.abs(out[k] / ref[k] - 1)) < 1e-10, (w.name, k)
        for k in ("ax", "ay", "az"):
            assert np.max(np.abs(out[k] - ref[k]) / ref["scale_a"]) < 1e-10, (w.name, k)
        assert np.array_equal(out["nngb"], ref["nngb"])
    for c in ctxs:
        c.close()


def test_batch_with_conductivity_in_one_set(sph, orc):
    """One set with alpha_AC = 1 makes the launch carry the conductivity
    term; it equals that set alone bit for bit.  The sets with alpha_AC = 0
    then run the conductivity variant of the force loop, which adds exact
    zeros for them: each equals its own single-set run (the variant without
    the term) bit for bit, and the oracle."""
    sets = [w for w, _, _ in _mix()[:3]]
    setups = [{**sets[0].setup, "alpha_ac": 1.0, "ac_signal": 1}, sets[1].setup, sets[2].setup]
    mix = list(zip(sets, setups))
    print("case: batch of 3 sets, the first with alpha_ac = 1", flush=True)
    with sph.Context(sph.Params.from_setup(setups[0], precision=0)) as ctx:
        p0 = sph.Particles.from_host(sets[0].arrays)
        ctx.evaluate(p0)
        ctx.sync()
        alone = p0.host()
    stream = torch.cuda.current_stream()
    ctxs = [sph.Context(sph.Params.from_setup(st, precision=0), stream=stream) for st in setups]
    parts = [sph.Particles.from_host(w.arrays) for w in sets]
    sph.batch_evaluate(ctxs, parts)
    for c in ctxs:
        c.sync()
    outs = [p.host() for p in parts]
    for f in _fields():
        assert np.array_equal(outs[0][f], alone[f]), f
    for (w, st), out in list(zip(mix, outs))[1:]:
        with sph.Context(sph.Params.from_setup(st, precision=0)) as ctx:
            p1 = sph.Particles.from_host(w.arrays)
            ctx.evaluate(p1)
            ctx.sync()
            own = p1.host()
        for f in _fields():
            assert np.array_equal(out[f], own[f]), (w.name, f)
    for (w, st), out in zip(mix, outs):
        a = w.arrays
        ref = orc.evaluate(orc.Params(**st), a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                           a["m"], a["u"], a["h"])
        for k in ("ax", "ay", "az"):
            assert np.max(np.abs(out[k] - ref[k]) / ref["scale_a"]) < 1e-10, (w.name, k)
        assert np.max(np.abs(out["dudt"] - ref["dudt"]) / ref["scale_u"]) < 1e-10, w.name
        assert np.array_equal(out["nforce"], ref["nforce"])
    for c in ctxs:
        c.close()


def test_batch_step_equals_single_steps(sph):
    mix = [(W.jittered_lattice(8, seed=11), 0, 16), (W.blob_in_lattice(10, seed=12), 0, 16),
           (W.jittered_lattice(9, seed=13), 1, 16)]
    nsteps = 4
    single = []
    for w, prec, leaf in mix:
        with sph.Context(sph.Params.from_setup(w.setup, precision=prec, leaf_size=leaf)) as ctx:
            ctx.upload_state(sph.Particles.from_host(w.arrays))
            for _ in range(nsteps):
                ctx.step(0.0)
            q = sph.Particles.from_host(w.arrays)
            ctx.download_state(q)
            ctx.sync()
            single.append(q.host())
    stream = torch.cuda.current_stream()
    ctxs = [sph.Context(sph.Params.from_setup(w.setup, precision=prec, leaf_size=leaf), stream=stream)
            for w, prec, leaf in mix]
    for c, (w, _, _) in zip(ctxs, mix):
        c.upload_state(sph.Particles.from_host(w.arrays))
    for _ in range(nsteps):
        sph.batch_step(ctxs, 0.0)
    for c, (w, _, _), ref in zip(ctxs, mix, single):
        q = sph.Particles.from_host(w.arrays)
        c.download_state(q)
        c.sync()
        out = q.host()
        for f in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho", "ax"):
            assert np.array_equal(out[f], ref[f]), (w.name, f)
        c.close()


def test_batch_rejects_mixed_streams(sph):
    w = W.jittered_lattice(6, seed=1)
    s2 = torch.cuda.Stream()
    c1 = sph.Context(sph.Params.from_setup(w.setup))
    c2 = sph.Context(sph.Params.from_setup(w.setup), stream=s2)
    with pytest.raises(sph.SphError) as e:
        sph.batch_density([c1, c2], [sph.Particles.from_host(w.arrays), sph.Particles.from_host(w.arrays)])
    assert e.value.code == sph.SPH_EINVAL
    c1.close()
    c2.close()
