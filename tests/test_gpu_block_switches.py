"""Viscosity switches under hierarchical block time-steps on the GPU
(section 2.1.4; the switches section 2.1.1 names), against the oracle.

* A lattice with a few hot particles (levels 0..3) and per-particle alpha
  under MM97 and under CD10: after two level-0 steps the sub-step count,
  the particle updates and every level are identical to the oracle's; x,
  v, u, h and alpha agree within 1e-8 (FP64).
* The hot-slab set of the oracle's closed-form pins (a hot slab two levels
  deeper than the cold gas), its lattice jittered by 5 % of the spacing:
  levels and sub-steps exact, alpha everywhere within 1e-8 of the oracle.
  (On the perfect lattice dt_max = min dt 2^k puts the uniform hot slab
  exactly on a level boundary, so a last-bit dip of a step in a later
  sub-step sends particles one level deeper: the oracle's own particle
  updates change under 1e-13 position noise there, and not with the
  jitter.)
* Artificial conductivity (alpha_AC = 1, both signal speeds) with the CD10
  switch under block time-steps: levels exact, state within 1e-8.
* FP32-pair mode, without a switch and with each: levels, sub-steps and
  particle updates identical to the FP64 oracle's, state within 1e-4.
* Every particle on one level: sub-steps with a switch are global steps
  with it, bit for bit (x, v, u, h, alpha).
* A per-particle alpha without a switch moves with the particles through
  the block re-sort: alpha = alpha_AV everywhere gives the bits of a run
  without per-particle alpha.
"""
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


def _sw(sph, name):
    return sph.SPH_AV_MM97 if name == "mm97" else sph.SPH_AV_CD10


def _hot_lattice(side=8, seed=3, factor=200.0, count=2):
    w = W.jittered_lattice(side, seed=seed)
    u = w.arrays["u"].copy()
    u[:count] *= factor
    return W.Workload(w.name + "_hot", {**w.arrays, "u": u}, w.setup)


def _alpha(n, seed):
    return np.random.default_rng(seed).uniform(0.1, 1.0, n)


def _run_block(sph, arrays, setup, nfull, alpha=None, lmax=20, lim=2, precision=0):
    params = sph.Params.from_setup({**setup, "block_lmax": lmax, "block_lim": lim},
                                   precision=precision)
    extra = {} if alpha is None else {"alpha": alpha}
    with sph.Context(params) as ctx:
        ctx.upload_state(sph.Particles.from_host({**arrays, **extra}))
        for _ in range(4096):
            if ctx.state_info()["block_full_steps"] >= nfull:
                break
            ctx.substep()
        ctx.sync()
        q = sph.Particles.from_host({**arrays, **extra}).with_level()
        ctx.download_state(q)
        ctx.sync()
        return q.host(), ctx.state_info()


def _compare(out, st, keys, tol, what):
    for k in ("x", "y", "z"):
        d = out[k] - st[k]
        d -= np.round(d)
        assert np.max(np.abs(d)) < tol, (what, k)
    for k in keys:
        e = np.max(np.abs(out[k] - st[k])) / max(1.0, np.max(np.abs(st[k])))
        print(f"{what} {k}: {e:.3e}")
        assert e < tol, (what, k)


@pytest.mark.parametrize("switch", ["mm97", "cd10"])
def test_block_switch_matches_oracle(sph, orc, switch):
    w = _hot_lattice()
    a = w.arrays
    setup = {**w.setup, "av_switch": _sw(sph, switch), "alpha_min": 0.1, "alpha_max": 1.0}
    al0 = _alpha(w.n, 61)
    nfull = 2
    p = orc.Params(**setup)
    st, energy, nsub, lev, t = orc.kdk_block(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                                             a["m"], a["u"], a["h"], nfull, alpha=al0)
    assert lev.max() >= 2
    assert np.max(np.abs(st["alpha"] - al0)) > 1e-3          # the switch did act
    print(f"case: block {switch} N={w.n} oracle sub-steps {nsub} levels {np.bincount(lev)}",
          flush=True)
    out, info = _run_block(sph, a, setup, nfull, alpha=al0)
    assert info["block_synchronised"] == 1
    assert info["block_substeps"] == nsub
    assert info["block_updates"] == st["updates"]
    assert np.array_equal(out["level"], lev)
    assert info["block_time"] == pytest.approx(t, rel=1e-12)
    _compare(out, st, ("vx", "vy", "vz", "u", "h", "alpha"), 1e-8, f"block {switch}")


@pytest.mark.parametrize("signal", [0, 1])
def test_block_conductivity_and_switch_match_oracle(sph, orc, signal):
    w = _hot_lattice(seed=5)
    a = w.arrays
    u = a["u"] * np.random.default_rng(64).uniform(0.5, 2.0, w.n)   # spread for the conductivity
    a = {**a, "u": u}
    setup = {**w.setup, "alpha_ac": 1.0, "ac_signal": signal, "av_switch": _sw(sph, "cd10"),
             "alpha_min": 0.1, "alpha_max": 1.0}
    al0 = _alpha(w.n, 65)
    st, energy, nsub, lev, t = orc.kdk_block(orc.Params(**setup), a["x"], a["y"], a["z"], a["vx"],
                                             a["vy"], a["vz"], a["m"], a["u"], a["h"], 2,
                                             alpha=al0)
    assert lev.max() >= 2
    print(f"case: block conductivity signal={signal} + cd10 N={w.n} sub-steps {nsub}", flush=True)
    out, info = _run_block(sph, a, setup, 2, alpha=al0)
    assert info["block_substeps"] == nsub
    assert info["block_updates"] == st["updates"]
    assert np.array_equal(out["level"], lev)
    _compare(out, st, ("vx", "vy", "vz", "u", "h", "alpha"), 1e-8, f"block ac{signal}")


@pytest.mark.parametrize("switch", ["none", "mm97", "cd10"])
def test_fp32_block_steps_match_oracle(sph, orc, switch):
    w = _hot_lattice()
    a = w.arrays
    setup = dict(w.setup)
    al0 = None
    if switch != "none":
        setup.update(av_switch=_sw(sph, switch), alpha_min=0.1, alpha_max=1.0)
        al0 = _alpha(w.n, 63)
    nfull = 2
    st, energy, nsub, lev, t = orc.kdk_block(orc.Params(**setup), a["x"], a["y"], a["z"], a["vx"],
                                             a["vy"], a["vz"], a["m"], a["u"], a["h"], nfull,
                                             alpha=al0)
    print(f"case: fp32 block {switch} N={w.n} oracle sub-steps {nsub}", flush=True)
    out, info = _run_block(sph, a, setup, nfull, alpha=al0, precision=1)
    assert info["block_substeps"] == nsub
    assert info["block_updates"] == st["updates"]
    assert np.array_equal(out["level"], lev)
    keys = ("vx", "vy", "vz", "u", "h") + (("alpha",) if al0 is not None else ())
    _compare(out, st, keys, 1e-4, f"fp32 block {switch}")


def _hot_slab(nx=32, ny=8, u_hot=17.6, jitter=0.05, seed=71):
    s = 1.0 / ny
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(ny), indexing="ij")
    rng = np.random.default_rng(seed)
    x, y, z = ((g.ravel() + 0.5 + jitter * rng.uniform(-1.0, 1.0, g.size)) * s
               for g in (ix, iy, iz))
    n = x.size
    Lx = nx * s
    zero = np.zeros(n)
    arrays = {"x": x, "y": y, "z": z, "vx": zero, "vy": zero.copy(), "vz": zero.copy(),
              "m": np.full(n, Lx / n), "u": np.where(x < 0.5 * Lx, u_hot, 1.0),
              "h": np.full(n, 1.2 * s)}
    setup = {**W.default_setup(True, (0.0, 0.0, 0.0), (Lx, 1.0, 1.0))}
    return arrays, setup


@pytest.mark.parametrize("switch", ["mm97", "cd10"])
def test_block_switch_hot_slab(sph, orc, switch):
    a, setup = _hot_slab()
    setup = {**setup, "av_switch": _sw(sph, switch), "alpha_min": 0.1, "alpha_max": 1.0}
    al0 = np.full(a["x"].size, 1.0)
    p = orc.Params(**setup)
    st, energy, nsub, lev, t = orc.kdk_block(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                                             a["m"], a["u"], a["h"], 1, alpha=al0)
    print(f"case: hot slab {switch} N={a['x'].size} oracle sub-steps {nsub}", flush=True)
    assert lev.max() >= 2 and np.any(lev == 0)
    assert np.max(np.abs(st["alpha"] - al0)) > 1e-3
    out, info = _run_block(sph, a, setup, 1, alpha=al0)
    assert info["block_substeps"] == nsub
    assert np.array_equal(out["level"], lev)
    _compare(out, st, ("vx", "vy", "vz", "u", "h", "alpha"), 1e-8, f"slab {switch}")


@pytest.mark.parametrize("switch", ["mm97", "cd10"])
def test_single_level_block_switch_equals_global_steps(sph, switch):
    w = W.jittered_lattice(9, seed=11, sigma_v=0.01)
    setup = {**w.setup, "av_switch": _sw(sph, switch), "alpha_min": 0.1, "alpha_max": 1.0}
    al0 = _alpha(w.n, 62)
    nsteps = 4
    print(f"case: single-level block {switch} vs global steps", flush=True)
    with sph.Context(sph.Params.from_setup(setup)) as ctx:
        ctx.upload_state(sph.Particles.from_host({**w.arrays, "alpha": al0}))
        for _ in range(nsteps):
            ctx.step(0.0)
        q = sph.Particles.from_host({**w.arrays, "alpha": al0})
        ctx.download_state(q)
        ctx.sync()
        glob = q.host()
    blk, info = _run_block(sph, w.arrays, setup, nsteps, alpha=al0)
    assert info["block_full_steps"] == nsteps and np.all(blk["level"] == 0)
    assert np.max(np.abs(glob["alpha"] - al0)) > 1e-4
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "alpha"):
        assert np.array_equal(blk[k], glob[k]), k


def test_block_per_particle_alpha_moves_with_particles(sph):
    w = _hot_lattice()
    print("case: block steps with a constant per-particle alpha", flush=True)
    plain, i0 = _run_block(sph, w.arrays, w.setup, 2)
    same, i1 = _run_block(sph, w.arrays, w.setup, 2, alpha=np.full(w.n, w.setup["alpha"]))
    assert i0["block_substeps"] == i1["block_substeps"]
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "level"):
        assert np.array_equal(plain[k], same[k]), k


def test_batch_substep_equals_single_substeps(sph):
    """Block states of different sizes, switches and precisions, each on its
    own clock, advanced together by sph_batch_substep: after every call each
    set is bit for bit where sph_substep alone takes it."""
    hot = _hot_lattice()
    blob = W.blob_in_lattice(9, seed=66)
    mix = [(hot.arrays, hot.setup, 0, None),
           (blob.arrays, {**blob.setup, "av_switch": sph.SPH_AV_CD10}, 0, _alpha(blob.n, 67)),
           (_hot_lattice(side=7, seed=8).arrays, {**hot.setup, "av_switch": sph.SPH_AV_MM97}, 0,
            _alpha(343, 68)),
           (hot.arrays, hot.setup, 1, None)]
    nsub = 12
    fields = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho", "ax", "level")

    def params(setup, prec):
        return sph.Params.from_setup({**setup, "block_lmax": 20, "block_lim": 2}, precision=prec)

    def parts(arrays, al):
        return sph.Particles.from_host({**arrays, **({} if al is None else {"alpha": al})})

    print(f"case: batched block sub-steps of {len(mix)} sets", flush=True)
    single = []
    for arrays, setup, prec, al in mix:
        with sph.Context(params(setup, prec)) as ctx:
            ctx.upload_state(parts(arrays, al))
            for _ in range(nsub):
                ctx.substep()
            q = parts(arrays, al).with_level()
            ctx.download_state(q)
            ctx.sync()
            single.append((q.host(), ctx.state_info()))
    stream = torch.cuda.current_stream()
    ctxs = [sph.Context(params(setup, prec), stream=stream) for _, setup, prec, _ in mix]
    for c, (arrays, _, _, al) in zip(ctxs, mix):
        c.upload_state(parts(arrays, al))
    for _ in range(nsub):
        sph.batch_substep(ctxs)
    for k, (c, (arrays, _, _, al), (ref, rinfo)) in enumerate(zip(ctxs, mix, single)):
        q = parts(arrays, al).with_level()
        c.download_state(q)
        c.sync()
        out, info = q.host(), c.state_info()
        assert info["block_substeps"] == rinfo["block_substeps"] == nsub, k
        assert info["block_updates"] == rinfo["block_updates"], k
        assert info["block_time"] == rinfo["block_time"], k
        for f in fields + (("alpha",) if al is not None else ()):
            assert np.array_equal(out[f], ref[f]), (k, f)
    # a context without block time-steps is refused before anything runs
    flat = sph.Context(sph.Params.from_setup(hot.setup), stream=stream)
    flat.upload_state(sph.Particles.from_host(hot.arrays))
    before = ctxs[0].state_info()["block_substeps"]
    with pytest.raises(sph.SphError) as e:
        sph.batch_substep([ctxs[0], flat])
    assert e.value.code == sph.SPH_ESTATE
    assert ctxs[0].state_info()["block_substeps"] == before
    for c in ctxs + [flat]:
        c.close()
