"""Hierarchical block time-steps (section 2.1.4) with the limiter (section
2.1.5) on the GPU, against the oracle's block integrator.

* A lattice with a few hot particles (levels 0..3): after two level-0
  steps the sub-step count, the particle updates and every particle's level
  are identical to the oracle's, and x, v, u, h agree within 1e-8 (FP64;
  the level decisions are exact comparisons of the CFL steps, integer
  arithmetic otherwise).
* When every particle shares one level, sub-steps are global steps: the
  state after k sub-steps is bit for bit that of k sph_step calls.
* A timeline too shallow for the hot particles reports SPH_ELEVEL; sph_step
  on a block context is refused.
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


def _hot_lattice(side=8, seed=3, factor=200.0, count=2):
    w = W.jittered_lattice(side, seed=seed)
    u = w.arrays["u"].copy()
    u[:count] *= factor
    return W.Workload(w.name + "_hot", {**w.arrays, "u": u}, w.setup)


def _run_gpu(sph, w, nfull, lmax=20, lim=2, precision=0):
    params = sph.Params.from_setup({**w.setup, "block_lmax": lmax, "block_lim": lim},
                                   precision=precision)
    with sph.Context(params) as ctx:
        ctx.upload_state(sph.Particles.from_host(w.arrays))
        for _ in range(4096):
            info = ctx.state_info()
            if info["block_full_steps"] >= nfull:
                break
            ctx.substep()
        ctx.sync()
        q = sph.Particles.from_host(w.arrays).with_level()
        ctx.download_state(q)
        ctx.sync()
        return q.host(), ctx.state_info()


@pytest.mark.parametrize("lim", [1, 2])
def test_block_steps_match_oracle(sph, orc, lim):
    w = _hot_lattice()
    a = w.arrays
    nfull = 2
    p = orc.Params(**w.setup)
    st, energy, nsub, lev, t = orc.kdk_block(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"],
                                             a["m"], a["u"], a["h"], nfull, lmax=20, lim=lim)
    assert lev.max() >= 2                      # several levels in play
    print(f"case: block steps N={w.n} lim={lim} oracle sub-steps {nsub} levels "
          f"{np.bincount(lev)}", flush=True)
    out, info = _run_gpu(sph, w, nfull, lim=lim)
    assert info["block_synchronised"] == 1
    assert info["block_substeps"] == nsub
    assert info["block_updates"] == st["updates"]
    assert np.array_equal(out["level"], lev)
    assert info["block_time"] == pytest.approx(t, rel=1e-12)
    for k in ("x", "y", "z"):
        d = out[k] - st[k]
        d -= np.round(d)
        assert np.max(np.abs(d)) < 1e-8, k
    for k in ("vx", "vy", "vz", "u", "h"):
        e = np.max(np.abs(out[k] - st[k])) / max(1.0, np.max(np.abs(st[k])))
        print(f"block lim {lim} {k}: {e:.3e}")
        assert e < 1e-8, k
    e = info["kinetic"] + info["thermal"]
    assert e == pytest.approx(energy[-1], rel=1e-9)


def test_single_level_substeps_equal_global_steps(sph):
    w = W.jittered_lattice(9, seed=11, sigma_v=0.01)
    nsteps = 4
    print("case: single-level block vs global steps", flush=True)
    with sph.Context(sph.Params.from_setup(w.setup)) as ctx:
        ctx.upload_state(sph.Particles.from_host(w.arrays))
        for _ in range(nsteps):
            ctx.step(0.0)
        q = sph.Particles.from_host(w.arrays)
        ctx.download_state(q)
        ctx.sync()
        glob = q.host()
    params = sph.Params.from_setup({**w.setup, "block_lmax": 20})
    with sph.Context(params) as ctx:
        ctx.upload_state(sph.Particles.from_host(w.arrays))
        for _ in range(nsteps):
            ctx.substep()
        info = ctx.state_info()
        q = sph.Particles.from_host(w.arrays).with_level()
        ctx.download_state(q)
        ctx.sync()
        blk = q.host()
    assert info["block_full_steps"] == nsteps and np.all(blk["level"] == 0)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho", "ax", "dudt"):
        assert np.array_equal(blk[k], glob[k]), k


def test_block_error_paths(sph):
    w = _hot_lattice(factor=1000.0)
    print("case: block error paths", flush=True)
    params = sph.Params.from_setup({**w.setup, "block_lmax": 1})
    with sph.Context(params) as ctx:
        ctx.upload_state(sph.Particles.from_host(w.arrays))
        assert ctx.sync_status() == sph.SPH_ELEVEL
        with pytest.raises(sph.SphError) as e:
            ctx.step(0.0)
        assert e.value.code == sph.SPH_ESTATE
