"""Branches of the pair loops that ordinary sets rarely take, forced and
checked against the oracle, and the neighbour-structure entry point on its
own.

* Truncated walk: a walk whose frontier would outgrow its LDS capacity stops
  one level above the leaves and tests the leaves under each returned node
  directly.  Forced by a few particles far outside a dense cluster: their
  converged 2h reaches across the whole cluster, so their walks (density and
  force) meet every cluster leaf (750 leaves of 8 > 512).
* Candidate-list overflow: a density sweep keeps at most 160 candidates per
  particle for the following Newton steps; a particle with more is swept
  again at every step.  The same far particles have the whole cluster
  (6000 particles) inside their 2h.

Both are asserted to have run (counters of sph_state_info) and every
particle is compared with the brute-force oracle at the usual tolerances.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1709_04488_amd import workloads as W  # noqa: E402
from test_gpu_parity import (FP32_ATOL, FP32_FIELD_TOL, FP32_TOL, _check,  # noqa: E402
                             _oracle_eval, fp32_error_sources)


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04488_amd import sph as s
    s.load()
    return s


def cluster_with_outliers(n_cluster=6000, seed=61):
    """A Gaussian cluster (sigma 0.02) and five particles at distance ~1 on
    different axes (open boundary, equal masses)."""
    rng = np.random.default_rng(seed)
    far = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0]])
    pos = np.concatenate([rng.normal(0.0, 0.02, (n_cluster, 3)), far])
    n = pos.shape[0]
    a = {"x": pos[:, 0].copy(), "y": pos[:, 1].copy(), "z": pos[:, 2].copy(),
         "vx": rng.normal(0, 0.1, n), "vy": rng.normal(0, 0.1, n), "vz": rng.normal(0, 0.1, n),
         "m": np.full(n, 1.0 / n), "u": rng.uniform(0.5, 1.5, n),
         "h": np.concatenate([np.full(n_cluster, 0.005), np.full(5, 0.5)])}
    return W.Workload("cluster6000_outliers5", a, W.default_setup(periodic=False))


@pytest.fixture(scope="module")
def outliers(orc):
    w = cluster_with_outliers()
    ref = _oracle_eval(orc, w)
    # the far particles' support holds the whole cluster
    assert np.all(ref["nngb"][-5:] >= 5900)
    return w, ref


@pytest.mark.parametrize("precision", [0, 1])
def test_truncated_walk_and_list_overflow(sph, orc, outliers, precision):
    w, ref = outliers
    print(f"case: cluster+outliers N={w.n} leaf 8 precision={precision}", flush=True)
    params = sph.Params.from_setup(w.setup, precision=precision, leaf_size=8)
    with sph.Context(params) as ctx:
        p = sph.Particles.from_host(w.arrays)
        ctx.evaluate(p)
        ctx.sync()
        info = ctx.state_info()
        out = p.host()
    print("overflows: density walks %d, force walks %d, density lists %d"
          % (info["density_walk_overflows"], info["force_walk_overflows"],
             info["dens_list_overflows"]))
    assert info["density_walk_overflows"] > 0
    assert info["force_walk_overflows"] > 0
    assert info["dens_list_overflows"] > 0
    if precision == 0:
        _check(out, ref, label="outliers fp64")
    else:
        _check(out, ref, tol=FP32_TOL, atol=FP32_ATOL, counts_exact=False,
               label="outliers fp32", field_tol=FP32_FIELD_TOL)
        far = np.zeros(w.n, bool)
        far[-5:] = True
        fp32_error_sources(orc, w, out, ref, edge_only=far)


def test_build_cells_then_forces(sph, orc):
    """sph_build_cells on its own: the structure it builds serves a following
    sph_forces on the same arrays (given the oracle's h, rho and Omega), and
    the forces match the oracle's; sph_neighbours over it matches too."""
    w = W.plummer(3000, seed=14)
    a = w.arrays
    params = orc.Params(**w.setup)
    d = orc.density(params, a["x"], a["y"], a["z"], a["m"], a["h"])
    f = orc.forces(params, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"],
                   d["h"], d["rho"], d["omega"])
    print("case: build_cells + forces plummer3000", flush=True)
    with sph.Context(sph.Params.from_setup(w.setup)) as ctx:
        p = sph.Particles.from_host({**a, "h": d["h"]})
        p.t["rho"].copy_(torch.as_tensor(d["rho"]))
        p.t["omega"].copy_(torch.as_tensor(d["omega"]))
        ctx.build_cells(p)
        ctx.forces(p)
        ctx.sync()
        out = p.host("ax", "ay", "az", "dudt", "vsig", "dt", "nforce")
        roff, ridx = orc.neighbours(params, a["x"], a["y"], a["z"], d["h"], 1)
        off, idx = ctx.neighbours(p, 1)
        assert np.array_equal(off.cpu().numpy(), roff)
        assert np.array_equal(idx.cpu().numpy(), ridx)
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(out[k] - f[k]) / f["scale_a"]) < 1e-10, k
    assert np.max(np.abs(out["dudt"] - f["dudt"]) / f["scale_u"]) < 1e-10
    for k in ("vsig", "dt"):
        assert np.max(np.abs(out[k] / f[k] - 1.0)) < 1e-10, k
    assert np.array_equal(out["nforce"], f["nforce"])
