"""Parity of the HIP path (through the C ABI) with the brute-force oracle.

Tolerances (FP64 mode): neighbour lists and neighbour counts bit-exact;
h, rho, omega, P, c_s, v_sig, dt within 1e-10 relative; a and du/dt within
1e-10 of the per-particle scale S_i = sum_j |pair term| (a ~ 0 by
cancellation on near-uniform sets makes a plain relative error meaningless).
FP32-pair mode: h, rho, P, c_s, v_sig, dt within 1e-5 relative, omega
within 5e-5, a and du/dt within 1e-4 of S_i.  The FP32 errors are checked to
have their two expected sources and no other: (1) the h solve stops within
its floored tolerance of the root (h within 1e-5), and (2) at the GPU's own h
the single-precision pair terms leave rho and omega within 1e-6 of the
oracle's sums at that same h; neighbour-count differences come only from
pairs within 1e-5 of the kernel edge (each count lies between the oracle's
counts at 2h(1 - 1e-5) and 2h(1 + 1e-5)).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1709_04488_amd import workloads as W  # noqa: E402

FP64_TOL = 1e-10
FP32_TOL = 1e-5
FP32_ATOL = 1e-4
# FP32-pair mode: Omega moves with h by d ln Omega / d ln h, which reaches
# ~10 at the edge of the Plummer set, so the ~2e-6 stop tolerance of the h
# solve shows up as up to 1.4e-5 in Omega (measured); 5e-5 is that maximum
# with a factor 3.5.  The pair arithmetic's own share is held to 1e-6 at the
# GPU's h (fp32_error_sources).
FP32_FIELD_TOL = {"omega": 5e-5}
FP32_EDGE = 1e-5      # relative band around the kernel edge q = 2
FP32_PAIR_TOL = 1e-6  # rho, Omega at the GPU's own h


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04488_amd import sph as s
    s.load()
    return s


def _oracle_eval(orc, w, **over):
    a = w.arrays
    p = orc.Params(**{**w.setup, **over})
    return orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])


def _gpu_eval(sph, w, precision=0, leaf_size=16, two_calls=False, **over):
    """sph_evaluate, or with two_calls sph_density then sph_forces."""
    params = sph.Params.from_setup({**w.setup, **over}, precision=precision, leaf_size=leaf_size)
    with sph.Context(params) as ctx:
        p = sph.Particles.from_host(w.arrays)
        if two_calls:
            ctx.density_then_forces(p)
        else:
            ctx.evaluate(p)
        ctx.sync()
        return p.host()


def _check(out, ref, tol=FP64_TOL, atol=FP64_TOL, counts_exact=True, label="", field_tol=None):
    field_tol = field_tol or {}
    for k in ("h", "rho", "omega", "pressure", "cs", "vsig", "dt"):
        rk = "P" if k == "pressure" else k
        rel = np.abs(out[k] / ref[rk] - 1.0)
        print(f"{label} {k}: max {rel.max():.3e} rms {np.sqrt(np.mean(rel ** 2)):.3e}")
        assert rel.max() < field_tol.get(k, tol), (label, k, rel.max())
    for k in ("ax", "ay", "az"):
        rel = np.abs(out[k] - ref[k]) / ref["scale_a"]
        print(f"{label} {k}/S: max {rel.max():.3e} rms {np.sqrt(np.mean(rel ** 2)):.3e}")
        assert rel.max() < atol, (label, k, rel.max())
    rel = np.abs(out["dudt"] - ref["dudt"]) / ref["scale_u"]
    print(f"{label} dudt/S: max {rel.max():.3e} rms {np.sqrt(np.mean(rel ** 2)):.3e}")
    assert rel.max() < atol, (label, "dudt", rel.max())
    if counts_exact:
        assert np.array_equal(out["nngb"], ref["nngb"]), label
        assert np.array_equal(out["nforce"], ref["nforce"]), label


@pytest.mark.parametrize("two_calls", [False, True])
def test_config0_full_parity_fp64(sph, orc, two_calls):
    w = W.config0()
    print("case: config0 N=%d fp64 two_calls=%s" % (w.n, two_calls), flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w, two_calls=two_calls)
    _check(out, ref, label="config0")


@pytest.mark.parametrize("precision", [0, 1])
def test_evaluate_equals_density_then_forces(sph, precision):
    """One sph_evaluate call against sph_density + sph_forces on the same set:
    the density results and every count are the same bits (same sort, same
    tree); the forces may sum in another order (the second call builds its
    tree with the converged h), so they agree to rounding."""
    w = W.plummer(3000, seed=8)
    print("case: evaluate vs two calls, plummer3000 precision=%d" % precision, flush=True)
    one = _gpu_eval(sph, w, precision=precision)
    two = _gpu_eval(sph, w, precision=precision, two_calls=True)
    for k in ("h", "rho", "omega", "pressure", "cs", "nngb", "nforce"):
        assert np.array_equal(one[k], two[k]), k
    tol = 1e-12 if precision == 0 else 1e-5
    scale = np.sqrt(two["ax"] ** 2 + two["ay"] ** 2 + two["az"] ** 2).max()
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(one[k] - two[k])) <= tol * scale, k
    assert np.max(np.abs(one["dudt"] - two["dudt"])) <= tol * np.abs(two["dudt"]).max()
    for k in ("vsig", "dt"):
        assert np.max(np.abs(one[k] / two[k] - 1.0)) <= tol, k


@pytest.mark.parametrize("leaf", [8, 16, 32])
def test_leaf_sizes_ragged_periodic(sph, orc, leaf):
    # random (Poisson) positions, N not a multiple of any leaf size
    rng = np.random.default_rng(77)
    n = 3001
    a = {"x": rng.uniform(0, 1, n), "y": rng.uniform(0, 1, n), "z": rng.uniform(0, 1, n),
         "vx": rng.normal(0, 0.3, n), "vy": rng.normal(0, 0.3, n), "vz": rng.normal(0, 0.3, n),
         "m": np.full(n, 1.0 / n), "u": rng.uniform(0.5, 1.5, n), "h": np.full(n, 0.08)}
    w = W.Workload("poisson3001", a, W.default_setup())
    print("case: poisson N=3001 leaf=%d" % leaf, flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w, leaf_size=leaf)
    _check(out, ref, label=f"leaf{leaf}")


@pytest.mark.parametrize("precision", [0, 1])
def test_unequal_masses(sph, orc, precision):
    """Masses spread over a factor 3: the density loop keeps r^2 and m in its
    candidate lists (the equal-mass path keeps r^2 only and stages no mass)."""
    rng = np.random.default_rng(91)
    n = 2500
    a = {"x": rng.uniform(0, 1, n), "y": rng.uniform(0, 1, n), "z": rng.uniform(0, 1, n),
         "vx": rng.normal(0, 0.3, n), "vy": rng.normal(0, 0.3, n), "vz": rng.normal(0, 0.3, n),
         "m": rng.uniform(0.5, 1.5, n) / n, "u": rng.uniform(0.5, 1.5, n),
         "h": np.full(n, 0.085)}
    w = W.Workload("poisson2500_unequal_m", a, W.default_setup())
    print("case: poisson N=2500 unequal masses precision=%d" % precision, flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w, precision=precision)
    if precision == 0:
        _check(out, ref, label="unequal m fp64")
    else:
        _check(out, ref, tol=FP32_TOL, atol=FP32_ATOL, counts_exact=False,
               label="unequal m fp32", field_tol=FP32_FIELD_TOL)
        fp32_error_sources(orc, w, out, ref)


def _hot_cold_gas(n, seed, **setup):
    # a Poisson gas with unequal masses and u spread over a factor 15
    rng = np.random.default_rng(seed)
    a = {"x": rng.uniform(0, 1, n), "y": rng.uniform(0, 1, n), "z": rng.uniform(0, 1, n),
         "vx": rng.normal(0, 0.3, n), "vy": rng.normal(0, 0.3, n), "vz": rng.normal(0, 0.3, n),
         "m": rng.uniform(0.5, 1.5, n) / n, "u": rng.uniform(0.2, 3.0, n),
         "h": np.full(n, 0.085)}
    return W.Workload(f"hotcold{n}", a, {**W.default_setup(), **setup})


@pytest.mark.parametrize("precision,signal,leaf", [
    (0, 0, 16), (0, 1, 16), (1, 0, 16), (1, 1, 16),
    (0, 1, 8), (1, 0, 8), (0, 0, 32), (1, 1, 32)])
def test_artificial_conductivity(sph, orc, precision, signal, leaf):
    """alpha_AC = 1 (second sum of eq. MON97ENERGYDISS) with the Wadsley
    (signal 0) or Price (signal 1) signal speed, every leaf size."""
    w = _hot_cold_gas(2500, 95, alpha_ac=1.0, ac_signal=signal)
    print("case: hot-cold gas N=2500 alpha_ac=1 signal=%d precision=%d leaf=%d"
          % (signal, precision, leaf), flush=True)
    ref = _oracle_eval(orc, w)
    # the term is large here, so the comparison is not vacuous
    off = _oracle_eval(orc, w, alpha_ac=0.0)
    assert np.median(np.abs(ref["dudt"] - off["dudt"]) / ref["scale_u"]) > 1e-2
    out = _gpu_eval(sph, w, precision=precision, leaf_size=leaf)
    if precision == 0:
        _check(out, ref, label=f"ac{signal} fp64")
    else:
        _check(out, ref, tol=FP32_TOL, atol=FP32_ATOL, counts_exact=False,
               label=f"ac{signal} fp32", field_tol=FP32_FIELD_TOL)


def test_open_boundary_plummer(sph, orc):
    w = W.plummer(2500, seed=31)
    print("case: plummer N=2500 open", flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w)
    _check(out, ref, label="plummer")


def test_blob_in_lattice_small(sph, orc):
    w = W.blob_in_lattice(14, seed=5)
    print("case: blob N=%d" % w.n, flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w)
    _check(out, ref, label="blob")


def test_smallest_periodic_box(sph, orc):
    # 5^3 lattice: 2h ~ 0.48 L, leaves span the box, per-pair minimum image
    w = W.jittered_lattice(5, seed=9)
    print("case: lattice5 periodic", flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w)
    _check(out, ref, label="lattice5")


@pytest.mark.parametrize("n", [6, 7, 17, 64])
def test_tiny_open_sets(sph, orc, n):
    rng = np.random.default_rng(n)
    a = {"x": rng.normal(0, 1, n), "y": rng.normal(0, 1, n), "z": rng.normal(0, 1, n),
         "vx": rng.normal(0, 1, n), "vy": rng.normal(0, 1, n), "vz": rng.normal(0, 1, n),
         "m": np.full(n, 1.0), "u": np.full(n, 1.0), "h": np.full(n, 1.0)}
    w = W.Workload(f"tiny{n}", a, W.default_setup(periodic=False))
    print("case: tiny open N=%d" % n, flush=True)
    ref = _oracle_eval(orc, w)
    out = _gpu_eval(sph, w)
    _check(out, ref, label=f"tiny{n}")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", ["config0", "plummer"])
def test_neighbour_lists_bit_exact(sph, orc, mode, case):
    w = W.config0() if case == "config0" else W.plummer(3000, seed=8)
    a = w.arrays
    p = orc.Params(**w.setup)
    h = orc.density(p, a["x"], a["y"], a["z"], a["m"], a["h"])["h"]
    # perturb h so that mode 1 differs from mode 0
    h = h * np.random.default_rng(3).uniform(0.8, 1.25, w.n)
    roff, ridx = orc.neighbours(p, a["x"], a["y"], a["z"], h, mode)
    print("case: neighbours %s mode %d" % (case, mode), flush=True)
    with sph.Context(sph.Params.from_setup(w.setup)) as ctx:
        pp = sph.Particles.from_host({**a, "h": h})
        off, idx = ctx.neighbours(pp, mode)
        off = off.cpu().numpy()
        idx = idx.cpu().numpy()
    assert np.array_equal(off, roff)
    assert np.array_equal(idx, ridx)


def test_momentum_and_energy_identity_on_gpu_outputs(sph):
    w = W.config0()
    out = _gpu_eval(sph, w)
    a = w.arrays
    m = a["m"]
    scale = np.sum(m * (np.abs(out["ax"]) + np.abs(out["ay"]) + np.abs(out["az"])))
    for k in ("ax", "ay", "az"):
        assert abs(np.sum(m * out[k])) < 1e-12 * scale
    e = np.sum(m * (a["vx"] * out["ax"] + a["vy"] * out["ay"] + a["vz"] * out["az"] + out["dudt"]))
    assert abs(e) < 1e-12 * np.sum(m * (np.abs(out["dudt"]) + scale))


def test_deterministic_bitwise(sph):
    w = W.blob_in_lattice(12, seed=2)
    o1 = _gpu_eval(sph, w)
    o2 = _gpu_eval(sph, w)
    for k in ("h", "rho", "ax", "ay", "az", "dudt", "vsig", "nngb", "nforce"):
        assert np.array_equal(o1[k], o2[k]), k


def test_empty_set_is_a_no_op(sph):
    with sph.Context(sph.Params()) as ctx:
        p = sph.Particles.from_host({k: np.zeros(0) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h")})
        ctx.evaluate(p)
        ctx.sync()


def test_no_root_reports_not_converged(sph):
    # 5 equal-mass particles in isolation: h^3 rho = eta^3 m has no root
    rng = np.random.default_rng(0)
    a = {k: rng.uniform(0, 1, 5) for k in ("x", "y", "z", "vx", "vy", "vz")}
    a.update(m=np.full(5, 0.2), u=np.ones(5), h=np.full(5, 0.3))
    with sph.Context(sph.Params(periodic=False, h_max_iter=30)) as ctx:
        p = sph.Particles.from_host(a)
        ctx.density(p)
        rc = ctx.sync_status()
        assert rc == sph.SPH_ENOTCONVERGED, ctx.last_error()


def test_box_too_small_reports_stencil(sph):
    w = W.lattice(2)
    with sph.Context(sph.Params()) as ctx:
        p = sph.Particles.from_host(w.arrays)
        ctx.density(p)
        rc = ctx.sync_status()
        assert rc == sph.SPH_ESTENCIL, ctx.last_error()


def test_nan_input_reports_nonfinite(sph):
    w = W.jittered_lattice(6, seed=1)
    a = dict(w.arrays)
    a["x"] = a["x"].copy()
    a["x"][7] = np.nan
    with sph.Context(sph.Params()) as ctx:
        p = sph.Particles.from_host(a)
        ctx.density(p)
        rc = ctx.sync_status()
        assert rc == sph.SPH_ENONFINITE, ctx.last_error()


def test_bad_arguments_are_rejected(sph):
    for bad in ({"leaf_size": 12}, {"alpha_ac": -1.0}, {"alpha_ac": float("inf")},
                {"ac_signal": 2}):
        with pytest.raises(sph.SphError) as e:
            sph.Context(sph.Params(**bad))
        assert e.value.code == sph.SPH_EINVAL, bad
    with sph.Context(sph.Params()) as ctx:
        p = sph.Particles.from_host(W.jittered_lattice(6, seed=1).arrays)
        p.t["rho"] = None
        with pytest.raises(sph.SphError) as e:
            ctx.density(p)
        assert e.value.code == sph.SPH_EINVAL
        with pytest.raises(sph.SphError) as e:
            ctx.step(0.0)
        assert e.value.code == sph.SPH_ESTATE


def test_budget_is_enforced(sph):
    w = W.jittered_lattice(10, seed=1)
    with sph.Context(sph.Params(), budget_bytes=100_000) as ctx:
        p = sph.Particles.from_host(w.arrays)
        with pytest.raises(sph.SphError) as e:
            ctx.density(p)
        assert e.value.code == sph.SPH_EBUDGET


@pytest.mark.parametrize("ac", [None, 0, 1])
def test_kdk_steps_match_oracle(sph, orc, ac):
    # ac: artificial conductivity off, or alpha_AC = 1 with that signal speed
    w = W.jittered_lattice(10, seed=21)
    if ac is not None:
        w = W.Workload(w.name, w.arrays, {**w.setup, "alpha_ac": 1.0, "ac_signal": ac})
    a = w.arrays
    nsteps = 10
    st, energy, dts = orc.kdk(orc.Params(**w.setup), a["x"], a["y"], a["z"], a["vx"], a["vy"],
                              a["vz"], a["m"], a["u"], a["h"], nsteps, 0.0)
    print("case: kdk N=%d steps=%d ac=%s" % (w.n, nsteps, ac), flush=True)
    with sph.Context(sph.Params.from_setup(w.setup)) as ctx:
        p = sph.Particles.from_host(a)
        ctx.upload_state(p)
        for _ in range(nsteps):
            ctx.step(0.0)
        ctx.sync()
        info = ctx.state_info()
        q = sph.Particles.from_host(a)
        ctx.download_state(q)
        ctx.sync()
        out = q.host()
    for k in ("x", "y", "z"):
        d = out[k] - st[k]
        d -= np.round(d)
        assert np.max(np.abs(d)) < 1e-10, k
    for k in ("vx", "vy", "vz", "u", "h"):
        assert np.max(np.abs(out[k] - st[k])) < 1e-8 * max(1.0, np.max(np.abs(st[k]))), k
    assert info["time"] == pytest.approx(np.sum(dts), rel=1e-9)
    e = info["kinetic"] + info["thermal"]
    assert e == pytest.approx(energy[-1], rel=1e-10)


@pytest.mark.parametrize("which", ["plummer", "blob"])
def test_resident_forces_after_h_grows(sph, orc, which):
    """Resident state from initial h at half the solution: the h solve doubles
    h, and the force walk must use the new h (all force pairs found)."""
    w = W.plummer(3000, seed=31) if which == "plummer" else W.blob_in_lattice(12, seed=32)
    a = dict(w.arrays)
    a["h"] = 0.5 * a["h"]
    print("case: resident %s N=%d h0/2" % (w.name, w.n), flush=True)
    p = orc.Params(**w.setup)
    ref = orc.evaluate(p, a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["m"], a["u"], a["h"])
    with sph.Context(sph.Params.from_setup(w.setup)) as ctx:
        ctx.upload_state(sph.Particles.from_host(a))
        q = sph.Particles.from_host(a)
        ctx.download_state(q)
        ctx.sync()
        out = q.host()
    assert np.median(out["h"] / a["h"]) > 1.5
    _check(out, ref, label="resident " + w.name)


def test_paper_tolerance_mode_satisfies_its_own_bound(sph, orc):
    """With the paper's ~1 % stopping rule (section 2.1.1) the result is not
    parity-checked, only held to that rule.  The iteration stops at an h whose
    next Newton step would move h by at most h_rtol h and rho by at most
    h_rtol rho (d ln rho / d ln h = 3 (Omega - 1), eq. EQN:OMEGA); Newton's
    step is the distance to the root up to its own second-order term, so h and
    rho lie within h_rtol (5 % slack for that term) of the oracle's root."""
    w = W.config0()
    print("case: h_rtol 1e-2", flush=True)
    params = sph.Params.from_setup(w.setup)
    params.h_rtol = 1e-2
    with sph.Context(params) as ctx:
        p = sph.Particles.from_host(w.arrays)
        ctx.density(p)
        ctx.sync()
        out = p.host("h", "rho", "omega")
    ref = _oracle_eval(orc, w)
    dh = np.max(np.abs(out["h"] / ref["h"] - 1.0))
    drho = np.max(np.abs(out["rho"] / ref["rho"] - 1.0))
    print(f"h_rtol 1e-2: max |h/h_root - 1| {dh:.3e}, max |rho/rho_root - 1| {drho:.3e}")
    assert dh < 1e-2 * 1.05
    assert drho < 1e-2 * 1.05


def fp32_error_sources(orc, w, out, ref, force_counts=True, edge_only=None):
    """The FP32-pair errors have their expected sources only (module doc).
    edge_only: boolean mask of particles whose density comes almost wholly
    from pairs near the kernel edge, where f ~ (2 - q)^3 / 4 magnifies the
    single-precision error of q by 3 q / (2 - q); they are held to 1e-4 at
    their own h instead."""
    a = w.arrays
    p = orc.Params(**w.setup)
    x, y, z, m = a["x"], a["y"], a["z"], a["m"]
    at = orc.rho_at(p, x, y, z, m, out["h"])
    om_at = 1.0 + out["h"] * at["drhodh"] / (3.0 * at["rho"])
    r_rho = np.abs(out["rho"] / at["rho"] - 1.0)
    r_om = np.abs(out["omega"] / om_at - 1.0)
    tol = np.full(w.n, FP32_PAIR_TOL)
    if edge_only is not None:
        tol[edge_only] = 1e-4
    print(f"{w.name} fp32 at own h: rho {r_rho.max():.3e} omega {r_om.max():.3e}")
    assert np.all(r_rho < tol) and np.all(r_om < tol)
    lo = orc.rho_at(p, x, y, z, m, ref["h"] * (1.0 - FP32_EDGE))["nngb"]
    hi = orc.rho_at(p, x, y, z, m, ref["h"] * (1.0 + FP32_EDGE))["nngb"]
    print(f"{w.name} fp32 density counts differing: {int(np.sum(out['nngb'] != ref['nngb']))}")
    assert np.all(lo <= out["nngb"]) and np.all(out["nngb"] <= hi)
    if force_counts:
        flo = np.diff(orc.neighbours(p, x, y, z, ref["h"] * (1.0 - FP32_EDGE), 1)[0])
        fhi = np.diff(orc.neighbours(p, x, y, z, ref["h"] * (1.0 + FP32_EDGE), 1)[0])
        assert np.all(flo <= out["nforce"]) and np.all(out["nforce"] <= fhi)


def test_fp32_pair_mode_tolerances(sph, orc):
    for w in (W.config0(), W.plummer(3000, seed=12)):
        print("case: fp32 %s" % w.name, flush=True)
        ref = _oracle_eval(orc, w)
        out = _gpu_eval(sph, w, precision=sph.SPH_FP32_PAIR)
        _check(out, ref, tol=FP32_TOL, atol=FP32_ATOL, counts_exact=False, label="fp32 " + w.name,
               field_tol=FP32_FIELD_TOL)
        fp32_error_sources(orc, w, out, ref)


def test_fp32_pair_momentum_conserved(sph):
    w = W.config0()
    out = _gpu_eval(sph, w, precision=sph.SPH_FP32_PAIR)
    m = w.arrays["m"]
    scale = np.sum(m * (np.abs(out["ax"]) + np.abs(out["ay"]) + np.abs(out["az"])))
    for k in ("ax", "ay", "az"):
        assert abs(np.sum(m * out[k])) < 1e-12 * scale
