"""The C-ABI library loads and exports every entry point include/sph.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*[\s\*]+(sph_[a-z_]+)\s*\(",
                                 src, flags=re.M)))


def _lib_path():
    from paper_1709_04488_amd import sph
    path = sph.library_path()
    if not os.path.exists(path):
        from paper_1709_04488_amd import build_lib
        build_lib.build()
    return path


def test_header_declares_the_boundary_calls():
    names = _declared()
    for required in ("sph_create", "sph_destroy", "sph_build_cells", "sph_density", "sph_forces",
                     "sph_evaluate", "sph_step", "sph_upload_state", "sph_download_state", "sph_neighbours",
                     "sph_sync", "sph_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing


def test_binding_covers_every_declared_symbol():
    from paper_1709_04488_amd import sph
    assert sorted(_declared()) == sorted(sph.EXPORTED)


def test_default_params_match_paper_values():
    from conftest import read_golden
    from paper_1709_04488_amd import sph
    sph.load()
    d = sph.default_params_from_library()
    g = read_golden("paper_values.txt")
    assert d["eta"] == g["eta_sph_default"]
    assert d["beta_av"] == g["beta_over_alpha_av"] * d["alpha_av"]
    assert d["c_cfl"] == g["ccfl_typical"]
    assert d["leaf_size"] in (8, 16, 32)
    # no conductivity unless asked for; the paper's default signal speed
    assert d["alpha_ac"] == 0.0 and d["ac_signal"] == sph.SPH_AC_WADSLEY
    # M4 kernel, global time-steps, the full LDS stage and one leaf per claim
    assert d["kernel"] == sph.SPH_KERNEL_M4 and d["block_lmax"] == 0
    assert d["stage_leaves"] == 0 and d["claim_leaves"] == 0


def test_python_defaults_equal_the_library_defaults():
    from paper_1709_04488_amd import sph
    sph.load()
    d = sph.default_params_from_library()
    c = sph.Params().c()
    for f, _ in sph._Params._fields_:
        v = getattr(c, f)
        v = tuple(v) if f in ("box_lo", "box_hi") else v
        assert v == d[f], f


def test_struct_layouts_match_header():
    # sizes of the ABI structs as the C compiler lays them out
    from paper_1709_04488_amd import sph
    # ... + alpha_ac, ac_signal, av_switch (filling the old tail padding),
    # alpha_min, alpha_max, av_ell
    assert ctypes.sizeof(sph._Params) == 6 * 8 + 2 * 4 + 6 * 8 + 2 * 4 + 8 + 4 + 4 + 3 * 8 + 2 * 4 + 4 * 4
    # ... + the optional alpha, divv, curlv, level
    assert ctypes.sizeof(sph._Particles) == 8 + 25 * 8
    # ... + the density and force walk overflows (2 x int32) and the list overflows
    assert ctypes.sizeof(sph._Stats) == 8 * 8 + 5 * 8 + 8 + 2 * 8 + 5 * 8 + 2 * 4 + 8 + 6 * 8 + 8


def test_struct_offsets_match_the_c_compiler(tmp_path):
    # every field offset and struct size of the binding equals what gcc lays
    # out from include/sph.h
    import shutil
    import subprocess
    from paper_1709_04488_amd import sph
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    pairs = (("sph_params", sph._Params), ("sph_particles", sph._Particles),
             ("sph_state_stats", sph._Stats), ("sph_mfv_set", sph._MfvSet),
             ("sph_request", sph._Request))
    cname_of = {"in_": "in"}   # Python keyword renamed in the binding
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sph.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field in py._fields_:
            f = field[0]
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {cname_of.get(f, f)}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line.strip()}
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field in py._fields_:
            assert got[(cname, field[0])] == getattr(py, field[0]).offset, (cname, field[0])


def test_server_plan_counts_the_context_and_the_particle_arrays():
    # an executor slot holds a context and the request's 19 FP64 and 2 int32
    # arrays (host-side arithmetic only: no device call)
    from paper_1709_04488_amd import sph
    for leaf in (8, 16, 32):
        p = sph.Params(leaf_size=leaf)
        for n in (1, 1000, 250_000):
            assert sph.server_plan_bytes(p, n) == sph.plan_bytes(p, n) + n * (19 * 8 + 2 * 4)
