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
                     "sph_step", "sph_upload_state", "sph_download_state", "sph_neighbours",
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


def test_struct_layouts_match_header():
    # sizes of the ABI structs as the C compiler lays them out
    from paper_1709_04488_amd import sph
    assert ctypes.sizeof(sph._Params) == 6 * 8 + 2 * 4 + 6 * 8 + 2 * 4
    assert ctypes.sizeof(sph._Particles) == 8 + 21 * 8
    assert ctypes.sizeof(sph._Stats) == 8 * 8 + 5 * 8 + 8 + 2 * 8
