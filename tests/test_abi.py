"""CPU-side checks of the C ABI: the library loads and exports every function
declared in include/sph.h; host-side argument validation (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:sph_status|void|const char \*)\s*\*?\s*(sph_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1404_2303_amd import sph
    lib = sph.load_library()
    decl = _declared()
    assert "sph_density" in decl and "sph_force" in decl and "sph_step" in decl
    for name in decl:
        assert hasattr(lib, name), name


def test_counting_build_alone_exports_the_walk_tally():
    # the counting build (build_lib --count) adds sph_walk_tally to the same
    # ABI; the production library has no trace of it
    from paper_1404_2303_amd import build_lib, sph
    if not os.path.exists(build_lib.COUNT_LIB):
        pytest.skip("the counting build is not built")
    count = ctypes.CDLL(build_lib.COUNT_LIB)
    assert hasattr(count, "sph_walk_tally")
    for name in _declared():
        assert hasattr(count, name), name
    assert not hasattr(sph.load_library(), "sph_walk_tally")


def test_status_strings_and_defaults():
    from paper_1404_2303_amd import sph
    lib = sph.load_library()
    for s in range(9):
        assert len(lib.sph_status_string(s)) > 0
    p = sph.sph_default_params()
    assert p.n_ngb == 48.0 and abs(p.gamma - 5 / 3) < 1e-15 and p.alpha == 0.8 and p.balsara_eps == 1e-4
    assert p.precision == sph.SPH_FP32_ACC64
    assert p.staging == sph.SPH_STAGING_COMPACT and p.shared_min == 128


def test_argument_validation_without_gpu():
    from paper_1404_2303_amd import sph
    lib = sph.load_library()
    # null context / null output pointer are rejected before any HIP call
    assert lib.sph_create(None, None) == sph.SPH_E_INVALID_ARG
    assert lib.sph_build_cells(None, None, None, None) == sph.SPH_E_INVALID_ARG
    assert lib.sph_sort(None, None) == sph.SPH_E_INVALID_ARG
    assert lib.sph_density(None, None, None, None) == sph.SPH_E_INVALID_ARG
    assert lib.sph_force(None, None, None, None) == sph.SPH_E_INVALID_ARG
    assert lib.sph_destroy(None) == sph.SPH_OK
    bad = sph.sph_default_params()
    bad.gamma = 1.0
    ctx = ctypes.c_void_p()
    assert lib.sph_create(ctypes.byref(bad), ctypes.byref(ctx)) == sph.SPH_E_INVALID_ARG
    bad = sph.sph_default_params()
    bad.n_ngb = 5.0   # below the self contribution 32/3: no root
    assert lib.sph_create(ctypes.byref(bad), ctypes.byref(ctx)) == sph.SPH_E_INVALID_ARG
    bad = sph.sph_default_params()
    bad.precision = 7
    assert lib.sph_create(ctypes.byref(bad), ctypes.byref(ctx)) == sph.SPH_E_INVALID_ARG
    bad = sph.sph_default_params()
    bad.staging = 2
    assert lib.sph_create(ctypes.byref(bad), ctypes.byref(ctx)) == sph.SPH_E_INVALID_ARG
    bad = sph.sph_default_params()
    bad.shared_min = 63   # a shared sweep needs more than one group of 64 targets
    assert lib.sph_create(ctypes.byref(bad), ctypes.byref(ctx)) == sph.SPH_E_INVALID_ARG
