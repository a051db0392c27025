"""CPU-side checks of the C ABI: the library loads and exports every symbol
that include/yk.h declares (no compute calls: no GPU here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "yk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(yk_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("yk_volume_potential", "yk_double_layer_apply", "yk_gmres_density", "yk_heat_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1007_5335_amd.yk as yk
    if not os.path.exists(yk.LIB_PATH):
        pytest.skip("libyk.so not built")
    lib = yk.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(yk.EXPORTS)


def test_default_options_and_null_handles():
    import ctypes
    import paper_1007_5335_amd.yk as yk
    if not os.path.exists(yk.LIB_PATH):
        pytest.skip("libyk.so not built")
    o = yk.yk_default_options()
    assert o.precision == 0 and o.p == 0 and o.direct == 0 and abs(o.fmm_tol - 1e-10) < 1e-20
    lib = yk.load_library()
    # null context / null output pointer are rejected without touching the GPU
    assert lib.yk_destroy(None) == yk.YK_ERR_ARG
    assert lib.yk_create(ctypes.byref(o), None) == yk.YK_ERR_ARG
    assert lib.yk_volume_potential(None, 1, None, None, 0, None, 1.0, None) == yk.YK_ERR_ARG


def test_order_above_31_is_rejected():
    """The expansion kernels exist for orders up to 31; a larger p is refused
    before any device work (no silently truncated expansion)."""
    import ctypes
    import paper_1007_5335_amd.yk as yk
    if not os.path.exists(yk.LIB_PATH):
        pytest.skip("libyk.so not built")
    lib = yk.load_library()
    o = yk.yk_default_options()
    h = ctypes.c_void_p()
    for p in (32, 40, 80):
        o.p = p
        assert lib.yk_create(ctypes.byref(o), ctypes.byref(h)) == yk.YK_ERR_ARG
        assert not h.value
