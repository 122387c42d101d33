"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kifmm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("kifmm_build_tree", "kifmm_precompute_operators", "kifmm_eval", "direct_eval",
              "kifmm_tree_destroy", "kifmm_ops_destroy", "kifmm_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2006_03515_amd import kifmm
    lib = ctypes.CDLL(kifmm.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(kifmm.EXPORTS) <= set(_declared())


def test_argument_errors_before_device_work():
    from paper_2006_03515_amd import kifmm as K
    lib = K._lib
    h = ctypes.c_void_p()
    # NULL grid
    assert lib.kifmm_build_tree(None, 64, None, ctypes.byref(h)) == K.EINVAL
    # a box that is not a column of whole cubes of leaves, nx != ny, hx != hy,
    # non-power-of-two, bad spacing, bad leaf cap
    g = K.Grid((8, 8, 4), (1e-3,) * 3).c()
    assert lib.kifmm_build_tree(ctypes.byref(g), 64, None, ctypes.byref(h)) == K.EUNSUPPORTED
    assert b"multiple" in lib.kifmm_last_error()
    g = K.Grid((8, 16, 16), (1e-3,) * 3).c()
    assert lib.kifmm_build_tree(ctypes.byref(g), 64, None, ctypes.byref(h)) == K.EUNSUPPORTED
    g = K.Grid((8, 8, 8), (1e-3, 2e-3, 1e-3)).c()
    assert lib.kifmm_build_tree(ctypes.byref(g), 64, None, ctypes.byref(h)) == K.EUNSUPPORTED
    g = K.Grid((12, 12, 12), (1e-3,) * 3).c()
    assert lib.kifmm_build_tree(ctypes.byref(g), 64, None, ctypes.byref(h)) == K.EUNSUPPORTED
    g = K.Grid((8, 8, 8), (1e-3, 0.0, 1e-3)).c()
    assert lib.kifmm_build_tree(ctypes.byref(g), 64, None, ctypes.byref(h)) == K.EINVAL
    g = K.Grid((8, 8, 8), (1e-3,) * 3).c()
    assert lib.kifmm_build_tree(ctypes.byref(g), 0, None, ctypes.byref(h)) == K.EINVAL
    assert lib.kifmm_build_tree(ctypes.byref(g), 8, None, ctypes.byref(h)) == K.EUNSUPPORTED
    assert h.value is None
    # direct_eval argument checks
    kern = K.Kernel(150.0).c()
    bad = K.Kernel(150.0, chi_min=2.0, chi_max=0.035).c()
    assert lib.direct_eval(ctypes.byref(g), ctypes.byref(kern), None, 1.0, None, 512, None, 1, None) == K.EINVAL
    assert lib.direct_eval(ctypes.byref(g), ctypes.byref(bad), ctypes.c_void_p(16), 1.0, None, 512,
                           ctypes.c_void_p(1 << 20), 1, None) == K.EINVAL
    assert lib.direct_eval(ctypes.byref(g), ctypes.byref(kern), ctypes.c_void_p(16), 1.0, None, 7,
                           ctypes.c_void_p(1 << 20), 1, None) == K.EINVAL
    # overlapping in/out
    assert lib.direct_eval(ctypes.byref(g), ctypes.byref(kern), ctypes.c_void_p(4096), 1.0, None, 512,
                           ctypes.c_void_p(4096 + 64), 1, None) == K.EINVAL
    assert b"overlap" in lib.kifmm_last_error()
    # eval / precompute with NULL handles
    assert lib.kifmm_eval(None, None, None, 1.0, None, 1, None) == K.EINVAL
    assert lib.kifmm_precompute_operators(None, ctypes.byref(kern), None, None, ctypes.byref(h)) == K.EINVAL
    lib.kifmm_tree_destroy(None)
    lib.kifmm_ops_destroy(None)
