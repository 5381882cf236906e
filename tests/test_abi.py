"""The C ABI without a GPU: the library loads, exports every function that
include/gbr.h declares, and the Python binding wraps each under the same name."""
import ctypes

import pytest

from paper_2503_12886_amd import gbr


def test_library_exports_every_declared_symbol():
    L = gbr.lib()
    syms = gbr.header_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing


def test_binding_has_same_names_and_signatures():
    for s in gbr.header_symbols():
        assert s in gbr._SIGS, s
        if s not in ("gbr_strerror", "gbr_create", "gbr_destroy"):
            assert hasattr(gbr, s), s


def test_error_strings():
    L = gbr.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.gbr_strerror(code)
    assert L.gbr_strerror(-99) == b"unknown error"


def test_create_rejects_bad_config_before_touching_a_device():
    L = gbr.lib()
    h = ctypes.c_void_p()
    bad = gbr.gbr_config(12, 128, 0, 4, 1000, 1000, 1000)          # tile 12 is not offered
    assert L.gbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = gbr.gbr_config(16, 100, 0, 4, 1000, 1000, 1000)          # chunk 100 is not offered
    assert L.gbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = gbr.gbr_config(16, 128, 0, 0, 1000, 1000, 1000)          # no frames
    assert L.gbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    assert L.gbr_destroy(None) == -1
    assert L.gbr_graph_destroy(None) == -1


def test_struct_layouts_match_header():
    # gbr_camera: 2 ints + 4 + 9 + 3 + 1 + 3 floats
    assert ctypes.sizeof(gbr.gbr_camera) == 88
    assert ctypes.sizeof(gbr.gbr_config) == 40
    assert gbr.gbr_status.loss.offset == 36
