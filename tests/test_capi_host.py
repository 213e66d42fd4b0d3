"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/hcg.h declares, and rejects bad arguments that
are validated before any device work."""
import ctypes
import os
import re

import pytest

import paper_2012_13173_amd as hcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hcg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("hcg_plan", "hcg_grid", "hcg_destroy", "hcg_last_error"):
        assert required in names
    assert set(names) == set(hcg.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = hcg.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_argument_errors_before_device_work():
    lib = hcg.load()
    vp = ctypes.c_void_p
    # NULL out handle
    g = hcg.GridDescC(10, 10, 180.0, 30.0, 0.01, 0.01)
    assert lib.hcg_plan(None, vp(1), vp(1), 10, ctypes.byref(g), 0.05, 0.05, None, None) == hcg.HCG_E_ARG
    h = vp()
    # NULL coordinates, n out of range, bad grid, bad kernel
    assert lib.hcg_plan(ctypes.byref(h), None, vp(1), 10, ctypes.byref(g), 0.05, 0.05, None, None) == hcg.HCG_E_ARG
    assert h.value is None
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 0, ctypes.byref(g), 0.05, 0.05, None, None) == hcg.HCG_E_ARG
    bad = hcg.GridDescC(0, 10, 180.0, 30.0, 0.01, 0.01)
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(bad), 0.05, 0.05, None, None) == hcg.HCG_E_ARG
    polar = hcg.GridDescC(10, 100, 0.0, 89.9, 0.01, 0.01)
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(polar), 0.05, 0.05, None, None) == hcg.HCG_E_ARG
    assert b"latitudes" in lib.hcg_last_error()
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(g), 0.0, 0.05, None, None) == hcg.HCG_E_ARG
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(g), 0.05, -1.0, None, None) == hcg.HCG_E_ARG
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(g), float("nan"), 0.05, None, None) == hcg.HCG_E_ARG
    opts = hcg.OptsC(3000, 0, 0, 0, 0, 0)  # not a power of two
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(g), 0.05, 0.05, ctypes.byref(opts), None) == hcg.HCG_E_ARG
    opts = hcg.OptsC(0, 16, 16, 0, 0, 0)  # tile shape not built
    assert lib.hcg_plan(ctypes.byref(h), vp(1), vp(1), 10, ctypes.byref(g), 0.05, 0.05, ctypes.byref(opts), None) == hcg.HCG_E_UNSUPPORTED
    # grid / destroy on handles that are not plans
    assert lib.hcg_grid(None, vp(1), 4, hcg.HCG_F32, None, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid(vp(12345), vp(1), 4, hcg.HCG_F32, None, vp(1), None, None) == hcg.HCG_E_STATE
    assert lib.hcg_destroy(None) == hcg.HCG_OK
    assert lib.hcg_destroy(vp(12345)) == hcg.HCG_E_STATE
    assert b"not a live plan" in lib.hcg_last_error()
    # single steps
    assert lib.hcg_ang2pix(vp(1), vp(1), -1, 16, vp(1), None) == hcg.HCG_E_ARG
    assert lib.hcg_ang2pix(vp(1), vp(1), 4, 17, vp(1), None) == hcg.HCG_E_ARG
    assert lib.hcg_sort_keys(vp(1), 4, 0, vp(2), vp(3), None) == hcg.HCG_E_ARG
    assert lib.hcg_sort_keys(vp(1), 4, 33, vp(2), vp(3), None) == hcg.HCG_E_ARG
    assert lib.hcg_sort_keys(vp(1), 4, 8, vp(1), vp(3), None) == hcg.HCG_E_ARG
    # encoders and the plan-ordered gather
    assert lib.hcg_quantize(vp(1), -1, 4, hcg.HCG_BF16, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_quantize(vp(1), 4, 4, hcg.HCG_F32, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_quantize(vp(1), 4, 4, hcg.HCG_FP8E4M3_SPLIT, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_quantize_packed(None, vp(1), 4, hcg.HCG_BF16, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_quantize_packed(vp(12345), vp(1), 4, hcg.HCG_BF16, vp(1), None, None) == hcg.HCG_E_STATE
    assert lib.hcg_grid_packed(None, vp(1), 4, hcg.HCG_BF16, None, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid_packed(vp(12345), vp(1), 4, hcg.HCG_BF16, None, vp(1), None, None) == hcg.HCG_E_STATE
    # the paper-scheme gather
    assert lib.hcg_grid_rowthreads(None, vp(1), 1, 64, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid_rowthreads(vp(12345), vp(1), 1, 64, vp(1), None, None) == hcg.HCG_E_STATE
    # host streaming
    assert lib.hcg_grid_host(None, vp(1), 4, hcg.HCG_F32, None, 0, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid_host(vp(12345), vp(1), 4, hcg.HCG_F32, None, 0, vp(1), None,
                             None) == hcg.HCG_E_STATE
    nbytes = ctypes.c_int64()
    assert lib.hcg_packed_bytes(None, 4, hcg.HCG_BF16, ctypes.byref(nbytes)) == hcg.HCG_E_ARG
    assert lib.hcg_packed_bytes(vp(12345), 4, hcg.HCG_BF16, ctypes.byref(nbytes)) == hcg.HCG_E_STATE


def test_binding_fails_loudly_without_library(tmp_path):
    saved = hcg._lib
    try:
        hcg._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            hcg.load(str(tmp_path / "nope.so"))
    finally:
        hcg._lib = saved
