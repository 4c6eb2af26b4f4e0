"""The C-ABI library loads, exports every declared symbol and validates its
arguments before touching the device (no compute calls: no GPU needed)."""
import ctypes
import os
from ctypes import byref, c_int64, c_void_p

import pytest

import synthetic as syn
from paper_2602_00395_amd import _lib
from paper_2602_00395_amd.api import make_desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs3tr.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libgs3tr.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _lib.declared_functions(HEADER)
    assert len(names) >= 20
    raw = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    # and the binding declares exactly the header's functions
    assert sorted(_lib._SIGS) == names


def test_param_count_and_version(lib):
    assert [lib.gs3_n_params(d) for d in range(4)] == [14, 23, 38, 59]
    assert lib.gs3_n_params(4) == -1 and lib.gs3_n_params(-1) == -1
    assert b"gfx950" in lib.gs3_version()


def test_scene_bytes_and_validation(lib):
    cams = [syn.make_camera((0, -4, 0), 64, 48), syn.make_camera((4, 0, 0), 32, 32)]
    d, keep = make_desc(1000, 3, cams)
    res, scr = c_int64(), c_int64()
    assert lib.gs3_scene_bytes(byref(d), byref(res), byref(scr)) == 0
    assert res.value == 4 * 59 * 1000 * 6 + 12 * (64 * 48 + 32 * 32)  # 6 TR state vectors + targets
    assert scr.value > 0
    bad, keep2 = make_desc(1000, 5, cams)
    assert lib.gs3_scene_bytes(byref(bad), byref(res), byref(scr)) == _lib.GS3_EINVAL
    assert b"sh_degree" in lib.gs3_last_error()
    bad, keep3 = make_desc(0, 0, cams)
    assert lib.gs3_scene_bytes(byref(bad), byref(res), byref(scr)) == _lib.GS3_EINVAL
    bad, keep4 = make_desc(10, 0, cams, lam=1.5)
    assert lib.gs3_scene_bytes(byref(bad), byref(res), byref(scr)) == _lib.GS3_EINVAL
    bad, keep5 = make_desc(10, 0, cams, train_mask=[0, 0])
    assert lib.gs3_scene_bytes(byref(bad), byref(res), byref(scr)) == _lib.GS3_EINVAL
    assert b"training" in lib.gs3_last_error()


def test_null_arguments_are_rejected_without_device_work(lib):
    cams = [syn.make_camera((0, -4, 0), 16, 16)]
    d, keep = make_desc(10, 0, cams)
    out = c_void_p()
    assert lib.gs3_scene_create(byref(d), None, None, None, byref(out)) == _lib.GS3_EINVAL
    assert out.value is None
    assert lib.gs3_scene_create(None, None, None, None, byref(out)) == _lib.GS3_EINVAL
    assert lib.gs3_render(None, 0, None, None) == _lib.GS3_EINVAL
    assert lib.gs3_grad(None, None, 0, None, None, None) == _lib.GS3_EINVAL
    assert lib.gs3_scene_destroy(None) == _lib.GS3_EINVAL
    with pytest.raises(_lib.GS3Error):
        _lib.check("gs3_render", lib.gs3_render(None, 0, None, None))
