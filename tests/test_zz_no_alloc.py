"""The allocation-free render (gs3_render_noalloc) against gs3_render of a
scene holding the same parameters: bit-identical images (same kernels), on
two calls in a row, the second with fewer Gaussians, a lower SH degree and a
smaller image; sizes beyond the static scratch are refused before any work."""
import ctypes
import sys
from ctypes import byref

import numpy as np
import pytest
import torch

import synthetic as syn
from paper_2602_00395_amd import Scene, _lib
from paper_2602_00395_amd.api import make_camera_struct

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(lib, x, deg, cam, bg):
    out = torch.empty((cam.height, cam.width, 3), device=DEV)
    c = make_camera_struct(cam)
    bgc = (ctypes.c_float * 3)(*bg)
    st = torch.cuda.current_stream().cuda_stream
    _lib.check("gs3_render_noalloc", lib.gs3_render_noalloc(x.shape[1], deg, x.data_ptr(), byref(c), bgc,
                                                            out.data_ptr(), ctypes.c_void_p(st)))
    return out


def _scene_render(x, deg, cam, bg):
    zeros = [torch.zeros((cam.height, cam.width, 3), device=DEV)]
    s = Scene(x, zeros, [cam], deg, lam=0.2, background=bg)
    img = s.render(0).clone()
    s.sync()
    s.close()
    return img


def test_noalloc_render_matches_scene_render_twice():
    lib = _lib.load()
    cases = [(syn.config2_scene(n=60_000, n_cams=4, res=640), 1, (0.1, 0.2, 0.3)),
             (syn.tiny_scene(5, n=3000, sh_degree=1, width=200, height=136, n_cams=2, spread=0.8,
                             log_scale_mean=np.log(0.03)), 0, (0.0, 0.0, 0.0))]
    for sc, j, bg in cases:
        x = torch.tensor(sc.init if sc.init is not None else sc.gt, device=DEV).contiguous()
        cam = sc.cameras[j]
        say("no-alloc render", sc.name, "camera", j, "N", sc.n, "SH", sc.sh_degree, f"{cam.width}x{cam.height}")
        got = _noalloc(lib, x, sc.sh_degree, cam, bg)
        torch.cuda.synchronize()
        ref = _scene_render(x, sc.sh_degree, cam, bg)
        assert torch.isfinite(got).all()
        assert float(got.abs().sum()) > 0.0
        assert torch.equal(got, ref), float((got - ref).abs().max())


def test_noalloc_render_refuses_what_does_not_fit():
    lib = _lib.load()
    cam = syn.make_camera((0, -4, 0), 64, 64)
    c = make_camera_struct(cam)
    out = torch.empty((64, 64, 3), device=DEV)
    x = torch.zeros((14, 8), device=DEV)
    rc = lib.gs3_render_noalloc(4_000_000, 0, x.data_ptr(), byref(c), None, out.data_ptr(), None)
    assert rc == _lib.GS3_EINVAL and b"static scratch" in lib.gs3_last_error()
    # a view whose pairs exceed the rest: many large splats covering every tile
    sc = syn.tiny_scene(9, n=400_000, sh_degree=0, width=1024, height=1024, n_cams=1, spread=0.2,
                        log_scale_mean=np.log(0.5), log_scale_std=0.01)
    xs = torch.tensor(sc.gt, device=DEV)
    cb = make_camera_struct(sc.cameras[0])
    big = torch.empty((1024, 1024, 3), device=DEV)
    rc = lib.gs3_render_noalloc(sc.n, 0, xs.data_ptr(), byref(cb), None, big.data_ptr(), None)
    assert rc == _lib.GS3_EINVAL and b"pairs" in lib.gs3_last_error()
