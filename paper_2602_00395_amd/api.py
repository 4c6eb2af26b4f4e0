"""Python binding of the gs3tr C ABI.  Argument marshalling only: every step
runs in the HIP library; torch provides device memory and the stream."""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_int64, c_uint8, c_void_p

import torch

from . import _lib

ADAM_GROUP_ORDER = ("mu", "f_dc", "f_rest", "opacity", "scale", "rot")
TR_MEAN_EXACT = 1  # GS3_TR_MEAN_EXACT
TR_SECOND_ORDER = 2  # GS3_TR_SECOND_ORDER
TR_SH_JOINT = 4  # GS3_TR_SH_JOINT


def n_params(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def make_camera_struct(cam) -> _lib.Camera:
    c = _lib.Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(v) for v in list(cam.R.reshape(-1))]
    t = [float(v) for v in list(cam.t.reshape(-1))]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = t[i]
    return c


def make_desc(n, sh_degree, cameras, lam=0.2, background=(0.0, 0.0, 0.0), train_mask=None):
    cams = (_lib.Camera * len(cameras))(*[make_camera_struct(c) for c in cameras])
    d = _lib.SceneDesc()
    d.n_gaussians = int(n)
    d.sh_degree = int(sh_degree)
    d.n_cameras = len(cameras)
    d.cameras = ctypes.cast(cams, POINTER(_lib.Camera))
    for i in range(3):
        d.background[i] = float(background[i])
    d.lambda_dssim = float(lam)
    d.flags = 0
    keep = [cams]
    if train_mask is not None:
        m = (c_uint8 * len(cameras))(*[1 if v else 0 for v in train_mask])
        d.train_mask = ctypes.cast(m, POINTER(c_uint8))
        keep.append(m)
    return d, keep


def scene_bytes(n, sh_degree, cameras):
    lib = _lib.load()
    d, _keep = make_desc(n, sh_degree, cameras)
    res, scr = c_int64(), c_int64()
    _lib.check("gs3_scene_bytes", lib.gs3_scene_bytes(byref(d), byref(res), byref(scr)))
    return res.value, scr.value


def trim_cache():
    """Release the device blocks destroyed scenes left in the library's cache."""
    lib = _lib.load()
    _lib.check("gs3_trim_cache", lib.gs3_trim_cache())


def profile_enable(names: str):
    """Bracket the named stages with HIP events (see gs3_profile_enable)."""
    lib = _lib.load()
    _lib.check("gs3_profile_enable", lib.gs3_profile_enable(names.encode() if names else None))


def profile_count(on: bool):
    """Whether bracketed blend launches count their work (see gs3_profile_count)."""
    lib = _lib.load()
    _lib.check("gs3_profile_count", lib.gs3_profile_count(1 if on else 0))


def profile_reset():
    lib = _lib.load()
    _lib.check("gs3_profile_reset", lib.gs3_profile_reset())


def profile_read(name: str) -> dict:
    lib = _lib.load()
    n, ms, w0, w1 = c_int64(), c_double(), c_int64(), c_int64()
    _lib.check("gs3_profile_read", lib.gs3_profile_read(name.encode(), byref(n), byref(ms), byref(w0), byref(w1)))
    return dict(launches=n.value, total_ms=ms.value, work0=w0.value, work1=w1.value)


class Scene:
    """A scene resident on the GPU: parameters, targets and optimizer state."""

    def __init__(self, params: torch.Tensor, targets, cameras, sh_degree: int, lam: float = 0.2,
                 background=(0.0, 0.0, 0.0), train_mask=None, stream=None):
        self.lib = _lib.load()
        self.cameras = list(cameras)
        self.sh_degree = int(sh_degree)
        self.P = n_params(sh_degree)
        self.N = int(params.shape[1])
        if tuple(params.shape) != (self.P, self.N) or params.dtype != torch.float32:
            raise ValueError(f"params must be float32 [{self.P}, N]")
        if isinstance(targets, (list, tuple)):
            flat = torch.cat([t.reshape(-1) for t in targets])
        else:
            flat = targets.reshape(-1)
        want = sum(3 * c.width * c.height for c in self.cameras)
        if flat.numel() != want or flat.dtype != torch.float32:
            raise ValueError(f"targets must hold {want} float32 values")
        self.device = params.device
        self._stream = stream
        d, keep = make_desc(self.N, sh_degree, self.cameras, lam, background, train_mask)
        h = c_void_p()
        params = params.contiguous()
        flat = flat.contiguous()
        _lib.check("gs3_scene_create",
                   self.lib.gs3_scene_create(byref(d), _ptr(params), _ptr(flat), _stream(stream), byref(h)))
        self.handle = h
        del keep

    # ------------------------------------------------------------------ helpers
    def _st(self):
        return _stream(self._stream)

    def _empty_like_params(self):
        return torch.empty((self.P, self.N), dtype=torch.float32, device=self.device)

    def _img(self, cam):
        c = self.cameras[cam]
        return torch.empty((c.height, c.width, 3), dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.check("gs3_scene_destroy", self.lib.gs3_scene_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ state
    def params(self) -> torch.Tensor:
        out = self._empty_like_params()
        self.export(x=out)
        return out

    def set_params(self, params: torch.Tensor):
        _lib.check("gs3_scene_set_params", self.lib.gs3_scene_set_params(self.handle, _ptr(params.contiguous()),
                                                                           self._st()))

    def export(self, x=None, ghat=None, dhat=None, adam_m=None, adam_v=None):
        _lib.check("gs3_scene_export", self.lib.gs3_scene_export(self.handle, _ptr(x), _ptr(ghat), _ptr(dhat),
                                                                 _ptr(adam_m), _ptr(adam_v), self._st()))

    def import_(self, x=None, ghat=None, dhat=None, adam_m=None, adam_v=None):
        _lib.check("gs3_scene_import", self.lib.gs3_scene_import(self.handle, _ptr(x), _ptr(ghat), _ptr(dhat),
                                                                 _ptr(adam_m), _ptr(adam_v), self._st()))

    def sync(self):
        _lib.check("gs3_scene_sync", self.lib.gs3_scene_sync(self.handle))

    def device_bytes(self) -> int:
        out = c_int64()
        _lib.check("gs3_scene_device_bytes", self.lib.gs3_scene_device_bytes(self.handle, byref(out)))
        return int(out.value)

    # ------------------------------------------------------------------ the method
    def render(self, cam: int, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._img(cam) if out is None else out
        _lib.check("gs3_render", self.lib.gs3_render(self.handle, int(cam), _ptr(out), self._st()))
        return out

    def bin(self, cam: int, capacity: int | None = None):
        """(keys uint64 [Pi], gids int32 [Pi], ranges int32 [tiles, 2]) of one view."""
        c = self.cameras[cam]
        n_tiles = ((c.width + 15) // 16) * ((c.height + 15) // 16)
        n = c_int64()
        _lib.check("gs3_bin", self.lib.gs3_bin(self.handle, int(cam), None, None, None, 0, byref(n), self._st()))
        cap = max(int(n.value), 1) if capacity is None else capacity
        keys = torch.empty(cap, dtype=torch.int64, device=self.device)
        gids = torch.empty(cap, dtype=torch.int32, device=self.device)
        ranges = torch.empty((n_tiles, 2), dtype=torch.int32, device=self.device)
        _lib.check("gs3_bin", self.lib.gs3_bin(self.handle, int(cam), _ptr(keys), _ptr(gids), _ptr(ranges), cap,
                                               byref(n), self._st()))
        return keys[: n.value], gids[: n.value], ranges

    def grad(self, cams, out: torch.Tensor | None = None, want_loss: bool = False):
        out = self._empty_like_params() if out is None else out
        arr = (c_int32 * len(cams))(*[int(c) for c in cams])
        loss = c_double()
        _lib.check("gs3_grad", self.lib.gs3_grad(self.handle, arr, len(cams), _ptr(out),
                                                 byref(loss) if want_loss else None, self._st()))
        return (out, loss.value) if want_loss else out

    def hvp_diag(self, cams, nu: int, seed: int, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._empty_like_params() if out is None else out
        arr = (c_int32 * len(cams))(*[int(c) for c in cams])
        _lib.check("gs3_hvp_diag", self.lib.gs3_hvp_diag(self.handle, arr, len(cams), int(nu),
                                                         ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(out),
                                                         self._st()))
        return out

    def tr_step(self, grad: torch.Tensor, D: torch.Tensor | None, theta1: float, theta2: float, epsilon: float,
                eta_out: torch.Tensor | None = None, dx_out: torch.Tensor | None = None, variant: int = 0):
        """variant: bits TR_MEAN_EXACT | TR_SECOND_ORDER | TR_SH_JOINT (0 = the printed radius)."""
        hp = _lib.TrHparams(float(theta1), float(theta2), float(epsilon), int(variant))
        _lib.check("gs3_tr_step", self.lib.gs3_tr_step(self.handle, _ptr(grad), _ptr(D), byref(hp), _ptr(eta_out),
                                                       _ptr(dx_out), self._st()))

    def tr_iteration(self, S1, S2, nu: int, seed: int, theta1: float, theta2: float, epsilon: float,
                     variant: int = 0, want_loss: bool = False):
        """One fused iteration of Algorithm 1 (gs3_tr_iteration); S2 empty = no Hutchinson step."""
        a1 = (c_int32 * len(S1))(*[int(c) for c in S1])
        a2 = (c_int32 * max(len(S2), 1))(*([int(c) for c in S2] or [0]))
        hp = _lib.TrHparams(float(theta1), float(theta2), float(epsilon), int(variant))
        loss = c_double()
        _lib.check("gs3_tr_iteration", self.lib.gs3_tr_iteration(
            self.handle, a1, len(S1), a2 if S2 else None, len(S2), int(nu), ctypes.c_uint64(int(seed) & (2**64 - 1)),
            byref(hp), byref(loss) if want_loss else None, self._st()))
        return loss.value if want_loss else None

    def adam_step(self, grad: torch.Tensor, lrs: dict, step: int, epsilon: float | None = None):
        arr = (c_float * 6)(*[float(lrs[k]) for k in ADAM_GROUP_ORDER])
        if epsilon is None:
            _lib.check("gs3_adam_step", self.lib.gs3_adam_step(self.handle, _ptr(grad), arr, int(step), self._st()))
        else:
            _lib.check("gs3_adam_tr_step", self.lib.gs3_adam_tr_step(self.handle, _ptr(grad), arr, int(step),
                                                                     float(epsilon), self._st()))

    def psnr(self, cam: int) -> float:
        out = c_double()
        _lib.check("gs3_psnr", self.lib.gs3_psnr(self.handle, int(cam), byref(out), self._st()))
        return out.value

    def render_vjp(self, cam: int, cot: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._empty_like_params() if out is None else out
        _lib.check("gs3_render_vjp", self.lib.gs3_render_vjp(self.handle, int(cam), _ptr(cot.contiguous()),
                                                             _ptr(out), self._st()))
        return out

    def render_jvp(self, cam: int, tangent: torch.Tensor):
        rgb, tan = self._img(cam), self._img(cam)
        _lib.check("gs3_render_jvp", self.lib.gs3_render_jvp(self.handle, int(cam), _ptr(tangent.contiguous()),
                                                             _ptr(rgb), _ptr(tan), self._st()))
        return rgb, tan
