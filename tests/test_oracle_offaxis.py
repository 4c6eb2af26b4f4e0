"""Pins of the off-axis screen covariance (EWA) against a finite-difference
Jacobian of the pinhole map, including points beyond the frustum clamp.

On the principal ray the terms -f x/z^2 of the EWA Jacobian vanish, so the
on-axis closed forms cannot see a sign or clamp mistake in them.  Here the
Jacobian of the textbook pinhole map p -> (f_x p_x/p_z + c_x, f_y p_y/p_z + c_y)
is taken numerically by central differences, at the camera-space mean, or --
beyond the frustum clamp -- at the point whose x/z and y/z are clamped to
+-1.3 tan(fov/2) (the original 3DGS design; the paper is silent on it).
"""
import math

import numpy as np
import torch

import synthetic as syn
from oracle import binning as B
from oracle import gaussians as G
from oracle import render as R

FOV_X = 60.0  # make_camera's horizontal field of view (degrees)


def _pinhole(p, cam):
    K = np.array([[cam.fx, 0.0, cam.cx], [0.0, cam.fy, cam.cy], [0.0, 0.0, 1.0]])
    h = K @ p
    return h[:2] / h[2]


def _fd_jacobian(p, cam):
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(p[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pinhole(p + e, cam) - _pinhole(p - e, cam)) / (2.0 * h)
    return J


def _offaxis_scene(cam, rng, n, spread):
    """Gaussians in front of the camera at camera-space x/z, y/z drawn in
    [-spread, spread] tan(fov/2), anisotropic and randomly rotated."""
    W = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    tan_x = math.tan(math.radians(FOV_X) / 2.0)
    tan_y = tan_x * cam.height / cam.width
    z = rng.uniform(1.0, 6.0, size=n)
    pc = np.stack([rng.uniform(-spread, spread, n) * tan_x * z, rng.uniform(-spread, spread, n) * tan_y * z, z], 1)
    mu = (pc - t[None, :]) @ W  # W^T (p - t)
    pc = mu @ W.T + t[None, :]  # the stored W is orthogonal only to float32 rounding
    x = np.zeros((14, n))
    x[0:3] = mu.T
    x[3:6] = rng.normal(math.log(0.08), 0.6, size=(3, n))
    q = rng.normal(size=(4, n))
    x[6:10] = q / np.linalg.norm(q, axis=0)
    x[10] = rng.normal(0, 1, n)
    return x, pc


def _cov2_of_conic(conic):
    a, b, c = conic[:, 0], conic[:, 1], conic[:, 2]
    det = a * c - b * b
    return np.stack([c / det, -b / det, a / det], 1)  # (cov_xx, cov_xy, cov_yy)


def _want_cov2(x, pc, cam, clamp=True):
    W = cam.R.astype(np.float64)
    Sigma = G.covariance(torch.tensor(x[3:6].T), torch.tensor(x[6:10].T)).numpy()
    # the camera's half field of view from its intrinsics: tan = (W/2) / f
    lim = 1.3 * np.array([0.5 * cam.width / cam.fx, 0.5 * cam.height / cam.fy])
    out = []
    for g in range(pc.shape[0]):
        p = pc[g].copy()
        if clamp:
            p[:2] = np.clip(p[:2] / p[2], -lim, lim) * p[2]
        J = _fd_jacobian(p, cam) @ W
        S2 = J @ Sigma[g] @ J.T + 0.3 * np.eye(2)
        out.append((S2[0, 0], S2[0, 1], S2[1, 1]))
    return np.array(out)


def test_offaxis_screen_covariance_matches_fd_jacobian_inside_the_frustum():
    rng = np.random.default_rng(31)
    cam = syn.make_camera((0.7, -4.0, 0.9), 96, 64)
    x, pc = _offaxis_scene(cam, rng, 400, 0.95)
    pr = R.project(torch.tensor(x), cam, 0)
    got = _cov2_of_conic(pr["conic"].numpy())
    want = _want_cov2(x, pc, cam)
    assert np.allclose(got, want, rtol=1e-7, atol=1e-9 * np.abs(want).max())
    # the centres are the textbook projection K p / p_z
    uv = np.stack([_pinhole(p, cam) for p in pc])
    assert np.allclose(pr["u"].numpy(), uv[:, 0], rtol=1e-12) and np.allclose(pr["v"].numpy(), uv[:, 1], rtol=1e-12)
    # the off-axis terms matter: dropping them (the on-axis Jacobian) is far off
    far = np.abs(pc[:, 0] / pc[:, 2]) > 0.4
    on_axis = _want_cov2(x, pc * np.array([0.0, 0.0, 1.0]), cam)
    assert np.median(np.abs(on_axis[far] - want[far]) / np.abs(want[far]).max(1, keepdims=True)) > 1e-2
    # the float32 binning's screen covariance is the same to float32 rounding
    a, b, c = B.project_f32(x.astype(np.float32), cam)["cov2"]
    got32 = np.stack([a, b, c], 1).astype(np.float64)
    scale = np.abs(want).max(1, keepdims=True)
    assert np.max(np.abs(got32 - want) / scale) < 2e-5


def test_screen_covariance_beyond_the_frustum_clamp():
    rng = np.random.default_rng(32)
    cam = syn.make_camera((-0.4, -4.0, 0.2), 80, 80)
    x, pc = _offaxis_scene(cam, rng, 300, 2.4)
    tan_x = math.tan(math.radians(FOV_X) / 2.0)
    r = np.abs(pc[:, :2] / pc[:, 2:3]) / (1.3 * tan_x)
    keep = np.all(np.abs(r - 1.0) > 1e-3, axis=1)  # away from the clamp's kink
    x, pc = x[:, keep], pc[keep]
    outside = np.any(np.abs(pc[:, :2] / pc[:, 2:3]) > 1.3 * tan_x, axis=1)
    assert outside.sum() > 100 and (~outside).sum() > 20
    pr = R.project(torch.tensor(x), cam, 0)
    got = _cov2_of_conic(pr["conic"].numpy())
    want = _want_cov2(x, pc, cam, clamp=True)
    assert np.allclose(got, want, rtol=1e-7, atol=1e-9 * np.abs(want).max())
    # without the clamp the Jacobian of points outside differs
    unclamped = _want_cov2(x, pc, cam, clamp=False)
    rel = np.abs(unclamped - want).max(1) / np.abs(want).max(1)
    assert np.all(rel[~outside] < 1e-8) and np.median(rel[outside]) > 1e-2
    a, b, c = B.project_f32(x.astype(np.float32), cam)["cov2"]
    got32 = np.stack([a, b, c], 1).astype(np.float64)
    assert np.max(np.abs(got32 - want) / np.abs(want).max(1, keepdims=True)) < 2e-5
