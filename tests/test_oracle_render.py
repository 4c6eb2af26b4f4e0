"""Pins of the oracle's blend: closed forms and a per-pixel sequential brute force."""
import math

import numpy as np
import torch

import synthetic as syn
from oracle import binning as B
from oracle import render as R


def _scene(mus, log_s, logits, dcs):
    n = len(mus)
    x = np.zeros((14, n), np.float32)
    for g in range(n):
        x[0:3, g] = mus[g]
        x[3:6, g] = log_s[g]
        x[6:10, g] = (0, 0, 0, 1)
        x[10, g] = logits[g]
        x[11:14, g] = dcs[g]
    return x


def _sig(v):
    return 1.0 / (1.0 + math.exp(-v))


def test_single_splat_closed_form():
    cam = syn.make_camera((0.0, -4.0, 0.0), 48, 48)
    s = 0.08
    x = _scene([(0, 0, 0)], [(math.log(s),) * 3], [0.4], [(0.5, -0.2, 1.0)])
    img = R.render(torch.tensor(x, dtype=torch.float64), cam, 0).numpy()
    var = (cam.fx * np.float32(s) / 4.0) ** 2 + 0.3
    a = _sig(0.4)
    rgb = np.maximum(0.28209479177387814 * np.array([0.5, -0.2, 1.0]) + 0.5, 0)
    for (i, j) in [(24, 24), (20, 26), (30, 17), (5, 5)]:
        d2 = (j + 0.5 - 24.0) ** 2 + (i + 0.5 - 24.0) ** 2
        ab = min(0.99, a * math.exp(-0.5 * d2 / var))
        want = rgb * ab if ab >= 1 / 255 else 0 * rgb
        assert np.allclose(img[i, j], want, rtol=2e-6, atol=1e-12), (i, j)


def test_two_splats_closed_form_front_to_back():
    cam = syn.make_camera((0.0, -4.0, 0.0), 32, 32)
    x = _scene([(0, 1.0, 0), (0, -1.0, 0)], [(math.log(0.2),) * 3] * 2, [0.0, 1.5],
               [(1.0, 0, 0), (0, 1.0, 0)])
    img = R.render(torch.tensor(x, dtype=torch.float64), cam, 0).numpy()
    # Gaussian 1 is at depth 3 (in front), Gaussian 0 at depth 5.
    i = j = 16
    d2 = 0.5 ** 2 * 2
    v_near = (cam.fx * np.float32(0.2) / 3.0) ** 2 + 0.3
    v_far = (cam.fx * np.float32(0.2) / 5.0) ** 2 + 0.3
    a1 = min(0.99, _sig(1.5) * math.exp(-0.5 * d2 / v_near))
    a2 = min(0.99, _sig(0.0) * math.exp(-0.5 * d2 / v_far))
    c1 = np.maximum(0.28209479177387814 * np.array([0, 1.0, 0]) + 0.5, 0)
    c2 = np.maximum(0.28209479177387814 * np.array([1.0, 0, 0]) + 0.5, 0)
    want = c1 * a1 + c2 * a2 * (1 - a1)
    assert np.allclose(img[i, j], want, rtol=2e-6)


def _brute_pixel(pr, bins, gids, px, py):
    """The blend rule read literally: one pixel, one splat at a time (the
    skip decision in float32 from the binning's float32 splat values)."""
    T, C, used = 1.0, np.zeros(3), 0
    f32 = np.float32
    for k, g in enumerate(gids):
        d = bins.dec
        dx32, dy32 = d["u"][g] - f32(px), d["v"][g] - f32(py)
        p32 = f32(-0.5) * ((d["ca"][g] * dx32) * dx32 + (d["cc"][g] * dy32) * dy32) - (d["cb"][g] * dx32) * dy32
        if p32 > 0 or p32 < d["tau"][g]:
            continue
        dx, dy = float(pr["u"][g]) - px, float(pr["v"][g]) - py
        ca, cb, cc = (float(v) for v in pr["conic"][g])
        power = -0.5 * (ca * dx * dx + cc * dy * dy) - cb * dx * dy
        ab = min(0.99, float(pr["alpha"][g]) * math.exp(power))
        if T * (1 - ab) < 1e-4:
            break
        C += pr["rgb"][g].numpy() * ab * T
        T *= 1 - ab
        used = k + 1
    return C, T, used


def test_blend_matches_sequential_brute_force_with_early_stop():
    sc = syn.tiny_scene(7, n=40, width=40, height=36, spread=0.3, log_scale_mean=math.log(0.15))
    x = sc.gt.copy()
    x[10] = 3.0  # opaque splats: many pixels terminate early
    xt = torch.tensor(x, dtype=torch.float64)
    cam = sc.cameras[0]
    img, aux = R.render(xt, cam, 0, return_aux=True)
    pr = aux["proj"]
    bins = aux["bins"]
    n_stopped = 0
    for i in range(cam.height):
        for j in range(cam.width):
            t = (i // 16) * bins.tiles_x + (j // 16)
            C, T, used = _brute_pixel(pr, bins, bins.tile_list(t), j + 0.5, i + 0.5)
            assert np.allclose(img[i, j].numpy(), C, rtol=1e-12, atol=1e-14)
            assert abs(float(aux["T_final"][i, j]) - T) < 1e-14
            assert int(aux["n_contrib"][i, j]) == used
            n_stopped += used < len(bins.tile_list(t))
    assert n_stopped > 50


def test_stacked_opaque_splats_stop_before_threshold():
    cam = syn.make_camera((0.0, -4.0, 0.0), 16, 16)
    logit = math.log(0.95 / 0.05)
    mus = [(0.05, 0.5 * k, 0.05) for k in range(5)]  # increasing depth
    x = _scene(mus, [(math.log(1.0),) * 3] * 5, [logit] * 5, [(1.0, 1.0, 1.0)] * 5)
    img, aux = R.render(torch.tensor(x, dtype=torch.float64), cam, 0, return_aux=True)
    # near the centre every splat has abar > 0.9: after three T is between
    # 1e-4 and 1e-3, so the fourth would take it below 1e-4 and is never added
    T = float(aux["T_final"][8, 8])
    assert 1e-4 <= T < 1e-3
    assert T * (1 - 0.9) < 1e-4
    assert int(aux["n_contrib"][8, 8]) == 3
    # identical colours c: sum_i c abar_i T_i telescopes to c (1 - T_final)
    c = 0.28209479177387814 + 0.5
    assert np.allclose(img[8, 8].numpy(), c * (1 - T), rtol=1e-12)


def test_empty_tiles_give_background():
    cam = syn.make_camera((0.0, -4.0, 0.0), 64, 64)
    x = _scene([(0, 0, 0)], [(math.log(0.01),) * 3], [0.0], [(0, 0, 0)])
    img = R.render(torch.tensor(x, dtype=torch.float64), cam, 0, background=(0.1, 0.2, 0.3))
    assert np.allclose(img[0, 0].numpy(), [0.1, 0.2, 0.3])
    assert np.allclose(img[63, 63].numpy(), [0.1, 0.2, 0.3])
