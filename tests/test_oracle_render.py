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


def _brute_flips(x, cam, bins, tiles):
    """The flip report taken literally: one pixel and one splat at a time."""
    pr = R.project(torch.tensor(x), cam, 0)
    f32 = np.float32
    want = dict(skip=0, clamp=0, stop=0, evaluations=0, pixels=0)
    d = bins.dec
    for t in tiles:
        gids = bins.tile_list(t)
        if len(gids) == 0:
            continue
        ty, tx = divmod(t, bins.tiles_x)
        for i in range(16 * ty, min(16 * ty + 16, cam.height)):
            for j in range(16 * tx, min(16 * tx + 16, cam.width)):
                want["pixels"] += 1
                T64, T32, s64, s32 = 1.0, f32(1.0), None, None
                for k, g in enumerate(gids):
                    dx, dy = float(pr["u"][g]) - (j + 0.5), float(pr["v"][g]) - (i + 0.5)
                    ca, cb, cc = (float(c) for c in pr["conic"][g])
                    p64 = -0.5 * (ca * dx * dx + cc * dy * dy) - cb * dx * dy
                    a64 = float(pr["alpha"][g]) * math.exp(p64)
                    v64 = p64 <= 0 and a64 >= 1 / 255
                    dx32, dy32 = d["u"][g] - f32(j + 0.5), d["v"][g] - f32(i + 0.5)
                    p32 = (f32(-0.5) * ((d["ca"][g] * dx32) * dx32 + (d["cc"][g] * dy32) * dy32)
                           - (d["cb"][g] * dx32) * dy32)
                    v32 = bool(p32 <= 0 and p32 >= d["tau"][g])
                    a32 = f32(pr["alpha"][g].item()) * np.exp(p32)
                    if s64 is None:
                        want["evaluations"] += 1
                        want["skip"] += v64 != v32
                        if v64 and v32:
                            want["clamp"] += (a64 >= 0.99) != bool(a32 >= f32(0.99))
                        if v64:
                            T64 *= 1 - min(a64, 0.99)
                            if T64 < 1e-4:
                                s64 = k
                    if s32 is None and v32:
                        T32 = f32(T32 * (f32(1) - min(a32, f32(0.99))))
                        if T32 < f32(1e-4):
                            s32 = k
                want["stop"] += (len(gids) if s64 is None else s64) != (len(gids) if s32 is None else s32)
    return want


def test_decision_flips_match_a_per_pixel_count():
    # tiny view with opaque and faint splats (many stops, clamps and skips)
    sc = syn.tiny_scene(9, n=30, width=32, height=32, spread=0.3, log_scale_mean=math.log(0.15))
    x = sc.gt.astype(np.float64)
    rng = np.random.default_rng(4)
    x[10] = rng.choice([-4.0, 6.0, 0.3], size=x.shape[1])
    cam = sc.cameras[1]
    bins = B.bin_view(x.astype(np.float32), cam)
    got = R.decision_flips(x, cam, 0, bins)
    want = _brute_flips(x, cam, bins, range(bins.tiles_x * bins.tiles_y))
    assert got == want, (got, want)
    assert got["evaluations"] > 1000


def test_decision_flips_find_a_real_flip():
    # one view of the plain workload holds a splat whose float32 skip decision
    # differs from float64 at one pixel: the report and the literal walk find it
    sc = syn.config1_scene()
    x = sc.init.astype(np.float64)
    cam = sc.cameras[2]
    bins = B.bin_view(x.astype(np.float32), cam)
    per_tile = {t: R.decision_flips(x, cam, 0, bins, tiles={t}) for t in range(bins.tiles_x * bins.tiles_y)}
    flipped = [t for t, r in per_tile.items() if r["skip"] + r["clamp"] + r["stop"] > 0]
    assert flipped
    got = R.decision_flips(x, cam, 0, bins, tiles=set(flipped))
    want = _brute_flips(x, cam, bins, flipped)
    assert got == want, (got, want)
    assert got["skip"] + got["clamp"] + got["stop"] >= 1
