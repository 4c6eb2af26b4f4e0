"""Pins of the oracle's loss: SSIM identities, brute-force windows, L1 and PSNR."""
import math

import numpy as np
import torch

from oracle import loss as Lo


def test_window_is_normalised_gaussian():
    g = Lo.gaussian_window().numpy()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    r = np.arange(11) - 5
    ratio = g[6] / g[5]
    assert abs(ratio - math.exp(-1 / (2 * 1.5 ** 2))) < 1e-14
    assert np.allclose(g, g[::-1])
    assert abs((g * r * r).sum() - 1.5 ** 2) < 0.02  # truncated at 3.3 sigma


def test_ssim_of_identical_images_is_one():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(size=(20, 23, 3)))
    assert torch.allclose(Lo.ssim_map(x, x), torch.ones(20, 23, 3, dtype=torch.float64), atol=1e-12)


def test_ssim_constant_images_closed_form_in_interior():
    a, b = 0.3, 0.7
    x = torch.full((24, 24, 3), a, dtype=torch.float64)
    y = torch.full((24, 24, 3), b, dtype=torch.float64)
    s = Lo.ssim_map(x, y)[5:-5, 5:-5]
    want = (2 * a * b + Lo.SSIM_C1) / (a * a + b * b + Lo.SSIM_C1)
    assert torch.allclose(s, torch.full_like(s, want), atol=1e-12)


def _brute_ssim(x, y, i, j, c):
    g = Lo.gaussian_window().numpy()
    H, W = x.shape[:2]
    acc = np.zeros(5)
    for di in range(-5, 6):
        for dj in range(-5, 6):
            ii, jj = i + di, j + dj
            if 0 <= ii < H and 0 <= jj < W:
                xv, yv = x[ii, jj, c], y[ii, jj, c]
            else:
                xv = yv = 0.0  # zero padding
            w = g[di + 5] * g[dj + 5]
            acc += w * np.array([xv, yv, xv * xv, yv * yv, xv * yv])
    mx, my, exx, eyy, exy = acc
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return ((2 * mx * my + Lo.SSIM_C1) * (2 * cxy + Lo.SSIM_C2)) / (
        (mx * mx + my * my + Lo.SSIM_C1) * (vx + vy + Lo.SSIM_C2))


def test_ssim_matches_brute_force_window_sums_including_borders():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(17, 21, 3))
    y = np.clip(x + rng.normal(0, 0.2, size=x.shape), 0, 1)
    s = Lo.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    for (i, j, c) in [(0, 0, 0), (8, 10, 1), (16, 20, 2), (3, 19, 0), (12, 1, 2)]:
        assert abs(s[i, j, c] - _brute_ssim(x, y, i, j, c)) < 1e-12


def test_loss_components_and_objective_scale():
    x = torch.tensor([[[0.2, 0.5, 0.9]]], dtype=torch.float64)
    y = torch.tensor([[[0.4, 0.5, 0.1]]], dtype=torch.float64)
    l1, ls = Lo.loss_components(x, y, 0.0)
    assert torch.allclose(l1, torch.tensor([[[0.2, 0.0, 0.8]]], dtype=torch.float64))
    assert torch.all(ls == 0)
    l1, ls = Lo.loss_components(x, y, 0.2)
    assert torch.allclose(l1, 0.8 * torch.tensor([[[0.2, 0.0, 0.8]]], dtype=torch.float64))
    assert Lo.components_per_image(4, 5) == 120


def test_psnr_textbook():
    x = torch.zeros(4, 4, 3, dtype=torch.float64)
    y = torch.full((4, 4, 3), 0.1, dtype=torch.float64)
    assert abs(Lo.psnr(x, y) - 20.0) < 1e-12
