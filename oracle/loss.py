"""Per-pixel loss components and the least-squares objective (FP64).

Paper: Background, Eq. pixel_loss (L = (1 - lambda) L1 + lambda D-SSIM, split
into one component per RGB channel) and Eq. objective (f = 1/(2m) ||F||^2 with
F the square roots of all m = 6 H W M loss components).  Readings:

* lambda = 0.2 and D-SSIM = 1 - SSIM (3DGS defaults; the paper gives neither);
* SSIM per channel with an 11x11 Gaussian window (sigma 1.5), zero-padded
  "same" filtering, C1 = 0.01^2, C2 = 0.03^2 (Wang et al.);
* component values: l1 = (1 - lambda)|r|, ls = lambda (1 - SSIM), so that
  f = 1/(2m) sum(l1 + ls) since each entry of F is the square root of one.

Pinned in tests/test_oracle_loss.py: SSIM(x, x) = 1, the closed form for
constant images, a brute-force window sum at sampled pixels, and L1 values.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as Fn

from .gaussians import DT

SSIM_WIN = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def gaussian_window(size: int = SSIM_WIN, sigma: float = SSIM_SIGMA) -> torch.Tensor:
    r = torch.arange(size, dtype=DT) - (size // 2)
    g = torch.exp(-(r * r) / (2.0 * sigma * sigma))
    return g / g.sum()


def _filter(img_chw: torch.Tensor) -> torch.Tensor:
    """Zero-padded same-size 2D Gaussian filtering of each channel."""
    g = gaussian_window()
    w2 = torch.outer(g, g)[None, None].expand(img_chw.shape[0], 1, SSIM_WIN, SSIM_WIN)
    return Fn.conv2d(img_chw[None], w2, padding=SSIM_WIN // 2, groups=img_chw.shape[0])[0]


def ssim_map(img: torch.Tensor, tgt: torch.Tensor) -> torch.Tensor:
    """SSIM at every pixel and channel; img, tgt: [H, W, 3] -> [H, W, 3]."""
    x = img.permute(2, 0, 1)
    y = tgt.permute(2, 0, 1).to(img.dtype)
    mx, my = _filter(x), _filter(y)
    sxx = _filter(x * x) - mx * mx
    syy = _filter(y * y) - my * my
    sxy = _filter(x * y) - mx * my
    num = (2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)
    den = (mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)
    return (num / den).permute(1, 2, 0)


def loss_components(img: torch.Tensor, tgt: torch.Tensor, lam: float):
    """(l1, ls): the 2 x 3 loss components of every pixel, each [H, W, 3]."""
    r = img - tgt.to(img.dtype)
    l1 = (1.0 - lam) * torch.abs(r)
    if lam == 0.0:
        return l1, torch.zeros_like(l1)
    ls = lam * (1.0 - ssim_map(img, tgt))
    return l1, ls


def components_per_image(h: int, w: int) -> int:
    """Each image contributes 6 H W components (2 loss types x 3 channels)."""
    return 6 * h * w


def psnr(img: torch.Tensor, tgt: torch.Tensor) -> float:
    """10 log10(1 / MSE) over pixels and channels (images in [0, 1])."""
    mse = float(((img.to(DT) - tgt.to(DT)) ** 2).mean())
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf")
