"""FP64 projection and front-to-back alpha blending, differentiable by autograd.

Paper: Background, "Review of Gaussian Splatting": pixel colour
C = sum_i c_i abar_i T_i with T_i = prod_{j<i} (1 - abar_j), over the
depth-sorted splats of the pixel's tile.  Readings (the paper is silent on the
rasteriser constants; these follow the original 3DGS design):

* abar = min(0.99, alpha exp(power)), power = -1/2 d^T conic d with d the
  offset from the splat centre to the pixel centre; power > 0 is skipped;
* alpha exp(power) < 1/255 is skipped -- a decision that picks which splats
  count, so it is taken in float32 exactly as the kernel takes it
  (``binning.contributes_f32``), while every value is computed in float64;
* if T (1 - abar) < 1e-4 the pixel stops before adding that splat;
* output C + T_final * background.

The per-tile lists come from ``binning.bin_view`` (float32 keys).  The stop
and clamp decisions are taken here in float64; all decisions are returned so
tests can detect one that flips between two nearby parameter vectors.  Pinned in
tests/test_oracle_render.py (one- and two-splat closed forms, T_final as a
product, the isotropic EWA closed form, central finite differences).
"""
from __future__ import annotations

import numpy as np
import torch

from .gaussians import DT, covariance, colour, split
from .binning import TILE, Bins, bin_view, contributes_f32

ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_STOP = 1e-4
NEAR = 0.2
DILATION = 0.3
FOV_CLAMP = 1.3


def cam_tensors(cam):
    W = torch.as_tensor(cam.R, dtype=DT)
    t = torch.as_tensor(cam.t, dtype=DT)
    centre = -(W.T @ t)
    return W, t, centre


def project(x: torch.Tensor, cam, sh_degree: int) -> dict:
    """Screen-space splat of every Gaussian: centre (u, v), conic, opacity, RGB."""
    p = split(x, sh_degree)
    W, t, centre = cam_tensors(cam)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    Sigma = covariance(p["log_s"], p["quat"])
    pc = p["mu"] @ W.T + t[None, :]
    z = pc[:, 2]
    limx = FOV_CLAMP * (0.5 * cam.width / fx)
    limy = FOV_CLAMP * (0.5 * cam.height / fy)
    txtz = torch.clamp(pc[:, 0] / z, -limx, limx)
    tytz = torch.clamp(pc[:, 1] / z, -limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([
        torch.stack([fx / z, zero, -fx * txtz / z], -1),
        torch.stack([zero, fy / z, -fy * tytz / z], -1),
    ], -2)
    T = J @ W[None]
    cov2 = T @ Sigma @ T.transpose(-1, -2)
    a = cov2[:, 0, 0] + DILATION
    b = cov2[:, 0, 1]
    c = cov2[:, 1, 1] + DILATION
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], -1)
    u = fx * pc[:, 0] / z + cx
    v = fy * pc[:, 1] / z + cy
    alpha = torch.sigmoid(p["logit"])
    rgb = colour(p["sh"], p["mu"], centre, sh_degree)
    return dict(u=u, v=v, conic=conic, alpha=alpha, rgb=rgb, depth=z)


def render(x: torch.Tensor, cam, sh_degree: int, bins: Bins | None = None, background=(0.0, 0.0, 0.0),
           return_aux: bool = False, tiles=None):
    """Render one view: image [H, W, 3] (and T_final, n_contrib, decisions).

    ``tiles`` (optional set of tile ids) restricts the work to those tiles;
    pixels of the other tiles are NaN.  Used to sample full-size views."""
    if bins is None:
        bins = bin_view(x.detach().to(torch.float32).numpy(), cam)
    pr = project(x, cam, sh_degree)
    H, Wd = cam.height, cam.width
    bg = torch.as_tensor(background, dtype=DT)
    rows = []
    T_rows = []
    n_rows = []
    decisions = {}
    for ty in range(bins.tiles_y):
        row_tiles = []
        row_T = []
        row_n = []
        for tx in range(bins.tiles_x):
            y_lo, y_hi = ty * TILE, min((ty + 1) * TILE, H)
            x_lo, x_hi = tx * TILE, min((tx + 1) * TILE, Wd)
            hh, ww = y_hi - y_lo, x_hi - x_lo
            gids = torch.as_tensor(bins.tile_list(ty * bins.tiles_x + tx), dtype=torch.long)
            if tiles is not None and (ty * bins.tiles_x + tx) not in tiles:
                row_tiles.append(torch.full((hh, ww, 3), float("nan"), dtype=DT))
                row_T.append(torch.full((hh, ww), float("nan"), dtype=DT))
                row_n.append(torch.zeros(hh, ww, dtype=torch.long))
                continue
            if gids.numel() == 0:
                row_tiles.append(bg.expand(hh, ww, 3).clone())
                row_T.append(torch.ones(hh, ww, dtype=DT))
                row_n.append(torch.zeros(hh, ww, dtype=torch.long))
                continue
            py, px = torch.meshgrid(torch.arange(y_lo, y_hi, dtype=DT) + 0.5,
                                    torch.arange(x_lo, x_hi, dtype=DT) + 0.5, indexing="ij")
            px = px.reshape(-1, 1)
            py = py.reshape(-1, 1)
            dx = pr["u"][gids][None, :] - px
            dy = pr["v"][gids][None, :] - py
            cn = pr["conic"][gids]
            power = -0.5 * (cn[None, :, 0] * dx * dx + cn[None, :, 2] * dy * dy) - cn[None, :, 1] * dx * dy
            abar = torch.clamp(pr["alpha"][gids][None, :] * torch.exp(power), max=ALPHA_MAX)
            gy, gx = np.meshgrid(np.arange(y_lo, y_hi) + 0.5, np.arange(x_lo, x_hi) + 0.5, indexing="ij")
            tile_ids = bins.tile_list(ty * bins.tiles_x + tx)
            valid = torch.as_tensor(contributes_f32(bins.dec, tile_ids, gx.reshape(-1), gy.reshape(-1)))
            a_eff = torch.where(valid, abar, torch.zeros_like(abar))
            one_minus = 1.0 - a_eff
            T_incl = torch.cumprod(one_minus, dim=1)
            with torch.no_grad():
                below = T_incl < T_STOP
                L = below.shape[1]
                idx = torch.arange(L)
                first = torch.where(below, idx[None, :], torch.full_like(below, L, dtype=torch.long)).min(1).values
                keep = idx[None, :] < first[:, None]
            T_excl = torch.cat([torch.ones_like(T_incl[:, :1]), T_incl[:, :-1]], 1)
            wgt = torch.where(keep, a_eff * T_excl, torch.zeros_like(a_eff))
            col = wgt @ pr["rgb"][gids]
            T_fin = torch.prod(torch.where(keep, one_minus, torch.ones_like(one_minus)), 1)
            out = col + T_fin[:, None] * bg[None, :]
            with torch.no_grad():
                used = keep & valid
                last = torch.where(used, idx[None, :] + 1, torch.zeros_like(idx)[None, :]).max(1).values
            row_tiles.append(out.reshape(hh, ww, 3))
            row_T.append(T_fin.reshape(hh, ww))
            row_n.append(last.reshape(hh, ww))
            if return_aux:
                decisions[ty * bins.tiles_x + tx] = (valid.clone(), keep.clone(), (abar >= ALPHA_MAX).detach())
        rows.append(torch.cat(row_tiles, 1))
        T_rows.append(torch.cat(row_T, 1))
        n_rows.append(torch.cat(row_n, 1))
    img = torch.cat(rows, 0)
    if not return_aux:
        return img
    return img, dict(T_final=torch.cat(T_rows, 0), n_contrib=torch.cat(n_rows, 0), decisions=decisions,
                     bins=bins, proj=pr)


def decisions_equal(d1: dict, d2: dict) -> bool:
    """True when every skip / stop / clamp decision agrees between two renders."""
    if d1.keys() != d2.keys():
        return False
    for k in d1:
        for a, b in zip(d1[k], d2[k]):
            if not torch.equal(a, b):
                return False
    return True


def decision_flips(x, cam, sh_degree: int, bins: Bins | None = None, tiles=None) -> dict:
    """How many blend decisions float32 arithmetic takes differently from
    exact float64 arithmetic on one view (a report beside a parity figure;
    the render itself takes the skip decision in float32, see above).

    skip:  the float32 log-domain rule (``binning.contributes_f32``) against
           power <= 0 and alpha exp(power) >= 1/255 from the float64 splat;
    clamp: float32 alpha exp(power) >= 0.99 against float64;
    stop:  the index where a pixel's walk stops, float32 transmittance and
           opacities against float64.
    skip and clamp count (pixel, splat) evaluations up to the pixel's float64
    stop (the splat that stops the walk included); stop counts pixels.  ``evaluations`` and ``pixels`` are the totals.
    """
    x = torch.as_tensor(np.asarray(x, np.float64))
    if bins is None:
        bins = bin_view(x.numpy().astype(np.float32), cam)
    with torch.no_grad():
        pr = project(x, cam, sh_degree)
    u, v = pr["u"].numpy(), pr["v"].numpy()
    con = pr["conic"].numpy()
    alpha = pr["alpha"].numpy()
    f32 = np.float32
    out = dict(skip=0, clamp=0, stop=0, evaluations=0, pixels=0)
    H, Wd = cam.height, cam.width
    for t in range(bins.tiles_x * bins.tiles_y):
        if tiles is not None and t not in tiles:
            continue
        gids = bins.tile_list(t)
        if len(gids) == 0:
            continue
        ty, tx = divmod(t, bins.tiles_x)
        gy, gx = np.meshgrid(np.arange(ty * TILE, min((ty + 1) * TILE, H)) + 0.5,
                             np.arange(tx * TILE, min((tx + 1) * TILE, Wd)) + 0.5, indexing="ij")
        px, py = gx.reshape(-1, 1), gy.reshape(-1, 1)
        dx, dy = u[gids][None, :] - px, v[gids][None, :] - py
        p64 = -0.5 * (con[gids, 0][None, :] * dx * dx + con[gids, 2][None, :] * dy * dy) - con[gids, 1][None, :] * dx * dy
        a64 = alpha[gids][None, :] * np.exp(p64)
        valid64 = (p64 <= 0) & (a64 >= 1.0 / 255.0)
        valid32 = contributes_f32(bins.dec, gids, gx.reshape(-1), gy.reshape(-1))
        from .binning import power_f32

        with np.errstate(all="ignore"):
            p32 = power_f32(bins.dec, gids, gx.reshape(-1), gy.reshape(-1))
            al32 = alpha[gids].astype(f32)[None, :]
            a32 = al32 * np.exp(p32)
        ab64 = np.where(valid64, np.minimum(a64, ALPHA_MAX), 0.0)
        ab32 = np.where(valid32, np.minimum(a32, f32(ALPHA_MAX)), f32(0.0)).astype(f32)
        T64 = np.cumprod(1.0 - ab64, axis=1)
        T32 = np.cumprod((f32(1.0) - ab32).astype(f32), axis=1, dtype=f32)
        L = len(gids)
        stop64 = np.where((T64 < T_STOP).any(1), (T64 < T_STOP).argmax(1), L)
        stop32 = np.where((T32 < f32(T_STOP)).any(1), (T32 < f32(T_STOP)).argmax(1), L)
        before = np.arange(L)[None, :] <= stop64[:, None]  # the stopping splat is evaluated too
        out["skip"] += int(((valid64 != valid32) & before).sum())
        both = valid64 & valid32 & before
        out["clamp"] += int(((a64 >= ALPHA_MAX) != (a32 >= f32(ALPHA_MAX)))[both].sum())
        out["stop"] += int((stop64 != stop32).sum())
        out["evaluations"] += int(before.sum())
        out["pixels"] += int(px.shape[0])
    return out
