"""Projection, tile keys, stable sort and per-tile ranges in IEEE float32.

The paper renders with a tile-based rasteriser (Background, "Review of
Gaussian Splatting"): Gaussians are projected to 2D splats, duplicated per
16x16 tile they overlap, and sorted by depth within each tile; the sort order
is what makes the loss only piecewise continuous (Introduction).  The paper
gives no constants for this stage; the readings below are those of the
original 3DGS design:

* near plane z <= 0.2 culls; pinhole u = f_x p_x / p_z + c_x (pixel i has its
  centre at i + 1/2);
* EWA screen covariance with the camera-space x/z, y/z clamped to
  +-1.3 tan(fov/2) inside the Jacobian, plus 0.3 px^2 of dilation;
  det <= 0 culls;
* radius r = ceil(3 sqrt(lambda_max)), lambda_max = mid + sqrt(max(mid^2 - det, 0));
* tile rectangle x in [clamp(floor((u - r)/16)), clamp(floor((u + r)/16) + 1)),
  same in y, clamped to the tile grid; an empty rectangle culls;
* key = (tile_id << 32) | float32 bits of depth p_z; pairs are emitted by
  Gaussian index, then tile row, then tile column, and sorted stably.

Because a float64 key could never equal a float32 GPU key, this stage alone is
written op for op in float32 (numpy float32 is IEEE round-to-nearest with no
fused multiply-add; exp of the log-scale is taken in float64 and rounded).

The same holds for the blend's skip decision, which decides an integer (which
splats contribute to a pixel) from floating point: it is taken in float32 on
both sides.  A splat is skipped at a pixel when its float32 power
-1/2 (a dx^2 + c dy^2) - b dx dy (evaluated left to right) is positive or
below tau = float32(-ln(255 alpha)); that is the 1/255 opacity threshold
alpha exp(power) < 1/255 moved to the log domain, where it needs no exp.
alpha = float32(sigmoid(logit)) is evaluated in float64 and rounded; the
conic is (c, -b, a) / det of the float32 screen covariance.
Pinned in tests/test_oracle_binning.py by brute-force rectangle checks, a
principal-ray projection and sort invariants.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TILE = 16
F = np.float32


@dataclass
class Bins:
    tiles_x: int
    tiles_y: int
    visible: np.ndarray  # bool[N]
    depth_bits: np.ndarray  # uint32[N]
    rect: np.ndarray  # int32[N, 4]: x0, y0, x1, y1 (half-open)
    tiles_touched: np.ndarray  # int64[N]
    keys: np.ndarray  # uint64[Pi], sorted
    gids: np.ndarray  # int64[Pi], Gaussian index of each sorted pair
    ranges: np.ndarray  # int64[tiles, 2], [start, end) into the sorted pairs
    dec: dict = None  # float32 decision inputs per Gaussian: u, v, conic_a, conic_b, conic_c, tau

    def tile_list(self, tile_id: int) -> np.ndarray:
        s, e = self.ranges[tile_id]
        return self.gids[s:e]


def project_f32(x32: np.ndarray, cam) -> dict:
    """Key-determining quantities of every Gaussian for one camera, float32."""
    x32 = np.asarray(x32, F)
    mu = x32[0:3]
    s = np.exp(x32[3:6].astype(np.float64)).astype(F)
    qx, qy, qz, qw = x32[6], x32[7], x32[8], x32[9]
    two = F(2.0)
    with np.errstate(all="ignore"):
        r2 = ((qx * qx + qy * qy) + qz * qz) + qw * qw
        Rt = [
            [((qw * qw + qx * qx) - qy * qy) - qz * qz, two * (qx * qy - qw * qz), two * (qx * qz + qw * qy)],
            [two * (qx * qy + qw * qz), ((qw * qw - qx * qx) + qy * qy) - qz * qz, two * (qy * qz - qw * qx)],
            [two * (qx * qz - qw * qy), two * (qy * qz + qw * qx), ((qw * qw - qx * qx) - qy * qy) + qz * qz],
        ]
        R = [[Rt[i][j] / r2 for j in range(3)] for i in range(3)]
        M = [[R[i][j] * s[j] for j in range(3)] for i in range(3)]
        W = np.asarray(cam.R, F)
        t = np.asarray(cam.t, F)
        p = [((W[i, 0] * mu[0] + W[i, 1] * mu[1]) + W[i, 2] * mu[2]) + t[i] for i in range(3)]
        fx, fy, cx, cy = F(cam.fx), F(cam.fy), F(cam.cx), F(cam.cy)
        limx = F(1.3) * ((F(cam.width) * F(0.5)) / fx)
        limy = F(1.3) * ((F(cam.height) * F(0.5)) / fy)
        txtz = np.minimum(limx, np.maximum(-limx, p[0] / p[2]))
        tytz = np.minimum(limy, np.maximum(-limy, p[1] / p[2]))
        j00 = fx / p[2]
        j02 = -(fx * txtz) / p[2]
        j11 = fy / p[2]
        j12 = -(fy * tytz) / p[2]
        T0 = [j00 * W[0, k] + j02 * W[2, k] for k in range(3)]
        T1 = [j11 * W[1, k] + j12 * W[2, k] for k in range(3)]
        V0 = [(T0[0] * M[0][j] + T0[1] * M[1][j]) + T0[2] * M[2][j] for j in range(3)]
        V1 = [(T1[0] * M[0][j] + T1[1] * M[1][j]) + T1[2] * M[2][j] for j in range(3)]
        dil = F(0.3)
        a = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + dil
        b = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2]
        c = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + dil
        det = a * c - b * b
        mid = F(0.5) * (a + c)
        lam = mid + np.sqrt(np.maximum(mid * mid - det, F(0.0)))
        radius = np.ceil(F(3.0) * np.sqrt(lam))
        u = (fx * p[0]) / p[2] + cx
        v = (fy * p[1]) / p[2] + cy
        conic = (c / det, -b / det, a / det)
        alpha = (1.0 / (1.0 + np.exp(-x32[10].astype(np.float64)))).astype(F)
        tau = (-np.log(255.0 * alpha.astype(np.float64))).astype(F)
    tx = (cam.width + TILE - 1) // TILE
    ty = (cam.height + TILE - 1) // TILE
    inv = F(1.0 / TILE)
    with np.errstate(all="ignore"):
        x0 = np.clip(np.floor((u - radius) * inv), F(0), F(tx))
        x1 = np.clip(np.floor((u + radius) * inv) + F(1), F(0), F(tx))
        y0 = np.clip(np.floor((v - radius) * inv), F(0), F(ty))
        y1 = np.clip(np.floor((v + radius) * inv) + F(1), F(0), F(ty))
    visible = (p[2] > F(0.2)) & (det > F(0.0)) & np.isfinite(u) & np.isfinite(v) & np.isfinite(radius)
    x0 = np.where(visible, x0, 0).astype(np.int64)
    x1 = np.where(visible, x1, 0).astype(np.int64)
    y0 = np.where(visible, y0, 0).astype(np.int64)
    y1 = np.where(visible, y1, 0).astype(np.int64)
    touched = np.maximum(x1 - x0, 0) * np.maximum(y1 - y0, 0)
    visible &= touched > 0
    touched = np.where(visible, touched, 0)
    return dict(visible=visible, depth=p[2].astype(F), u=u, v=v, radius=radius, det=det, cov2=(a, b, c),
                conic=conic, alpha=alpha, tau=tau,
                rect=np.stack([x0, y0, x1, y1], 1).astype(np.int32), tiles_touched=touched,
                tiles_x=tx, tiles_y=ty)


def bin_view(x32: np.ndarray, cam) -> Bins:
    """Emit (key, Gaussian) pairs, sort them stably and find each tile's range."""
    pr = project_f32(x32, cam)
    tx, ty = pr["tiles_x"], pr["tiles_y"]
    vis = pr["visible"]
    depth_bits = np.where(vis, pr["depth"].view(np.uint32), 0).astype(np.uint32)
    rect = pr["rect"].astype(np.int64)
    touched = pr["tiles_touched"].astype(np.int64)
    total = int(touched.sum())
    gid = np.repeat(np.arange(len(touched)), touched)
    offs = np.cumsum(touched) - touched
    local = np.arange(total) - np.repeat(offs, touched)
    w = np.repeat(rect[:, 2] - rect[:, 0], touched)
    ty_ = np.repeat(rect[:, 1], touched) + local // np.maximum(w, 1)
    tx_ = np.repeat(rect[:, 0], touched) + local % np.maximum(w, 1)
    tile = ty_ * tx + tx_
    keys = (tile.astype(np.uint64) << np.uint64(32)) | depth_bits[gid].astype(np.uint64)
    order = np.argsort(keys, kind="stable")
    keys_sorted = keys[order]
    gids_sorted = gid[order]
    tile_sorted = (keys_sorted >> np.uint64(32)).astype(np.int64)
    n_tiles = tx * ty
    starts = np.searchsorted(tile_sorted, np.arange(n_tiles), side="left")
    ends = np.searchsorted(tile_sorted, np.arange(n_tiles), side="right")
    dec = dict(u=pr["u"], v=pr["v"], ca=pr["conic"][0], cb=pr["conic"][1], cc=pr["conic"][2], tau=pr["tau"])
    return Bins(tx, ty, vis, depth_bits, pr["rect"], touched, keys_sorted, gids_sorted,
                np.stack([starts, ends], 1), dec)


def power_f32(dec: dict, gids: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """float32 power of splats `gids` at pixel centres (px, py): [pixels, len(gids)]."""
    with np.errstate(all="ignore"):
        dx = dec["u"][gids][None, :] - px.astype(F)[:, None]
        dy = dec["v"][gids][None, :] - py.astype(F)[:, None]
        ca, cb, cc = dec["ca"][gids][None, :], dec["cb"][gids][None, :], dec["cc"][gids][None, :]
        return F(-0.5) * ((ca * dx) * dx + (cc * dy) * dy) - (cb * dx) * dy


def contributes_f32(dec: dict, gids: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """The skip decision: True where the splat is not skipped (power <= 0 and power >= tau)."""
    pw = power_f32(dec, gids, px, py)
    return (pw <= F(0.0)) & (pw >= dec["tau"][gids][None, :])
