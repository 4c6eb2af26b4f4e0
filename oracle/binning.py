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
* tile list (see tile_spans): the tiles of the rectangle whose block of pixel
  centres the splat's skip ellipse, widened for float32 rounding, can reach;
  a splat that reaches none culls;
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
    visible &= (x1 > x0) & (y1 > y0)
    rect = np.stack([x0, y0, x1, y1], 1)
    spans = tile_spans(u, v, conic, tau, rect, visible)
    touched = np.maximum(spans[:, :, 1] - spans[:, :, 0], 0).sum(axis=1) if spans.size else np.zeros(len(u), np.int64)
    visible &= touched > 0
    touched = np.where(visible, touched, 0)
    return dict(visible=visible, depth=p[2].astype(F), u=u, v=v, radius=radius, det=det, cov2=(a, b, c),
                conic=conic, alpha=alpha, tau=tau,
                rect=rect.astype(np.int32), tiles_touched=touched, spans=spans,
                tiles_x=tx, tiles_y=ty)


def tile_spans(u, v, conic, tau, rect, visible) -> np.ndarray:
    """Which tiles of each splat's rectangle the splat can reach: int64
    [N, max rows, 2], the half-open column range [lo, hi) of rectangle row j
    (tile row y0 + j), empty where hi <= lo.

    The skip test passes only where the float32 power p of -1/2 d^T Q d is at
    least tau, Q = (a, b; b, c) the conic of the record: (a, b, c) = (-2 qa,
    -qb, -2 qc) for the stored qa = -a/2, qb = -b, qc = -c/2.  The float32
    power errs by at most a relative 4u (1 + rho) / (1 - rho) (u = 2^-24,
    rho^2 = b^2 / (a c)), below 1e-3 for rho^2 <= 0.999, so every passing
    pixel centre lies in E = {d : d^T Q d <= k}, k = 2.02 (-tau) + 1e-3, with
    room to spare (the extra 0.9% of k, and a 0.01-pixel margin on every edge
    below, cover the float32 rounding of the extent computed here, a few
    1e-4 relative at most).  A tile is listed when E meets the 16 x 16 block
    of pixel centres of the tile, widened by the margin: the band of rows
    [16 ty + 0.49, 16 ty + 15.51] cuts E in a convex set whose x-extent runs
    from the left end of E at the band row nearest E's leftmost point to the
    right end at the row nearest its rightmost point.  The rightmost point
    of E is (xm, yr), xm = sqrt(k c / det), yr = -b xm / c, det = a c - b^2;
    the leftmost is (-xm, -yr); E spans |y| <= sqrt(k a / det); at height y
    it covers x in ((-b y) -+ sqrt(k a - det y^2)) / a.  Columns of the
    x-extent [xl, xr] (relative to u): ceil((u + xl - 15.51) / 16) to
    floor((u + xr - 0.49) / 16), clipped to the rectangle.  Splats with
    rho^2 > 0.999 or a conic that is not positive definite or finite keep
    the whole rectangle; tau > 0 reaches nothing.  Each step is written out
    in float32 in a fixed order (numpy float32 is IEEE round-to-nearest with
    no fused multiply-add), since the listed tiles are integers decided from
    floating point.
    """
    n = len(u)
    h = np.where(visible, rect[:, 3] - rect[:, 1], 0)
    rows = int(h.max()) if n else 0
    spans = np.zeros((n, rows, 2), np.int64)
    if rows == 0:
        return spans
    ca, cb, cc = (np.asarray(t, F) for t in conic)
    qa, qb, qc = F(-0.5) * ca, -cb, F(-0.5) * cc
    a, b, c = F(-2.0) * qa, -qb, F(-2.0) * qc
    tau32 = np.asarray(tau, F)
    uu, vv = np.asarray(u, F), np.asarray(v, F)
    x0, y0, x1 = rect[:, 0].astype(F), rect[:, 1], rect[:, 2].astype(F)
    with np.errstate(all="ignore"):
        det = a * c - b * b
        ellipse = (a > F(0)) & (c > F(0)) & (det * F(1000.0) >= a * c) & (det < F(np.inf))
        whole = ~ellipse
        none = tau32 > F(0.0)
        k = F(-2.02) * tau32 + F(1e-3)
        ka = k * a
        inv_a = F(1.0) / a
        ymax = np.sqrt(ka / det)
        yr = (-b * np.sqrt((k * c) / det)) / c
        for j in range(rows):
            row = F(16.0) * (y0 + j).astype(F)
            ya = np.fmax((row + F(0.49)) - vv, -ymax)
            yb = np.fmin((row + F(15.51)) - vv, ymax)
            y_r = np.fmin(np.fmax(yr, ya), yb)
            y_l = np.fmin(np.fmax(-yr, ya), yb)
            xr = (-b * y_r + np.sqrt(np.fmax(ka - (det * y_r) * y_r, F(0.0)))) * inv_a
            xl = (-b * y_l - np.sqrt(np.fmax(ka - (det * y_l) * y_l, F(0.0)))) * inv_a
            clo = np.ceil(((uu + xl) - F(15.51)) * F(0.0625))
            chi = np.floor(((uu + xr) - F(0.49)) * F(0.0625)) + F(1.0)
            lo = np.fmin(np.fmax(clo, x0), x1)
            hi = np.fmax(np.fmin(chi, x1), x0)
            empty = ~(ya <= yb)
            lo = np.where(whole, x0, np.where(empty, x0, lo))
            hi = np.where(whole, x1, np.where(empty, x0, hi))
            live = visible & (j < h) & ~none
            spans[:, j, 0] = np.where(live, lo, 0).astype(np.int64)
            spans[:, j, 1] = np.where(live, hi, 0).astype(np.int64)
    return spans


def bin_view(x32: np.ndarray, cam) -> Bins:
    """Emit (key, Gaussian) pairs, sort them stably and find each tile's range."""
    pr = project_f32(x32, cam)
    tx, ty = pr["tiles_x"], pr["tiles_y"]
    vis = pr["visible"]
    depth_bits = np.where(vis, pr["depth"].view(np.uint32), 0).astype(np.uint32)
    rect = pr["rect"].astype(np.int64)
    touched = pr["tiles_touched"].astype(np.int64)
    spans = pr["spans"]
    # one segment per (Gaussian, rectangle row) with listed tiles, in
    # Gaussian then row order, expanded into its columns
    seg_n = np.maximum(spans[:, :, 1] - spans[:, :, 0], 0) if spans.size else np.zeros((len(touched), 0), np.int64)
    seg_n = np.where(vis[:, None], seg_n, 0).reshape(-1)
    rows = spans.shape[1]
    seg_g = np.repeat(np.arange(len(touched)), rows)
    seg_ty = rect[seg_g, 1] + np.tile(np.arange(rows), len(touched))
    seg_lo = spans[:, :, 0].reshape(-1) if spans.size else np.zeros(0, np.int64)
    keep = seg_n > 0
    seg_g, seg_ty, seg_lo, seg_n = seg_g[keep], seg_ty[keep], seg_lo[keep], seg_n[keep]
    total = int(seg_n.sum())
    assert total == int(touched.sum())
    gid = np.repeat(seg_g, seg_n)
    first = np.cumsum(seg_n) - seg_n
    tx_ = np.repeat(seg_lo, seg_n) + (np.arange(total) - np.repeat(first, seg_n))
    ty_ = np.repeat(seg_ty, seg_n)
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
