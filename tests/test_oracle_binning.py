"""Pins of the oracle's float32 binning: projection, rectangles, keys and order."""
import math

import numpy as np
import torch

import synthetic as syn
from oracle import binning as B
from oracle import render as R


def _one_gaussian(mu, log_s=(-2.0, -2.0, -2.0), q=(0, 0, 0, 1.0), logit=0.0, rgb_dc=(0.0, 0.0, 0.0)):
    x = np.zeros((14, 1), np.float32)
    x[0:3, 0] = mu
    x[3:6, 0] = log_s
    x[6:10, 0] = q
    x[10, 0] = logit
    x[11:14, 0] = rgb_dc
    return x


def test_principal_ray_projects_to_image_centre():
    cam = syn.make_camera((0.0, -4.0, 0.0), 64, 48)
    pr = B.project_f32(_one_gaussian((0, 0, 0)), cam)
    assert pr["u"][0] == np.float32(32.0) and pr["v"][0] == np.float32(24.0)
    assert pr["depth"][0] == np.float32(4.0)


def test_isotropic_ewa_closed_form_on_axis():
    # On the principal ray an isotropic Gaussian projects to (f s / z)^2 I + 0.3 I.
    cam = syn.make_camera((0.0, -4.0, 0.0), 64, 64)
    s = 0.1
    pr = B.project_f32(_one_gaussian((0, 0, 0), log_s=(math.log(s),) * 3), cam)
    a, b, c = (float(v[0]) for v in pr["cov2"])
    want = (cam.fx * s / 4.0) ** 2 + 0.3
    assert abs(a - want) < 2e-6 * want and abs(c - want) < 2e-6 * want and abs(b) < 1e-6
    assert pr["radius"][0] == math.ceil(3.0 * math.sqrt(float(np.float32(a))))


def test_culling_near_plane_and_behind():
    cam = syn.make_camera((0.0, -4.0, 0.0), 64, 64)
    x = np.concatenate([_one_gaussian((0, -3.85, 0)), _one_gaussian((0, -3.75, 0)), _one_gaussian((0, -6, 0))], 1)
    pr = B.project_f32(x, cam)
    assert pr["visible"].tolist() == [False, True, False]


def _brute_rect(u, v, r, tx, ty):
    lo_x, hi_x = np.float32(u - r), np.float32(u + r)
    lo_y, hi_y = np.float32(v - r), np.float32(v + r)
    xs = [k for k in range(tx) if 16 * k <= float(hi_x) and 16 * (k + 1) > float(lo_x)]
    ys = [k for k in range(ty) if 16 * k <= float(hi_y) and 16 * (k + 1) > float(lo_y)]
    return xs, ys


def test_tile_rectangles_match_brute_force_enumeration():
    sc = syn.config1_scene()
    cam = syn.make_camera((0.3, -3.0, 0.4), 80, 56)  # ragged: 5 x 4 tiles, last row partial
    x = sc.gt.copy()
    x[3:6] += 1.2  # larger splats so rectangles span several tiles
    pr = B.project_f32(x, cam)
    assert pr["tiles_x"] == 5 and pr["tiles_y"] == 4
    n_checked = 0
    for g in range(x.shape[1]):
        if not (pr["depth"][g] > np.float32(0.2) and pr["det"][g] > 0):
            continue
        xs, ys = _brute_rect(pr["u"][g], pr["v"][g], pr["radius"][g], 5, 4)
        x0, y0, x1, y1 = pr["rect"][g]
        if x1 > x0 and y1 > y0:
            assert list(range(x0, x1)) == xs and list(range(y0, y1)) == ys
            n_checked += 1
        else:
            assert len(xs) == 0 or len(ys) == 0
            assert not pr["visible"][g]
    assert n_checked > 1000


def test_keys_order_and_ranges_invariants():
    sc = syn.config1_scene()
    cam = sc.cameras[3]
    b = B.bin_view(sc.gt, cam)
    tiles = (b.keys >> np.uint64(32)).astype(np.int64)
    assert np.all(np.diff(b.keys.astype(np.float64)) >= 0) or np.all(b.keys[1:] >= b.keys[:-1])
    assert len(b.keys) == int(b.tiles_touched.sum())
    # each visible Gaussian occurs exactly once in each tile of its tile
    # list, and only in tiles of its rectangle
    spans = B.project_f32(sc.gt, cam)["spans"]
    for g in np.flatnonzero(b.visible)[:300]:
        x0, y0, x1, y1 = b.rect[g]
        want = sorted((y0 + j) * b.tiles_x + tx for j in range(y1 - y0) for tx in range(*spans[g, j]))
        got = sorted(tiles[b.gids == g].tolist())
        assert got == want and len(got) == b.tiles_touched[g] > 0
        assert all(x0 <= t % b.tiles_x < x1 and y0 <= t // b.tiles_x < y1 for t in got)
    # ranges partition the sorted pairs by tile; within a tile depth is
    # non-decreasing and equal depths keep Gaussian order (stable sort)
    assert b.ranges[0, 0] == 0 and b.ranges[-1, 1] == len(b.keys)
    for t in range(b.tiles_x * b.tiles_y):
        s, e = b.ranges[t]
        assert np.all(tiles[s:e] == t)
        d = (b.keys[s:e] & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
        assert np.all(np.diff(d) >= 0)
        assert np.all(d == b.depth_bits[b.gids[s:e]].view(np.float32))
        same = np.diff(d) == 0
        assert np.all(np.diff(b.gids[s:e])[same] > 0)


def test_float32_binning_agrees_with_float64_projection():
    sc = syn.config1_scene()
    cam = sc.cameras[0]
    pr32 = B.project_f32(sc.gt, cam)
    pr64 = R.project(torch.tensor(sc.gt, dtype=torch.float64), cam, 0)
    vis = pr32["visible"]
    assert np.allclose(pr32["u"][vis], pr64["u"].numpy()[vis], rtol=1e-5, atol=1e-4)
    assert np.allclose(pr32["v"][vis], pr64["v"].numpy()[vis], rtol=1e-5, atol=1e-4)
    assert np.allclose(pr32["depth"][vis], pr64["depth"].numpy()[vis], rtol=1e-6)
    a, b, c = pr32["cov2"]
    det64 = 1.0 / (pr64["conic"][:, 0] * pr64["conic"][:, 2] - pr64["conic"][:, 1] ** 2)
    assert np.allclose((a * c - b * b)[vis], det64.numpy()[vis], rtol=1e-4)


def test_log_domain_skip_threshold_matches_the_opacity_threshold():
    # alpha exp(power) < 1/255  <=>  power < -ln(255 alpha): the float32 form
    # agrees with the exact float64 test except within rounding of the boundary
    rng = np.random.default_rng(3)
    logit = rng.normal(0, 2, size=200000).astype(np.float32)
    alpha = (1.0 / (1.0 + np.exp(-logit.astype(np.float64)))).astype(np.float32)
    tau = (-np.log(255.0 * alpha.astype(np.float64))).astype(np.float32)
    power = rng.uniform(-9, 0, size=logit.size).astype(np.float32)
    exact = alpha.astype(np.float64) * np.exp(power.astype(np.float64)) < 1.0 / 255.0
    f32 = power < tau
    margin = np.abs(np.log(255.0 * alpha.astype(np.float64)) + power.astype(np.float64))
    assert np.all(exact[margin > 1e-6] == f32[margin > 1e-6])
    assert (exact != f32).mean() < 1e-4
    # bins carry the float32 decision inputs
    sc = syn.config1_scene()
    b = B.bin_view(sc.gt, sc.cameras[0])
    assert b.dec["tau"].dtype == np.float32 and b.dec["ca"].dtype == np.float32
    pr = B.project_f32(sc.gt, sc.cameras[0])
    a, bb, c = pr["cov2"]
    assert np.array_equal(b.dec["ca"], c / (a * c - bb * bb))


def _varied_splats(seed, n=600):
    """Anisotropic, rotated splats of every opacity in front of a 160x128 camera."""
    rng = np.random.default_rng(seed)
    x = np.zeros((14, n), np.float32)
    x[0] = rng.uniform(-1.2, 1.2, n)
    x[1] = rng.uniform(-0.8, 0.8, n)
    x[2] = rng.uniform(-1.0, 1.0, n)
    x[3:6] = rng.normal(np.log(0.06), 0.8, (3, n))
    q = rng.normal(size=(4, n))
    x[6:10] = q / np.linalg.norm(q, axis=0)
    x[10] = rng.normal(0.0, 3.0, n)  # opacities from ~0 to ~1 (some below 1/255)
    cam = syn.make_camera((0.2, -3.5, 0.3), 160, 128)
    return x, cam


def test_tile_lists_hold_every_reached_pixel():
    """Brute force: every pixel centre where a splat passes the float32 skip
    test lies in a tile of that splat's list, so the render and its
    derivatives equal those of the whole rectangle."""
    for seed in (11, 12):
        x, cam = _varied_splats(seed)
        b = B.bin_view(x, cam)
        pr = B.project_f32(x, cam)
        tiles = (b.keys >> np.uint64(32)).astype(np.int64)
        listed = {(int(g), int(t)) for g, t in zip(b.gids, tiles)}
        py, px = np.meshgrid(np.arange(cam.height) + 0.5, np.arange(cam.width) + 0.5, indexing="ij")
        px, py = px.reshape(-1), py.reshape(-1)
        rect_ok = (pr["rect"][:, 2] > pr["rect"][:, 0]) & (pr["rect"][:, 3] > pr["rect"][:, 1])
        gs = np.flatnonzero(rect_ok)
        reached = 0
        for g in gs:
            hit = B.contributes_f32(b.dec, np.array([g]), px, py)[:, 0]
            if not hit.any():
                continue
            t = (py[hit] // 16).astype(np.int64) * b.tiles_x + (px[hit] // 16).astype(np.int64)
            x0, y0, x1, y1 = pr["rect"][g]
            in_rect = (t % b.tiles_x >= x0) & (t % b.tiles_x < x1) & (t // b.tiles_x >= y0) & (t // b.tiles_x < y1)
            for tt in np.unique(t[in_rect]):
                assert (int(g), int(tt)) in listed, (seed, g, tt)
                reached += 1
        assert reached > 500
        # and the lists drop tiles: fewer pairs than the rectangles hold
        area = (pr["rect"][:, 2] - pr["rect"][:, 0]) * (pr["rect"][:, 3] - pr["rect"][:, 1])
        assert len(b.gids) < 0.9 * area[rect_ok].sum()


def _rect_min(a, b, c, x0, x1, y0, y1):
    """min of a x^2 + 2 b x y + c y^2 (positive definite) over [x0, x1] x [y0, y1]."""
    if x0 <= 0 <= x1 and y0 <= 0 <= y1:
        return 0.0
    q = lambda x, y: a * x * x + 2 * b * x * y + c * y * y
    best = math.inf
    for x in (x0, x1):  # vertical edges: minimiser y = -b x / c, clamped
        best = min(best, q(x, min(max(-b * x / c, y0), y1)))
    for y in (y0, y1):  # horizontal edges: x = -b y / a, clamped
        best = min(best, q(min(max(-b * y / a, x0), x1), y))
    return best


def test_tile_lists_match_the_rectangle_minimum():
    """Independent formulation: a tile of the rectangle is listed exactly when
    the minimum of d^T Q d over its block of pixel centres (widened by 0.01
    pixel) is at most k = 2.02 (-tau) + 1e-3 (ellipse splats; cases within
    the float32 rounding of the listing, 2e-3 relative, are not judged), the
    whole rectangle when the conic is nearly degenerate, nothing when
    tau > 0."""
    x, cam = _varied_splats(13)
    pr = B.project_f32(x, cam)
    b = B.bin_view(x, cam)
    tiles = (b.keys >> np.uint64(32)).astype(np.int64)
    listed = {(int(g), int(t)) for g, t in zip(b.gids, tiles)}
    ca, cb, cc = (np.asarray(t, np.float32) for t in pr["conic"])
    judged = dropped = 0
    kinds = set()
    for g in range(x.shape[1]):
        x0, y0, x1, y1 = (int(v) for v in pr["rect"][g])
        if not (x1 > x0 and y1 > y0):
            continue
        a, bb, c = float(ca[g]), float(cb[g]), float(cc[g])
        tau = float(pr["tau"][g])
        det = a * c - bb * bb
        if tau > 0:
            kinds.add("none")
            assert not any((g, ty * b.tiles_x + tx) in listed for ty in range(y0, y1) for tx in range(x0, x1))
            continue
        if not (a > 0 and c > 0 and det * 1000 >= a * c):
            kinds.add("whole")
            assert all((g, ty * b.tiles_x + tx) in listed for ty in range(y0, y1) for tx in range(x0, x1))
            continue
        kinds.add("ellipse")
        k = -2.02 * tau + 1e-3
        u, v = float(pr["u"][g]), float(pr["v"][g])
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                m = _rect_min(a, bb, c, 16 * tx + 0.49 - u, 16 * tx + 15.51 - u, 16 * ty + 0.49 - v,
                              16 * ty + 15.51 - v)
                if abs(m - k) <= 2e-3 * k:
                    continue
                assert ((g, ty * b.tiles_x + tx) in listed) == (m <= k), (g, tx, ty, m, k)
                judged += 1
                dropped += m > k
    assert judged > 2000 and dropped > 200
    assert {"none", "ellipse"} <= kinds
