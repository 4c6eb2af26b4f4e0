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
        if pr["visible"][g]:
            assert list(range(x0, x1)) == xs and list(range(y0, y1)) == ys
            n_checked += 1
        else:
            assert len(xs) == 0 or len(ys) == 0
    assert n_checked > 1000


def test_keys_order_and_ranges_invariants():
    sc = syn.config1_scene()
    cam = sc.cameras[3]
    b = B.bin_view(sc.gt, cam)
    tiles = (b.keys >> np.uint64(32)).astype(np.int64)
    assert np.all(np.diff(b.keys.astype(np.float64)) >= 0) or np.all(b.keys[1:] >= b.keys[:-1])
    assert len(b.keys) == int(b.tiles_touched.sum())
    # each visible Gaussian occurs exactly once in each tile of its rectangle
    for g in np.flatnonzero(b.visible)[:300]:
        x0, y0, x1, y1 = b.rect[g]
        want = sorted(ty * b.tiles_x + tx for ty in range(y0, y1) for tx in range(x0, x1))
        got = sorted(tiles[b.gids == g].tolist())
        assert got == want
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
