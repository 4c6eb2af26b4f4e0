"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bit-exact: tile keys, sorted Gaussian order, per-tile ranges.  Floating
point: relative L2 <= 1e-4 per parameter group (images, gradients, Hessian
diagonals, trust-region steps).  Inputs are seeded; targets for the loss are
the oracle's render plus +-U[0.05, 0.15] so every residual is far from the L1
kink and the Gauss-Newton weights are well conditioned.
"""
import math
import sys

import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import binning as B
from oracle import method as Mth
from oracle import render as R
from tests.helpers import group_errors, group_max_abs, offset_targets, rel_l2, view_flips

pytestmark = pytest.mark.gpu
TOL = 1e-4
# largest elementwise error of a group, relative to its largest entry
MAX_ABS = 1e-3
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(got, want, p, flips=None):
    """rel-L2 <= TOL per parameter group and the largest elementwise error
    <= MAX_ABS of the group's largest entry; prints both, and the
    float32-vs-float64 decision flips of the views involved when given."""
    errs = group_errors(got, want, p)
    mx = group_max_abs(got, want, p)
    say("  rel-L2 per group", errs)
    say("  max-abs per group", mx, "flips", flips)
    assert all(e <= TOL for e in errs.values()), errs
    assert all(e <= MAX_ABS for e in mx.values()), mx


def make_scene(x, targets, cams, deg, lam=0.2, bg=(0.0, 0.0, 0.0)):
    from paper_2602_00395_amd import Scene

    xt = torch.tensor(np.asarray(x, np.float32), device=DEV)
    tg = [torch.tensor(np.asarray(t, np.float32), device=DEV) for t in targets]
    return Scene(xt, tg, cams, deg, lam=lam, background=bg)


@pytest.fixture(scope="module")
def c1():
    sc = syn.config1_scene()
    x = sc.init.astype(np.float32)
    targets = offset_targets(x, sc.cameras, 0, seed=4001)
    return sc, x, targets


def _check_bins(gpu, ob, tag):
    keys, gids, ranges = gpu
    k = keys.cpu().numpy().view(np.uint64)
    assert len(k) == len(ob.keys), (tag, len(k), len(ob.keys))
    assert np.array_equal(k, ob.keys), tag
    assert np.array_equal(gids.cpu().numpy().astype(np.int64), ob.gids), tag
    # an empty tile's range is any [s, s); non-empty ranges are unique
    r = ranges.cpu().numpy().astype(np.int64)
    empty = ob.ranges[:, 0] == ob.ranges[:, 1]
    assert np.array_equal(r[~empty], ob.ranges[~empty]), tag
    assert np.all(r[empty, 0] == r[empty, 1]), tag


def test_binning_bit_exact_config1(c1):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    for j, cam in enumerate(sc.cameras):
        say("bin c1 camera", j)
        _check_bins(s.bin(j), B.bin_view(x, cam), f"cam{j}")
    s.close()


def test_binning_bit_exact_ragged_and_large_splats():
    sc = syn.config1_scene()
    x = sc.gt.copy()
    x[3:6] += 1.5  # splats spanning many tiles
    cams = [syn.make_camera((0.3, -3.0, 0.4), 80, 56), syn.make_camera((2.5, 2.0, 1.0), 37, 71)]
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in cams]
    s = make_scene(x, targets, cams, 0)
    for j, cam in enumerate(cams):
        say("bin ragged camera", j)
        ob = B.bin_view(x, cam)
        assert ob.tiles_touched.max() > 8
        _check_bins(s.bin(j), ob, f"ragged{j}")
    s.close()


def test_binning_bit_exact_object_scale():
    sc = syn.config2_scene()
    cams = sc.cameras[:3]
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in cams]
    for name, x in (("gt", sc.gt), ("init", sc.init)):
        s = make_scene(x, targets, cams, 3)
        for j, cam in enumerate(cams):
            say("bin object-scale", name, "camera", j)
            ob = B.bin_view(x, cam)
            _check_bins(s.bin(j), ob, f"{name}{j}")
        s.close()


def test_render_parity_config1(c1):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    xt = torch.tensor(x, dtype=torch.float64)
    for j, cam in enumerate(sc.cameras):
        say("render c1 camera", j)
        want = R.render(xt, cam, 0).numpy()
        got = s.render(j).cpu().numpy()
        assert rel_l2(got, want) <= TOL, (j, rel_l2(got, want))
    s.close()


def test_render_parity_background_and_empty_view():
    sc = syn.config1_scene()
    x = sc.gt.astype(np.float32)
    cams = [sc.cameras[0], syn.make_camera((0.0, 0.0, 30.0), 48, 40, target=(0.0, 0.0, 60.0))]
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in cams]
    bg = (0.2, 0.5, 0.9)
    s = make_scene(x, targets, cams, 0, bg=bg)
    got = s.render(0).cpu().numpy()
    want = R.render(torch.tensor(x, dtype=torch.float64), cams[0], 0, background=bg).numpy()
    assert rel_l2(got, want) <= TOL
    empty = s.render(1).cpu().numpy()  # looking away from every Gaussian
    assert np.allclose(empty, np.broadcast_to(np.array(bg, np.float32), empty.shape))
    g = s.grad([1]).cpu().numpy()
    assert np.all(g == 0)
    s.close()


def test_render_parity_object_scale_sampled_tiles():
    sc = syn.config2_scene()
    cam = sc.cameras[5]
    x = sc.init.astype(np.float32)
    s = make_scene(x, [np.zeros((cam.height, cam.width, 3), np.float32)], [cam], 3)
    got = s.render(0).cpu().numpy()
    ob = B.bin_view(x, cam)
    counts = ob.ranges[:, 1] - ob.ranges[:, 0]
    rng = np.random.default_rng(7)
    busy = np.argsort(counts)[-3:]
    pick = set(int(t) for t in busy) | set(int(t) for t in rng.choice(len(counts), 5, replace=False))
    say("render object-scale tiles", sorted(pick), "longest list", int(counts.max()))
    want = R.render(torch.tensor(x, dtype=torch.float64), cam, 3, ob, tiles=pick).numpy()
    m = ~np.isnan(want[..., 0])
    assert m.sum() >= 6 * 256
    assert rel_l2(got[m], want[m]) <= TOL
    s.close()


def test_render_ignores_stale_lds_contents():
    """Kernels that leave infinities and NaNs in LDS (block reductions over
    such a tensor) run right before each render and gradient: the blend
    kernels' idle walk slots must never read a stale slot, so the image and
    the gradient stay finite and equal to the ones rendered after clean
    kernels, bit for bit."""
    sc = syn.config2_scene()
    cams = sc.cameras[:2]
    x = sc.init.astype(np.float32)
    targets = [np.full((c.height, c.width, 3), 0.5, np.float32) for c in cams]
    s = make_scene(x, targets, cams, 3)
    ref_img = s.render(0).clone()
    ref_g = s.grad([1]).clone()
    junk = torch.full((1 << 22,), float("inf"), device=DEV)
    junk[::7] = float("nan")
    junk[::11] = -float("inf")
    for rep in range(3):
        say("stale LDS: repeat", rep)
        for _ in range(4):
            junk.sum()
            junk.cumsum(0)
        img = s.render(0)
        for _ in range(4):
            junk.sum()
            junk.cumsum(0)
        g = s.grad([1])
        torch.cuda.synchronize()
        assert torch.isfinite(img).all() and torch.isfinite(g).all()
        assert torch.equal(img, ref_img) and torch.equal(g, ref_g)
    s.close()


@pytest.mark.parametrize("lam", [0.2, 0.0])
def test_grad_parity_config1(c1, lam):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0, lam=lam)
    prob = Mth.Problem(sc.cameras, targets, 0, lam=lam)
    for S1 in ([1], [0, 5]):
        say("grad c1 lam", lam, "S1", S1)
        want, f_want = Mth.gradient(x, prob, S1)
        got, f_got = s.grad(S1, want_loss=True)
        check(got.cpu().numpy(), want, 14, flips=view_flips(x, sc.cameras, S1, 0))
        assert abs(f_got - f_want) <= 1e-5 * abs(f_want)
    s.close()


def test_grad_is_deterministic(c1):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    a = s.grad([2]).cpu()
    b = s.grad([2]).cpu()
    assert torch.equal(a, b)
    s.close()


def test_counting_kernels_match_plain_kernels(c1):
    """The instrumented blend instances (profiling with work counters) give
    the same gradient and Hutchinson diagonal bit for bit, and count work."""
    from paper_2602_00395_amd import profile_count, profile_enable, profile_read, profile_reset

    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    plain_g = s.grad([2]).cpu()
    plain_d = s.hvp_diag([3], 1, 5003).cpu()
    profile_reset()
    profile_count(True)
    profile_enable("blend_fwd,blend_bwd,blend_jvp")
    try:
        counted_g = s.grad([2]).cpu()
        counted_d = s.hvp_diag([3], 1, 5003).cpu()
        torch.cuda.synchronize()
    finally:
        profile_enable("")
    st = {k: profile_read(k) for k in ("blend_fwd", "blend_bwd", "blend_jvp")}
    profile_reset()
    say("  counters", st)
    assert torch.equal(plain_g, counted_g) and torch.equal(plain_d, counted_d)
    for k, v in st.items():
        assert v["launches"] >= 1 and v["work0"] >= v["work1"] > 0, (k, v)
    s.close()


def test_hvp_diag_parity_config1(c1):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    prob = Mth.Problem(sc.cameras, targets, 0, lam=0.2)
    S2, nu, seed = [2], 2, 5001
    say("hvp_diag c1 S2", S2, "nu", nu)
    want = Mth.hutchinson(x, prob, S2, nu, seed)
    got = s.hvp_diag(S2, nu, seed).cpu().numpy()
    check(got, want, 14, flips=view_flips(x, sc.cameras, S2, 0))
    s.close()


def test_render_vjp_and_jvp_parity(c1):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    cam = sc.cameras[4]
    rng = np.random.default_rng(11)
    cot = rng.normal(size=(cam.height, cam.width, 3))
    tan = rng.normal(size=x.shape)
    xt = torch.tensor(x, dtype=torch.float64)
    bins = B.bin_view(x, cam)
    f = lambda xx: R.render(xx, cam, 0, bins)  # noqa: E731
    img, vjp_fn = torch.func.vjp(f, xt)
    want_g = vjp_fn(torch.tensor(cot))[0].numpy()
    got_g = s.render_vjp(4, torch.tensor(cot, dtype=torch.float32, device=DEV)).cpu().numpy()
    errs = group_errors(got_g, want_g, 14)
    say("vjp rel-L2", errs)
    assert all(e <= TOL for e in errs.values()), errs
    _, want_t = torch.func.jvp(f, (xt,), (torch.tensor(tan),))
    rgb, got_t = s.render_jvp(4, torch.tensor(tan, dtype=torch.float32, device=DEV))
    assert rel_l2(rgb.cpu().numpy(), img.detach().numpy()) <= TOL
    assert rel_l2(got_t.cpu().numpy(), want_t.numpy()) <= TOL, rel_l2(got_t.cpu().numpy(), want_t.numpy())
    s.close()


def test_grad_parity_object_scale_crop():
    """The 500 Gaussians nearest the origin of the object-scale scene, SH degree 3,
    rendered at 800x800 from two cameras."""
    sc = syn.config2_scene()
    d = np.linalg.norm(sc.init[0:3].T, axis=1)
    keep = np.argsort(d)[:500]
    x = sc.init[:, keep].copy()
    x[11 + 3:] = sc.gt[11 + 3:, keep]  # non-zero higher-order SH so every row is exercised
    cams = [sc.cameras[0], sc.cameras[17]]
    targets = offset_targets(x, cams, 3, seed=4002)
    s = make_scene(x, targets, cams, 3)
    prob = Mth.Problem(cams, targets, 3, lam=0.2)
    say("grad crop")
    want, _ = Mth.gradient(x, prob, [1])
    got = s.grad([1]).cpu().numpy()
    check(got, want, 59)
    s.close()


def _sampled_gaussians(ob, rng, k, max_tiles):
    """k visible Gaussians whose rectangles hold 1..max_tiles tiles, and the set of those tiles."""
    area = (ob.rect[:, 2] - ob.rect[:, 0]) * (ob.rect[:, 3] - ob.rect[:, 1])
    cand = np.flatnonzero((ob.tiles_touched >= 1) & (area <= max_tiles))
    pick = np.sort(rng.choice(cand, size=k, replace=False))
    tiles = set()
    for g in pick:
        x0, y0, x1, y1 = (int(v) for v in ob.rect[g])
        tiles |= {ty * ob.tiles_x + tx for ty in range(y0, y1) for tx in range(x0, x1)}
    return pick, tiles


def test_render_vjp_object_scale_sampled_gaussians():
    """Full object scale (100k Gaussians, SH 3, 800x800): J^T cot for sampled
    Gaussians; a Gaussian's gradient only involves the pixels of its own
    tiles, so the oracle renders just those tiles (with every splat in them)."""
    sc = syn.config2_scene()
    cam = sc.cameras[3]
    x = sc.init.astype(np.float32)
    x[14:] = sc.gt[14:]  # non-zero higher-order SH so every row is exercised
    s = make_scene(x, [np.zeros((cam.height, cam.width, 3), np.float32)], [cam], 3)
    ob = B.bin_view(x, cam)
    rng = np.random.default_rng(41)
    pick, tiles = _sampled_gaussians(ob, rng, 5, 3)
    say("vjp object scale: Gaussians", pick.tolist(), "tiles", len(tiles))
    cot = rng.normal(size=(cam.height, cam.width, 3))
    got = s.render_vjp(0, torch.tensor(cot, dtype=torch.float32, device=DEV)).cpu().numpy()[:, pick]
    xg = torch.tensor(x, dtype=torch.float64).requires_grad_(True)
    img = R.render(xg, cam, 3, ob, tiles=tiles)
    m = ~torch.isnan(img)
    (img[m] * torch.tensor(cot)[m]).sum().backward()
    want = xg.grad.numpy()[:, pick]
    check(got, want, 59)
    s.close()


def test_hvp_diag_object_scale_sampled_gaussians():
    """Full object scale: the Hutchinson diagonal (L1 loss, one probe) for
    sampled Gaussians.  J z, the Gauss-Newton weights and J^T y of those
    Gaussians only involve their own tiles; the targets there are the
    oracle's render offset by +-U[0.05, 0.15] (every residual away from 0)."""
    sc = syn.config2_scene()
    cam = sc.cameras[11]
    x = sc.init.astype(np.float32)
    ob = B.bin_view(x, cam)
    rng = np.random.default_rng(42)
    pick, tiles = _sampled_gaussians(ob, rng, 4, 2)
    say("hvp object scale: Gaussians", pick.tolist(), "tiles", len(tiles))
    xt = torch.tensor(x, dtype=torch.float64)
    f = lambda xx: R.render(xx, cam, 3, ob, tiles=tiles)  # noqa: E731
    with torch.no_grad():
        base = f(xt)
    m = ~torch.isnan(base)
    off = rng.uniform(0.05, 0.15, size=base.shape) * rng.choice([-1.0, 1.0], size=base.shape)
    tgt = np.full(base.shape, 0.5)
    tgt[m.numpy()] = base.numpy()[m.numpy()] + off[m.numpy()]
    s = make_scene(x, [tgt.astype(np.float32)], [cam], 3, lam=0.0)
    seed = 5077
    got = s.hvp_diag([0], 1, seed).cpu().numpy()[:, pick]
    p, n = x.shape
    z = Mth.probe(seed, 0, p, n)
    img, u = torch.func.jvp(f, (xt,), (torch.tensor(z),))
    tg = torch.tensor(tgt)
    y = torch.zeros_like(img)
    y[m] = Mth.gn_cotangent(img[m], tg[m], u[m], 0.0)
    xg = xt.clone().requires_grad_(True)
    out = f(xg)
    (out[m] * y[m]).sum().backward()
    scale = 1.0 / (6.0 * cam.height * cam.width)  # M / (m |S2| nu) with one training view
    want = (z * xg.grad.numpy() * scale)[:, pick]
    check(got, want, 59)
    s.close()


def _long_tile_picks(ob, rng, n_tiles, per_seg, seg=256):
    """Gaussians from every depth segment of the `n_tiles` longest tile lists
    (segments of `seg` pairs), each touching at most 4 tiles, and the tiles
    they touch."""
    counts = ob.ranges[:, 1] - ob.ranges[:, 0]
    longest = np.argsort(counts)[-n_tiles:]
    assert counts[longest].min() > 2 * seg, counts[longest]
    pick = set()
    for t in longest:
        lo, hi = (int(v) for v in ob.ranges[t])
        for q in range(lo, hi, seg):
            g = ob.gids[q:min(q + seg, hi)]
            area = (ob.rect[g, 2] - ob.rect[g, 0]) * (ob.rect[g, 3] - ob.rect[g, 1])
            g = g[area <= 4]
            pick |= set(int(v) for v in rng.choice(g, size=min(per_seg, len(g)), replace=False))
    pick = np.array(sorted(pick))
    tiles = set()
    for g in pick:
        x0, y0, x1, y1 = (int(v) for v in ob.rect[g])
        tiles |= {ty * ob.tiles_x + tx for ty in range(y0, y1) for tx in range(x0, x1)}
    return pick, tiles, longest


def test_vjp_and_hvp_long_tiles_every_depth_segment():
    """Full object scale: Gaussians from every 256-pair depth segment of the
    two longest tile lists.  Each segment's backward starts from the
    transmittance and colour the forward (or, for the Hutchinson diagonal,
    the JVP) stored at the segment boundaries, so a wrong state shows up in
    the gradients of the earlier segments' Gaussians."""
    sc = syn.config2_scene()
    cam = sc.cameras[3]
    x = sc.init.astype(np.float32)
    x[14:] = sc.gt[14:]
    ob = B.bin_view(x, cam)
    rng = np.random.default_rng(43)
    pick, tiles, longest = _long_tile_picks(ob, rng, 2, 1)
    say("long tiles", longest.tolist(), "lists", (ob.ranges[longest, 1] - ob.ranges[longest, 0]).tolist(),
        "Gaussians", len(pick), "tiles", len(tiles))
    xt = torch.tensor(x, dtype=torch.float64)
    f = lambda xx: R.render(xx, cam, 3, ob, tiles=tiles)  # noqa: E731
    with torch.no_grad():
        base = f(xt)
    m = ~torch.isnan(base)
    # render VJP with a random cotangent
    cot = rng.normal(size=(cam.height, cam.width, 3))
    s = make_scene(x, [np.zeros((cam.height, cam.width, 3), np.float32)], [cam], 3)
    got = s.render_vjp(0, torch.tensor(cot, dtype=torch.float32, device=DEV)).cpu().numpy()[:, pick]
    s.close()
    xg = xt.clone().requires_grad_(True)
    (f(xg)[m] * torch.tensor(cot)[m]).sum().backward()
    want = xg.grad.numpy()[:, pick]
    # Gaussians behind every pixel's last contribution have zero gradient
    assert np.count_nonzero(np.abs(want).sum(axis=0)) >= 4
    say("  vjp")
    check(got, want, 59)
    # Hutchinson diagonal (L1 loss, one probe) through the JVP's states
    off = rng.uniform(0.05, 0.15, size=base.shape) * rng.choice([-1.0, 1.0], size=base.shape)
    tgt = np.full(base.shape, 0.5)
    tgt[m.numpy()] = base.numpy()[m.numpy()] + off[m.numpy()]
    s = make_scene(x, [tgt.astype(np.float32)], [cam], 3, lam=0.0)
    seed = 5081
    got = s.hvp_diag([0], 1, seed).cpu().numpy()[:, pick]
    s.close()
    p, n = x.shape
    z = Mth.probe(seed, 0, p, n)
    img, u = torch.func.jvp(f, (xt,), (torch.tensor(z),))
    y = torch.zeros_like(img)
    y[m] = Mth.gn_cotangent(img[m], torch.tensor(tgt)[m], u[m], 0.0)
    xg = xt.clone().requires_grad_(True)
    (f(xg)[m] * y[m]).sum().backward()
    scale = 1.0 / (6.0 * cam.height * cam.width)
    want = (z * xg.grad.numpy() * scale)[:, pick]
    say("  hvp")
    check(got, want, 59)


def _stacked_tile_scene(L, seed):
    """Exactly L small, faint Gaussians whose footprints lie inside tile 0 of a
    32x32 view (so that tile's list holds L pairs and the other tiles none);
    opacities ~0.1 keep every pixel blending through the whole list, a few
    opaque ones stop some pixels early."""
    from synthetic import scenes as S

    cam = syn.make_camera((0.0, -3.0, 0.3), 32, 32)
    rng = np.random.default_rng(seed)
    parts, have = [], 0
    while have < L:
        x = S.random_scene(rng, 8 * L, 0, -0.9, 0.9, math.log(0.01), 0.2, 0.1)
        # the final faint opacities before binning: a splat's tile list
        # depends on its opacity
        x[10] = np.log(0.1 / 0.9) + rng.normal(0.0, 0.3, size=x.shape[1])
        ob = B.bin_view(x, cam)
        ok = np.flatnonzero((ob.tiles_touched == 1) & np.all(ob.rect == [0, 0, 1, 1], axis=1))
        parts.append(x[:, ok])
        have += len(ok)
    x = np.concatenate(parts, axis=1)[:, :L].copy()
    # a few opaque ones: a larger skip ellipse, the same rectangle (tile 0)
    x[10, rng.choice(L, size=max(1, L // 64), replace=False)] = 3.0
    return x.astype(np.float32), cam


@pytest.mark.parametrize("L", [256, 257, 512, 513])
def test_grad_and_hvp_segment_boundaries(L):
    """A tile list of exactly 256, 257, 512 or 513 pairs: one full depth
    segment, a full one plus one pair, two full ones, two plus one.  The
    whole view's gradient and Hutchinson diagonal against the oracle."""
    x, cam = _stacked_tile_scene(L, 9100 + L)
    ob = B.bin_view(x, cam)
    assert int(ob.ranges[0, 1] - ob.ranges[0, 0]) == L
    targets = offset_targets(x, [cam], 0, seed=9200 + L)
    s = make_scene(x, targets, [cam], 0)
    prob = Mth.Problem([cam], targets, 0, lam=0.2)
    say("segment boundaries: list of", L, "pairs")
    want, _ = Mth.gradient(x, prob, [0])
    got = s.grad([0]).cpu().numpy()
    say("  grad")
    check(got, want, 14)
    want = Mth.hutchinson(x, prob, [0], 1, 5301)
    got = s.hvp_diag([0], 1, 5301).cpu().numpy()
    say("  hvp")
    check(got, want, 14)
    s.close()


def test_tr_step_parity():
    sc = syn.config2_scene(n=4000, n_cams=2, res=64)
    x = sc.gt.astype(np.float32)
    p, n = x.shape
    rng = np.random.default_rng(12)
    g = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
    ghat = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
    dhat = rng.uniform(-0.2, 1.0, size=x.shape).astype(np.float32)
    dhat[:, :50] = 0.0  # the D <= 0 rule
    D = rng.uniform(0.0, 2.0, size=x.shape).astype(np.float32)
    x[10, :100] = -16.0  # eps >= alpha: unconstrained mean and rotation
    x[3:6, 100:150] = math.log(0.07)  # isotropic: free rotation
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in sc.cameras]
    for hutch in (True, False):
        say("tr_step hutch", hutch)
        s = make_scene(x, targets, sc.cameras, 3)
        gh_t = torch.tensor(ghat, device=DEV)
        dh_t = torch.tensor(dhat, device=DEV)
        s.import_(ghat=gh_t, dhat=dh_t)
        eta_t = torch.empty_like(gh_t)
        dx_t = torch.empty_like(gh_t)
        eps = 3e-7
        s.tr_step(torch.tensor(g, device=DEV), torch.tensor(D, device=DEV) if hutch else None, 0.9, 0.999, eps,
                  eta_out=eta_t, dx_out=dx_t)
        x_new = s.params().cpu().numpy()
        eta_want = Mth.shd_eta(x.astype(np.float64), eps, 3)
        xw, ghw, dhw, dxw, _ = Mth.tr_step(x, g, ghat, dhat, D if hutch else None, 0.9, 0.999, eps, 3,
                                           eta=eta_want)
        eta_got = eta_t.cpu().numpy()
        assert np.array_equal(np.isinf(eta_got), np.isinf(eta_want))
        fin = np.isfinite(eta_want)
        assert rel_l2(eta_got[fin], eta_want[fin]) <= TOL
        errs = group_errors(dx_t.cpu().numpy(), dxw, p)
        say("  step rel-L2", errs)
        assert all(e <= TOL for e in errs.values()), errs
        # x' = x + step: its error is the step's error plus float32 rounding of x
        assert np.linalg.norm(x_new - xw) <= TOL * np.linalg.norm(dxw) + 1e-6 * np.linalg.norm(x)
        ghn, dhn = torch.empty_like(gh_t), torch.empty_like(gh_t)
        s.export(ghat=ghn, dhat=dhn)
        assert rel_l2(ghn.cpu().numpy(), ghw) <= 1e-6 and rel_l2(dhn.cpu().numpy(), dhw) <= 1e-6
        s.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 7])
def test_tr_step_radius_variants(variant):
    # GS3_TR_MEAN_EXACT (1), GS3_TR_SECOND_ORDER (2), GS3_TR_SH_JOINT (4) and
    # combinations, against the oracle's mean_bound="exact",
    # constants="second_order" and sh_rest="joint"
    sc = syn.config2_scene(n=3000, n_cams=2, res=64)
    x = sc.gt.astype(np.float32)
    p, n = x.shape
    rng = np.random.default_rng(31)
    g = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
    ghat = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
    dhat = rng.uniform(-0.2, 1.0, size=x.shape).astype(np.float32)
    x[10, :60] = -16.0
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in sc.cameras]
    say("tr_step variant", variant)
    s = make_scene(x, targets, sc.cameras, 3)
    s.import_(ghat=torch.tensor(ghat, device=DEV), dhat=torch.tensor(dhat, device=DEV))
    eta_t = torch.empty((p, n), device=DEV)
    dx_t = torch.empty((p, n), device=DEV)
    eps = 3e-7
    s.tr_step(torch.tensor(g, device=DEV), None, 0.9, 0.999, eps, eta_out=eta_t, dx_out=dx_t, variant=variant)
    mb = "exact" if variant & 1 else "printed"
    ko = "second_order" if variant & 2 else "printed"
    sr = "joint" if variant & 4 else "base"
    eta_want = Mth.shd_eta(x.astype(np.float64), eps, 3, mean_bound=mb, constants=ko, sh_rest=sr)
    _, _, _, dxw, _ = Mth.tr_step(x, g, ghat, dhat, None, 0.9, 0.999, eps, 3, eta=eta_want)
    eta_got = eta_t.cpu().numpy()
    assert np.array_equal(np.isinf(eta_got), np.isinf(eta_want))
    fin = np.isfinite(eta_want)
    assert rel_l2(eta_got[fin], eta_want[fin]) <= TOL
    errs = group_errors(dx_t.cpu().numpy(), dxw, p)
    say("  step rel-L2", errs)
    assert all(e <= TOL for e in errs.values()), errs
    s.close()


def test_adam_and_adam_tr_parity():
    sc = syn.config2_scene(n=3000, n_cams=2, res=64)
    x = sc.init.astype(np.float32)
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in sc.cameras]
    rng = np.random.default_rng(13)
    lrs = Mth.adam_lrs(10, 100, 2.0)
    for eps in (None, 1e-6):
        s = make_scene(x, targets, sc.cameras, 3)
        xo, m, v = x.astype(np.float64), np.zeros(x.shape), np.zeros(x.shape)
        for step in range(1, 4):
            g = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
            s.adam_step(torch.tensor(g, device=DEV), lrs, step, epsilon=eps)
            if eps is None:
                xo, m, v = Mth.adam_step(xo, g, m, v, step, lrs, 3)
            else:
                eta = Mth.shd_eta(xo, eps, 3)
                xn, m, v = Mth.adam_step(xo, g, m, v, step, lrs, 3)
                xo = xo + np.clip(xn - xo, -eta, eta)
        got = s.params().cpu().numpy()
        errs = group_errors(got - x, xo - x, 59)
        say("adam eps", eps, errs)
        assert all(e <= TOL for e in errs.values()), errs
        s.close()


def test_psnr_matches_oracle(c1):
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    want = R.render(torch.tensor(x, dtype=torch.float64), sc.cameras[3], 0)
    from oracle.loss import psnr

    assert abs(s.psnr(3) - psnr(want, torch.tensor(targets[3], dtype=torch.float64))) < 1e-3
    s.close()


def test_fused_iteration_matches_separate_calls(c1):
    """gs3_tr_iteration (Hutchinson + gradient + update fused into the last
    view's projection backward) against gs3_hvp_diag + gs3_grad + gs3_tr_step,
    bit for bit, over three iterations (with and without a Hutchinson step, one
    and two gradient views).  Each of those calls is checked against the
    oracle by its own test, so the fused iteration inherits their parity."""
    sc, x, targets = c1
    a = make_scene(x, targets, sc.cameras, 0)
    b = make_scene(x, targets, sc.cameras, 0)
    g = a._empty_like_params()
    D = a._empty_like_params()
    plan = [([1], [3], 2, 1e-6), ([1, 4], [], 1, 8e-7), ([2], [], 1, 6e-7)]
    for it, (S1, S2, nu, eps) in enumerate(plan):
        say("fused iteration", it, "S1", S1, "S2", S2)
        seed = 7000 + it
        if S2:
            a.hvp_diag(S2, nu, seed, out=D)
        a.grad(S1, out=g)
        a.tr_step(g, D if S2 else None, 0.9, 0.999, eps, variant=4)
        b.tr_iteration(S1, S2, nu, seed, 0.9, 0.999, eps, variant=4)
        for name in ("x", "ghat", "dhat"):
            ta, tb = a._empty_like_params(), b._empty_like_params()
            a.export(**{name: ta})
            b.export(**{name: tb})
            assert torch.equal(ta, tb), (it, name, float((ta - tb).abs().max()))
    a.close()
    b.close()


@pytest.mark.parametrize("deg", [1, 2])
def test_grad_and_hvp_parity_sh_degrees(deg):
    """SH degrees 1 and 2 (the kernels are instantiated per degree; the other
    tests cover 0 and 3): gradient and Hutchinson diagonal against the oracle."""
    sc = syn.tiny_scene(300 + deg, n=60, sh_degree=deg, width=48, height=40, n_cams=3,
                        log_scale_mean=np.log(0.08))
    x = sc.gt.astype(np.float32)
    x[0:3] += np.random.default_rng(deg).normal(0, 0.02, size=x[0:3].shape).astype(np.float32)
    targets = offset_targets(x, sc.cameras, deg, seed=4100 + deg)
    s = make_scene(x, targets, sc.cameras, deg)
    prob = Mth.Problem(sc.cameras, targets, deg, lam=0.2)
    p = x.shape[0]
    say("grad sh degree", deg)
    want, _ = Mth.gradient(x, prob, [1])
    check(s.grad([1]).cpu().numpy(), want, p, flips=view_flips(x, sc.cameras, [1], deg))
    say("hvp sh degree", deg)
    want = Mth.hutchinson(x, prob, [2], 1, 5200 + deg)
    check(s.hvp_diag([2], 1, 5200 + deg).cpu().numpy(), want, p, flips=view_flips(x, sc.cameras, [2], deg))
    s.close()


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_tr_step_parity_sh_degrees(deg):
    """The update kernel for P = 14, 23, 38 rows (the object-scale test covers 59)."""
    sc = syn.config2_scene(n=2000, n_cams=1, res=32)
    p = Mth.n_params(deg)
    x = np.concatenate([sc.gt[:11], sc.gt[11:11 + p - 11]]).astype(np.float32)
    rng = np.random.default_rng(50 + deg)
    g = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
    ghat = (rng.normal(size=x.shape) * 1e-3).astype(np.float32)
    dhat = rng.uniform(-0.2, 1.0, size=x.shape).astype(np.float32)
    D = rng.uniform(0.0, 2.0, size=x.shape).astype(np.float32)
    targets = [np.zeros((c.height, c.width, 3), np.float32) for c in sc.cameras]
    s = make_scene(x, targets, sc.cameras, deg)
    s.import_(ghat=torch.tensor(ghat, device=DEV), dhat=torch.tensor(dhat, device=DEV))
    eta_t = torch.empty(x.shape, device=DEV)
    dx_t = torch.empty(x.shape, device=DEV)
    eps = 2e-7
    say("tr_step sh degree", deg)
    s.tr_step(torch.tensor(g, device=DEV), torch.tensor(D, device=DEV), 0.9, 0.999, eps, eta_out=eta_t, dx_out=dx_t,
              variant=4)
    eta_want = Mth.shd_eta(x.astype(np.float64), eps, deg, sh_rest="joint")
    _, _, _, dxw, _ = Mth.tr_step(x, g, ghat, dhat, D, 0.9, 0.999, eps, deg, eta=eta_want)
    eta_got = eta_t.cpu().numpy()
    assert np.array_equal(np.isinf(eta_got), np.isinf(eta_want))
    fin = np.isfinite(eta_want)
    assert rel_l2(eta_got[fin], eta_want[fin]) <= TOL
    errs = group_errors(dx_t.cpu().numpy(), dxw, p)
    say("  step rel-L2", errs)
    assert all(e <= TOL for e in errs.values()), errs
    s.close()


def test_single_gaussian_render_and_grad():
    """N = 1: one splat, one tile list of length one per tile it touches."""
    sc = syn.tiny_scene(77, n=1, sh_degree=0, width=40, height=36, n_cams=2, log_scale_mean=np.log(0.3))
    x = sc.gt.astype(np.float32)
    targets = offset_targets(x, sc.cameras, 0, seed=4300)
    s = make_scene(x, targets, sc.cameras, 0)
    want_img = R.render(torch.tensor(x, dtype=torch.float64), sc.cameras[0], 0).numpy()
    assert rel_l2(s.render(0).cpu().numpy(), want_img) <= TOL
    prob = Mth.Problem(sc.cameras, targets, 0, lam=0.2)
    want, _ = Mth.gradient(x, prob, [0])
    say("single Gaussian grad")
    check(s.grad([0]).cpu().numpy(), want, 14)
    s.close()


def test_grad_and_hvp_splats_over_many_tiles():
    """Pair sums of splats covering more than 48 tiles (summed by the whole
    workgroup) next to splats covering fewer (nine threads per Gaussian), up
    to more than 2,048 tiles (several slots per thread of the workgroup): a
    few large Gaussians at 200x184 and 800x720."""
    sc = syn.tiny_scene(91, n=12, sh_degree=1, width=200, height=184, n_cams=2, log_scale_mean=np.log(0.35),
                        log_scale_std=0.7)
    x = sc.gt.astype(np.float32)
    cams = [sc.cameras[0], syn.make_camera(tuple(syn.fibonacci_sphere(2, 3.0)[1]), 800, 720)]
    counts = [B.bin_view(x, c).tiles_touched for c in cams]
    say("tiles touched", [sorted(c.tolist()) for c in counts])
    assert counts[0].min() <= 48 < counts[0].max()
    assert counts[1].max() > 2048
    targets = offset_targets(x, cams, 1, seed=4400)
    s = make_scene(x, targets, cams, 1)
    prob = Mth.Problem(cams, targets, 1, lam=0.2)
    for j in range(2):
        say("many-tile grad view", j)
        want, _ = Mth.gradient(x, prob, [j])
        check(s.grad([j]).cpu().numpy(), want, 23, flips=view_flips(x, cams, [j], 1))
    say("many-tile hvp")
    want = Mth.hutchinson(x, prob, [0, 1], 1, 4401)
    check(s.hvp_diag([0, 1], 1, 4401).cpu().numpy(), want, 23, flips=view_flips(x, cams, [0, 1], 1))
    s.close()
