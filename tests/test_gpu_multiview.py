"""Several views (and probes) in one launch: the gradient over a mini-batch S1
and the Hutchinson diagonal over S2 x nu probes run one blend-forward, one
blend-backward and one projection-backward launch per batch of up to eight
(view, probe) entries.  Checked against the FP64 oracle at relative L2
<= 1e-4 per parameter group (plain workload, whole views; object workload,
sampled Gaussians of four views), across a batch boundary (ten views), and
for consistency with the single-view calls."""
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
MAX_ABS = 1e-3
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(got, want, p, flips=None):
    errs = group_errors(got, want, p)
    mx = group_max_abs(got, want, p)
    say("  rel-L2 per group", errs)
    say("  max-abs per group", mx, "flips", flips)
    assert all(e <= TOL for e in errs.values()), errs
    assert all(e <= MAX_ABS for e in mx.values()), mx


def make_scene(x, targets, cams, deg, lam=0.2):
    from paper_2602_00395_amd import Scene

    xt = torch.tensor(np.asarray(x, np.float32), device=DEV)
    tg = [torch.tensor(np.asarray(t, np.float32), device=DEV) for t in targets]
    return Scene(xt, tg, cams, deg, lam=lam)


@pytest.fixture(scope="module")
def c1():
    sc = syn.config1_scene()
    x = sc.init.astype(np.float32)
    targets = offset_targets(x, sc.cameras, 0, seed=4001)
    return sc, x, targets


@pytest.mark.parametrize("S1", [[0, 3, 5, 6], [0, 1, 2, 3, 4, 5, 6, 7, 1, 4]])
def test_batched_gradient_parity_plain(c1, S1):
    """Four views in one batch, and ten views (a batch of eight, then two)."""
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    prob = Mth.Problem(sc.cameras, targets, 0, lam=0.2)
    say("batched grad plain S1", S1)
    want, f_want = Mth.gradient(x, prob, S1)
    got, f_got = s.grad(S1, want_loss=True)
    check(got.cpu().numpy(), want, 14, flips=view_flips(x, sc.cameras, sorted(set(S1)), 0))
    assert abs(f_got - f_want) <= 1e-5 * abs(f_want)
    s.close()


def test_batched_hutchinson_parity_plain(c1):
    """S2 = four views with two probes each: eight (view, probe) entries in one launch."""
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    prob = Mth.Problem(sc.cameras, targets, 0, lam=0.2)
    S2, nu, seed = [1, 2, 4, 7], 2, 5011
    say("batched hvp plain S2", S2, "nu", nu)
    want = Mth.hutchinson(x, prob, S2, nu, seed)
    got = s.hvp_diag(S2, nu, seed).cpu().numpy()
    check(got, want, 14, flips=view_flips(x, sc.cameras, S2, 0))
    # three views with three probes: nine entries, a batch boundary inside a view
    S2b, nub = [0, 3, 6], 3
    say("batched hvp plain S2", S2b, "nu", nub)
    want = Mth.hutchinson(x, prob, S2b, nub, seed + 1)
    got = s.hvp_diag(S2b, nub, seed + 1).cpu().numpy()
    check(got, want, 14, flips=view_flips(x, sc.cameras, S2b, 0))
    s.close()


def test_batched_equals_mean_of_single_views(c1):
    """g over four views in one batch equals the mean of the four single-view
    gradients (each scaled by M/|S1| with |S1| = 1) up to float32 rounding."""
    sc, x, targets = c1
    s = make_scene(x, targets, sc.cameras, 0)
    S1 = [2, 3, 5, 7]
    batched = s.grad(S1).cpu().numpy().astype(np.float64)
    singles = np.mean([s.grad([j]).cpu().numpy().astype(np.float64) for j in S1], axis=0)
    say("batched vs single views rel-L2", rel_l2(batched, singles))
    assert rel_l2(batched, singles) <= 1e-6
    s.close()


def test_batched_fused_iteration_matches_separate_calls(c1):
    """gs3_tr_iteration against the separate calls on the same views, bit for
    bit: |S1| = 4 with |S2| = 2 and nu = 2 (eight entries: D_t formed inside
    the update launch), |S1| = |S2| = 4 with nu = 2 (twelve entries: D_t
    through memory), and a step without Hutchinson."""
    sc, x, targets = c1
    a = make_scene(x, targets, sc.cameras, 0)
    b = make_scene(x, targets, sc.cameras, 0)
    g = a._empty_like_params()
    D = a._empty_like_params()
    plan = [([0, 2, 4, 6], [1, 3], 2), ([0, 2, 4, 6], [1, 3, 5, 7], 2), ([1, 2, 3, 4], [], 1)]
    for it, (S1, S2, nu) in enumerate(plan):
        seed = 7100 + it
        say("batched fused iteration", it, "S1", S1, "S2", S2, "nu", nu)
        if S2:
            a.hvp_diag(S2, nu, seed, out=D)
        a.grad(S1, out=g)
        a.tr_step(g, D if S2 else None, 0.9, 0.999, 1e-6, variant=4)
        b.tr_iteration(S1, S2, nu, seed, 0.9, 0.999, 1e-6, variant=4)
        for name in ("x", "ghat", "dhat"):
            ta, tb = a._empty_like_params(), b._empty_like_params()
            a.export(**{name: ta})
            b.export(**{name: tb})
            assert torch.equal(ta, tb), (it, name, float((ta - tb).abs().max()))
    a.close()
    b.close()


def test_batched_gradient_object_scale_sampled_gaussians():
    """Object scale (100k Gaussians, SH 3, 800x800), S1 = four views, L1 loss:
    the gradient of sampled Gaussians.  In each view a Gaussian's L1 gradient
    involves only the pixels of its own tiles, so the oracle renders just the
    tiles the sampled Gaussians touch in that view (every splat in them), with
    targets offset from its render by +-U[0.05, 0.15] there."""
    sc = syn.config2_scene()
    cam_ids = [2, 9, 17, 30]
    cams = [sc.cameras[j] for j in cam_ids]
    x = sc.init.astype(np.float32)
    x[14:] = sc.gt[14:]  # non-zero higher-order SH so every row is exercised
    rng = np.random.default_rng(43)
    obs = [B.bin_view(x, c) for c in cams]
    # Gaussians visible (1..3 tiles) in every one of the four views
    ok = np.ones(x.shape[1], bool)
    for ob in obs:
        area = (ob.rect[:, 2] - ob.rect[:, 0]) * (ob.rect[:, 3] - ob.rect[:, 1])
        ok &= (ob.tiles_touched >= 1) & (area <= 3)
    pick = np.sort(rng.choice(np.flatnonzero(ok), size=4, replace=False))
    xt = torch.tensor(x, dtype=torch.float64)
    targets, tiles_of, masks = [], [], []
    for c, ob in zip(cams, obs):
        tiles = set()
        for g in pick:
            x0, y0, x1, y1 = (int(v) for v in ob.rect[g])
            tiles |= {ty * ob.tiles_x + tx for ty in range(y0, y1) for tx in range(x0, x1)}
        with torch.no_grad():
            base = R.render(xt, c, 3, ob, tiles=tiles)
        m = ~torch.isnan(base)
        off = rng.uniform(0.05, 0.15, size=base.shape) * rng.choice([-1.0, 1.0], size=base.shape)
        tgt = np.full(base.shape, 0.5)
        tgt[m.numpy()] = base.numpy()[m.numpy()] + off[m.numpy()]
        targets.append(tgt.astype(np.float32))
        tiles_of.append(tiles)
        masks.append(m)
    say("batched grad object scale: Gaussians", pick.tolist(), "tiles", [len(t) for t in tiles_of])
    s = make_scene(x, targets, cams, 3, lam=0.0)
    got = s.grad([0, 1, 2, 3]).cpu().numpy()[:, pick]
    s.close()
    # g = (M / (2 m |S1|)) grad sum_j sum_k l_jk, l = |r| (lambda = 0)
    m_comp = sum(6 * c.height * c.width for c in cams)
    scale = len(cams) / (2.0 * m_comp * 4)
    xg = xt.clone().requires_grad_(True)
    tot = 0.0
    for c, ob, tiles, tgt, m in zip(cams, obs, tiles_of, targets, masks):
        img = R.render(xg, c, 3, ob, tiles=tiles)
        tot = tot + torch.abs(img[m] - torch.tensor(tgt, dtype=torch.float64)[m]).sum()
    tot.backward()
    want = (xg.grad * scale).numpy()[:, pick]
    check(got, want, 59)
