"""Pins of the oracle's optimizer: gradient, Gauss-Newton HVP, Hutchinson,
Hellinger distance, trust-region radius, TR step, Adam and the schedules."""
import math
import os

import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import binning as B
from oracle import gaussians as G
from oracle import loss as Lo
from oracle import method as Mth
from oracle import render as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# helpers: a tiny problem with residuals bounded away from zero


def offset_targets(x, cams, sh_degree, seed, lo=0.05, hi=0.15):
    """Targets = render(x) +- U[lo, hi]: every |r| >= lo, far from the L1 kink."""
    rng = np.random.default_rng(seed)
    out = []
    for cam in cams:
        img = R.render(torch.tensor(x, dtype=torch.float64), cam, sh_degree).numpy()
        sgn = rng.choice([-1.0, 1.0], size=img.shape)
        out.append(img + sgn * rng.uniform(lo, hi, size=img.shape))
    return out


def tiny_problem(seed=3, n=5, sh_degree=1, lam=0.2, size=24, n_cams=2):
    sc = syn.tiny_scene(seed, n=n, sh_degree=sh_degree, width=size, height=size, n_cams=n_cams,
                        log_scale_mean=math.log(0.2))
    x = sc.gt.astype(np.float64)
    tg = offset_targets(x, sc.cameras, sh_degree, seed + 100)
    return x, Mth.Problem(sc.cameras, tg, sh_degree, lam=lam)


def _f_and_decisions(x, prob, bins):
    xt = torch.tensor(x, dtype=torch.float64)
    tot, dec = 0.0, []
    for j in prob.train_ids:
        img, aux = R.render(xt, prob.cameras[j], prob.sh_degree, bins[j], return_aux=True)
        l1, ls = Lo.loss_components(img, torch.tensor(prob.targets[j]), prob.lam)
        tot += float(l1.sum() + ls.sum())
        dec.append(aux["decisions"])
    return tot / (2 * prob.m), dec


def _same(d1, d2):
    return all(R.decisions_equal(a, b) for a, b in zip(d1, d2))


# ----------------------------------------------------------------------------
# probes


def test_splitmix64_published_sequence():
    want = [int(line, 16) for line in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if line.strip() and not line.startswith("#")]
    state = np.array([0], np.uint64)
    got = []
    for _ in range(4):
        got.append(int(Mth.splitmix64(state)[0]))
        with np.errstate(over="ignore"):
            state = state + np.uint64(0x9E3779B97F4A7C15)
    assert got == want


def test_probes_are_balanced_signs_and_pairwise_uncorrelated():
    Z = np.stack([Mth.probe(77, i, 7, 40).ravel() for i in range(2000)])
    assert set(np.unique(Z)) == {-1.0, 1.0}
    assert abs(Z.mean()) < 0.01
    C = (Z.T @ Z) / Z.shape[0]
    off = C[~np.eye(C.shape[0], dtype=bool)]
    assert np.abs(off).max() < 5.0 / math.sqrt(Z.shape[0])
    # different seeds and probe indices give different vectors
    assert not np.array_equal(Mth.probe(1, 0, 3, 10), Mth.probe(2, 0, 3, 10))
    assert not np.array_equal(Mth.probe(1, 0, 3, 10), Mth.probe(1, 1, 3, 10))


# ----------------------------------------------------------------------------
# gradient


def test_gradient_matches_central_finite_differences():
    x, prob = tiny_problem()
    bins = Mth.bins_for(x, prob, prob.train_ids)
    g, f = Mth.gradient(x, prob, prob.train_ids, bins)
    f0, dec0 = _f_and_decisions(x, prob, bins)
    assert abs(f - f0) < 1e-14 * max(1.0, abs(f0))
    rng = np.random.default_rng(5)
    n_ok = 0
    dirs = [rng.normal(size=x.shape) for _ in range(8)]
    for _ in range(40):
        e = np.zeros_like(x)
        e[rng.integers(x.shape[0]), rng.integers(x.shape[1])] = 1.0
        dirs.append(e)
    for v in dirs:
        h = 1e-5
        fp, dp = _f_and_decisions(x + h * v, prob, bins)
        fm, dm = _f_and_decisions(x - h * v, prob, bins)
        if not (_same(dp, dec0) and _same(dm, dec0)):
            continue
        fd = (fp - fm) / (2 * h)
        an = float((g * v).sum())
        roundoff = 50 * np.finfo(float).eps * abs(f0) / h
        assert abs(fd - an) <= 1e-6 * abs(an) + roundoff, (fd, an)
        n_ok += 1
    assert n_ok >= 40


def test_minibatch_gradient_scale():
    x, prob = tiny_problem(n_cams=3, lam=0.0)
    g_all, _ = Mth.gradient(x, prob, prob.train_ids)
    g_each = [Mth.gradient(x, prob, [j])[0] for j in prob.train_ids]
    # each single-image estimate carries M/|S1| = 3; their mean is the full gradient
    assert np.allclose(np.mean(g_each, 0), g_all, rtol=1e-12, atol=1e-18)


# ----------------------------------------------------------------------------
# Gauss-Newton HVP


def _component_jacobian(x, prob, j, bins, h=1e-6):
    """d(loss components of image j)/dx by central differences, plus the components."""
    xt = torch.tensor(x, dtype=torch.float64)

    def comps(xx):
        img = R.render(torch.tensor(xx, dtype=torch.float64), prob.cameras[j], prob.sh_degree, bins)
        l1, ls = Lo.loss_components(img, torch.tensor(prob.targets[j]), prob.lam)
        return torch.cat([l1.reshape(-1), ls.reshape(-1)]).numpy()

    l0 = comps(x)
    J = np.zeros((l0.size, x.size))
    flat = x.ravel()
    for k in range(x.size):
        e = np.zeros_like(flat)
        e[k] = h
        J[:, k] = (comps((flat + e).reshape(x.shape)) - comps((flat - e).reshape(x.shape))) / (2 * h)
    del xt
    return J, l0


def test_gn_hvp_matches_explicit_jacobian_product():
    x, prob = tiny_problem(n=3, sh_degree=1, size=20)
    j = 0
    bins = B.bin_view(x.astype(np.float32), prob.cameras[j])
    J, l0 = _component_jacobian(x, prob, j, bins)
    assert l0.min() > 1e-3  # the weight floor is inactive on this problem
    H = J.T @ (J / (4.0 * l0[:, None]))
    rng = np.random.default_rng(2)
    for _ in range(3):
        z = rng.choice([-1.0, 1.0], size=x.shape)
        h = Mth.gn_hvp_image(x, prob, j, z, bins)
        want = (H @ z.ravel()).reshape(x.shape)
        assert np.linalg.norm(h - want) <= 1e-5 * np.linalg.norm(want)


def test_gn_hvp_is_symmetric_and_psd():
    x, prob = tiny_problem(n=4, sh_degree=0, size=24)
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=x.shape), rng.normal(size=x.shape)
    Ha = Mth.gn_hvp_image(x, prob, 1, a)
    Hb = Mth.gn_hvp_image(x, prob, 1, b)
    lhs, rhs = float((a * Hb).sum()), float((b * Ha).sum())
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0)
    assert float((a * Ha).sum()) >= 0 and float((b * Hb).sum()) >= 0


def test_gn_weight_floor_only_changes_tiny_components():
    img = torch.tensor([[[0.5, 0.5, 0.5]]], dtype=torch.float64)
    tgt = torch.tensor([[[0.5, 0.5 + 1e-9, 0.2]]], dtype=torch.float64)
    u = torch.ones_like(img)
    y = Mth.gn_cotangent(img, tgt, u, 0.0).numpy()[0, 0]
    # r = 0 exactly -> sign 0 -> no contribution; tiny r -> floored weight; large r exact
    assert y[0] == 0.0
    assert abs(y[1] - 1.0 / (4 * 1e-6)) < 1e-6 * (1.0 / (4 * 1e-6))
    assert abs(y[2] - 1.0 / (4 * 0.3)) < 1e-12


# ----------------------------------------------------------------------------
# Hutchinson


def test_hutchinson_is_the_scaled_probe_sum():
    x, prob = tiny_problem(n=3, sh_degree=0, size=20)
    S2 = [0, 1]
    bins = Mth.bins_for(x, prob, S2)
    Hs = []
    for j in S2:
        J, l0 = _component_jacobian(x, prob, j, bins[j])
        Hs.append(J.T @ (J / (4.0 * np.maximum(l0, Mth.GN_FLOOR)[:, None])))
    H = sum(Hs)
    nu, seed = 3, 11
    D = Mth.hutchinson(x, prob, S2, nu, seed, bins)
    acc = np.zeros(x.size)
    for i in range(nu):
        z = Mth.probe(seed, i, *x.shape).ravel()
        acc += z * (H @ z)
    want = acc * prob.M / (prob.m * len(S2) * nu)
    assert np.linalg.norm(D.ravel() - want) <= 1e-5 * np.linalg.norm(want)


def test_hutchinson_mean_converges_to_the_diagonal():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(30, 12))
    H = A.T @ A
    n = H.shape[0]
    nu = 4096
    acc = np.zeros(n)
    for i in range(nu):
        z = Mth.probe(99, i, 1, n).ravel()
        acc += z * (H @ z)
    mean = acc / nu
    var = (H ** 2).sum(1) - np.diag(H) ** 2
    assert np.all(np.abs(mean - np.diag(H)) <= 5 * np.sqrt(var / nu))
    # exactly unbiased over all 2^n sign vectors
    signs = np.array(np.meshgrid(*[[-1.0, 1.0]] * n, indexing="ij")).reshape(n, -1).T
    full = (signs * (signs @ H)).mean(0)
    assert np.allclose(full, np.diag(H), rtol=1e-12)


# ----------------------------------------------------------------------------
# Hellinger distance and the trust region


def test_hellinger_closed_form_matches_quadrature_1d_2d():
    # 1D
    Z1, m1, v1, Z2, m2, v2 = 0.7, 0.1, 0.3, 1.3, -0.4, 0.8
    zs = np.linspace(-12, 12, 200001)
    g1 = Z1 * np.exp(-0.5 * (zs - m1) ** 2 / v1) / math.sqrt(2 * math.pi * v1)
    g2 = Z2 * np.exp(-0.5 * (zs - m2) ** 2 / v2) / math.sqrt(2 * math.pi * v2)
    quad = 0.5 * np.trapezoid((np.sqrt(g1) - np.sqrt(g2)) ** 2, zs)
    assert abs(Mth.hellinger2(Z1, m1, [[v1]], Z2, m2, [[v2]]) - quad) < 1e-10
    # 2D
    S1 = np.array([[0.5, 0.2], [0.2, 0.3]])
    S2 = np.array([[0.4, -0.1], [-0.1, 0.6]])
    mu1, mu2 = np.array([0.1, 0.0]), np.array([-0.2, 0.3])
    g = np.linspace(-6, 6, 1201)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X, Y], -1)

    def dens(Z, mu, S):
        d = P - mu
        q = np.einsum("...i,ij,...j->...", d, np.linalg.inv(S), d)
        return Z * np.exp(-0.5 * q) / (2 * math.pi * math.sqrt(np.linalg.det(S)))

    quad2 = 0.5 * np.trapezoid(np.trapezoid((np.sqrt(dens(0.9, mu1, S1)) - np.sqrt(dens(1.1, mu2, S2))) ** 2, g), g)
    assert abs(Mth.hellinger2(0.9, mu1, S1, 1.1, mu2, S2) - quad2) < 1e-9


def test_hellinger_identities():
    rng = np.random.default_rng(6)
    for _ in range(20):
        A = rng.normal(size=(3, 3))
        S1 = A @ A.T + 0.1 * np.eye(3)
        B_ = rng.normal(size=(3, 3))
        S2 = B_ @ B_.T + 0.1 * np.eye(3)
        m1, m2 = rng.normal(size=3), rng.normal(size=3)
        Z1, Z2 = rng.uniform(0.1, 2, size=2)
        h = Mth.hellinger2(Z1, m1, S1, Z2, m2, S2)
        assert abs(h - Mth.hellinger2(Z2, m2, S2, Z1, m1, S1)) < 1e-13
        assert 0 <= h / (0.5 * (Z1 + Z2)) <= 1
        assert abs(Mth.hellinger2(Z1, m1, S1, Z1, m1, S1)) < 1e-13


def _activated(col):
    s = np.exp(col[3:6])
    R_ = G.rotation(torch.tensor(col[6:10])).numpy()
    return col[0:3], s, R_ @ np.diag(s * s) @ R_.T, 1 / (1 + math.exp(-col[10])), 0.5 + G.SH_C0 * col[11:14]


def _ratio(col, j, eta, eps, channel=None):
    """Exact H^2 / det S of a one-parameter raw step of size eta, over eps."""
    mu, s, S, a, C = _activated(col)
    y = col.copy()
    y[j] += eta
    mu2, s2, S2, a2, C2 = _activated(y)
    w1 = a * (C[channel] if channel is not None else 1.0)
    w2 = a2 * (C2[channel] if channel is not None else 1.0)
    return Mth.hellinger2(w1 * np.prod(s), mu, S, w2 * np.prod(s2), mu2, S2) / np.prod(s) / eps


@pytest.mark.parametrize("eps", [1e-7, 1e-9])
def test_trust_region_radius_meets_its_hellinger_budget(eps):
    col = np.zeros(14)
    col[3:6] = np.log([0.3, 0.1, 0.05])
    col[10] = 0.5
    col[11:14] = [0.5, -0.3, 1.0]
    col[6:10] = [0, 0, 0, 1]  # axis aligned
    eta = Mth.shd_eta(col[:, None], eps, 0)[:, 0]
    for c in range(3):
        assert abs(_ratio(col, c, eta[c], eps) - 1.0) < 1e-3  # mean: exact
        assert abs(_ratio(col, 3 + c, eta[3 + c], eps) - 0.75) < 2e-3  # scale
        assert abs(_ratio(col, 11 + c, eta[11 + c], eps, channel=c) - 0.5) < 2e-3  # colour
    assert abs(_ratio(col, 10, eta[10], eps) - 0.5) < 2e-3  # opacity
    for c in range(3):  # quaternion (q_w has beta = 0 at the identity: unconstrained)
        assert abs(_ratio(col, 6 + c, eta[6 + c], eps) - 0.5) < 2e-3
    assert np.isinf(eta[9])
    # a rotated anisotropic Gaussian: printed mean bound is exceeded by at most
    # lambda_max / lambda_min, the quaternion bound still lands at ~0.5
    col[6:10] = [0.3, -0.5, 0.2, 0.7]
    eta = Mth.shd_eta(col[:, None], eps, 0)[:, 0]
    lam = np.exp(2 * col[3:6])
    for c in range(3):
        assert 1.0 - 1e-3 <= _ratio(col, c, eta[c], eps) <= lam.max() / lam.min()
    for c in range(4):
        assert abs(_ratio(col, 6 + c, eta[6 + c], eps) - 0.5) < 5e-3
    # the exact mean-bound variant lands on eps for any rotation
    eta_x = Mth.shd_eta(col[:, None], eps, 0, mean_bound="exact")[:, 0]
    for c in range(3):
        assert abs(_ratio(col, c, eta_x[c], eps) - 1.0) < 1e-3


@pytest.mark.parametrize("eps", [1e-7, 1e-9])
def test_second_order_constants_spend_the_whole_budget(eps):
    # with the second-order constants every class lands on H^2 = eps (to
    # second order), for an axis-aligned and a rotated anisotropic Gaussian
    col = np.zeros(14)
    col[3:6] = np.log([0.3, 0.1, 0.05])
    col[10] = -0.7
    col[11:14] = [0.5, -0.3, 1.0]
    for quat in ([0, 0, 0, 1], [0.3, -0.5, 0.2, 0.7]):
        col[6:10] = quat
        eta = Mth.shd_eta(col[:, None], eps, 0, mean_bound="exact", constants="second_order")[:, 0]
        printed = Mth.shd_eta(col[:, None], eps, 0)[:, 0]
        for c in range(3):
            assert abs(_ratio(col, c, eta[c], eps) - 1.0) < 1e-3
            assert abs(_ratio(col, 3 + c, eta[3 + c], eps) - 1.0) < 3e-3
            assert abs(_ratio(col, 11 + c, eta[11 + c], eps, channel=c) - 1.0) < 3e-3
            assert eta[3 + c] > printed[3 + c] and eta[11 + c] > printed[11 + c]
        assert abs(_ratio(col, 10, eta[10], eps) - 1.0) < 3e-3
        for c in range(4):
            if np.isfinite(eta[6 + c]):
                assert abs(_ratio(col, 6 + c, eta[6 + c], eps) - 1.0) < 1e-2


def test_quaternion_beta_matches_second_difference_of_T():
    rng = np.random.default_rng(8)
    for _ in range(5):
        q = rng.normal(size=4) * rng.uniform(0.5, 2.0)
        ls = rng.normal(-2, 0.7, size=3)
        beta = Mth.quaternion_beta(ls, q)[0]
        s = np.exp(ls)
        R0 = G.rotation(torch.tensor(q)).numpy()

        def T(d, c):
            qq = q.copy()
            qq[c] += d
            dR = R0.T @ G.rotation(torch.tensor(qq)).numpy()
            return float(((np.diag(s) @ dR @ np.diag(1 / s)) ** 2).sum())

        for c in range(4):
            h = 1e-4 * np.linalg.norm(q)
            fd = (T(h, c) - 2 * T(0, c) + T(-h, c)) / h ** 2
            assert abs(fd - beta[c]) <= 1e-5 * max(abs(beta[c]), 1.0)


def test_radius_follows_the_anisotropy_intuitions():
    # elongated along x (long) with short y, z; identity rotation
    col = np.zeros(14)
    col[3:6] = np.log([0.5, 0.05, 0.05])
    col[6:10] = [0, 0, 0, 1]
    col[10] = 0.0
    col[11:14] = 0.5
    eps = 1e-7
    eta = Mth.shd_eta(col[:, None], eps, 0)[:, 0]
    assert eta[0] > eta[1]  # moves more freely along the long axis
    assert np.isinf(eta[6])  # rotation about the long axis leaves it unchanged
    assert eta[8] < np.inf and eta[7] < np.inf  # rotations tipping the long axis are bounded
    col2 = col.copy()
    col2[10] = -2.0  # more transparent
    eta2 = Mth.shd_eta(col2[:, None], eps, 0)[:, 0]
    assert np.all(eta2[0:3] > eta[0:3]) and np.all(eta2[6:9][np.isfinite(eta[6:9])] > eta[6:9][np.isfinite(eta[6:9])])
    # isotropic Gaussians are rotation invariant
    col3 = col.copy()
    col3[3:6] = math.log(0.1)
    assert np.all(np.isinf(Mth.shd_eta(col3[:, None], eps, 0)[6:10, 0]))
    # eps >= alpha leaves mean and rotation unconstrained
    col4 = col.copy()
    col4[10] = -20.0
    eta4 = Mth.shd_eta(col4[:, None], 1e-6, 0)[:, 0]
    assert np.all(np.isinf(eta4[0:3]))


# ----------------------------------------------------------------------------
# the update


def test_tr_step_reduces_to_diagonal_newton_and_clips():
    rng = np.random.default_rng(9)
    x = rng.normal(size=(14, 6))
    g = rng.normal(size=x.shape)
    D = rng.uniform(0.5, 2.0, size=x.shape)
    inf = np.full(x.shape, np.inf)
    # theta1 = theta2 = 0 and an unbounded radius: plain diagonal Gauss-Newton
    xn, gh, Dh, dx, _ = Mth.tr_step(x, g, np.zeros_like(x), np.zeros_like(x), D, 0.0, 0.0, 1e-6, 0, eta=inf)
    assert np.allclose(dx, -g / D) and np.allclose(xn, x - g / D)
    # EMA on a non-Hutchinson step keeps Dhat
    xn, gh, Dh2, dx, _ = Mth.tr_step(x, g, g, D, None, 0.9, 0.999, 1e-6, 0, eta=inf)
    assert np.array_equal(Dh2, D) and np.allclose(gh, g)
    # clip to the radius
    eta = np.full(x.shape, 0.01)
    xn, gh, Dh, dx, _ = Mth.tr_step(x, g, np.zeros_like(x), np.zeros_like(x), D, 0.0, 0.0, 1e-6, 0, eta=eta)
    assert np.all(np.abs(dx) <= 0.01 + 1e-18)
    assert np.allclose(dx, np.clip(-g / D, -0.01, 0.01))
    # non-positive curvature: step to the radius against the gradient
    Dn = -D
    xn, gh, Dh, dx, _ = Mth.tr_step(x, g, np.zeros_like(x), np.zeros_like(x), Dn, 0.0, 0.0, 1e-6, 0, eta=eta)
    assert np.allclose(dx, -np.sign(g) * 0.01)
    xn, gh, Dh, dx, _ = Mth.tr_step(x, g, np.zeros_like(x), np.zeros_like(x), Dn, 0.0, 0.0, 1e-6, 0, eta=inf)
    assert np.all(dx == 0)


def test_ema_without_bias_correction():
    g = np.array([[1.0]])
    gh, Dh = np.zeros((1, 1)), np.zeros((1, 1))
    for t in range(1, 4):
        _, gh, Dh, _, _ = Mth.tr_step(np.zeros((1, 1)), g, gh, Dh, np.array([[2.0]]) if t == 1 else None,
                                      0.9, 0.999, 1e-6, 0, eta=np.full((1, 1), np.inf))
    assert abs(gh[0, 0] - (1 - 0.9 ** 3)) < 1e-15
    assert abs(Dh[0, 0] - 0.001 * 2.0) < 1e-15


def test_schedules():
    assert Mth.eps_schedule(1, 100) == pytest.approx(1e-6, rel=1e-14)
    assert Mth.eps_schedule(100, 100) == pytest.approx(1e-8, rel=1e-14)
    assert Mth.eps_schedule(50.5, 100) == pytest.approx(1e-7, rel=1e-12)
    assert [Mth.is_hutchinson_step(t, 10) for t in (1, 2, 10, 11, 21)] == [True, False, False, True, True]
    assert all(Mth.is_hutchinson_step(t, 1) for t in range(1, 5))


def test_adam_matches_torch_optim_for_one_group():
    rng = np.random.default_rng(10)
    x0 = rng.normal(size=(14, 5))
    p = torch.nn.Parameter(torch.tensor(x0))
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.999), eps=1e-15)
    x, m, v = x0.copy(), np.zeros_like(x0), np.zeros_like(x0)
    lrs = {k: 0.01 for k in Mth.ADAM_GROUPS}
    for step in range(1, 6):
        g = rng.normal(size=x0.shape)
        p.grad = torch.tensor(g)
        opt.step()
        x, m, v = Mth.adam_step(x, g, m, v, step, lrs, 0)
    assert np.allclose(x, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_learning_rate_schedule():
    lr0 = Mth.adam_lrs(0, 100, 2.0)
    lr1 = Mth.adam_lrs(100, 100, 2.0)
    assert lr0["mu"] == pytest.approx(3.2e-4) and lr1["mu"] == pytest.approx(3.2e-6)
    assert Mth.adam_lrs(50, 100, 2.0)["mu"] == pytest.approx(3.2e-5)
    assert lr0["f_rest"] == pytest.approx(1.25e-4)


def test_sh_rest_abs_max_pins():
    # degree 1: max over the sphere of C1 (|x| + |y| + |z|) = C1 sqrt(3) in closed form
    assert abs(Mth.sh_rest_abs_max(1) - math.sqrt(3.0) * math.sqrt(3.0 / (4.0 * math.pi))) < 1e-9
    assert Mth.sh_rest_abs_max(0) == 0.0
    # brute force over a dense independent sampling never exceeds the maximum
    # and comes close to it
    rng = np.random.default_rng(77)
    d = rng.normal(size=(200000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for deg in (1, 2, 3):
        v = G.sh_basis(torch.tensor(d), deg)[:, 1:].abs().sum(1).numpy()
        S = Mth.sh_rest_abs_max(deg)
        assert v.max() <= S + 1e-12 and v.max() >= S - 1e-4


def test_joint_sh_radius_bounds_the_colour_change():
    # moving every view-dependent coefficient of a channel by its full radius,
    # with the worst signs for a direction, changes that direction's colour by
    # at most eta_C; the DC radius is unchanged
    rng = np.random.default_rng(78)
    x = np.zeros((59, 1))
    x[3:6, 0] = np.log([0.2, 0.1, 0.05])
    x[6:10, 0] = [0.1, 0.2, -0.3, 0.9]
    x[10, 0] = 0.3
    x[11:14, 0] = [0.4, -0.2, 0.9]
    eps = 1e-6
    base = Mth.shd_eta(x, eps, 3)[:, 0]
    joint = Mth.shd_eta(x, eps, 3, sh_rest="joint")[:, 0]
    assert np.array_equal(base[:14], joint[:14])
    d = rng.normal(size=(20000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = G.sh_basis(torch.tensor(d), 3).numpy()  # [n, 16]
    for c in range(3):
        eta_c = joint[11 + c] * G.SH_C0  # eta_C of the channel
        rest = joint[11 + 3 + c::3][:15]
        assert np.allclose(rest, rest[0])
        worst = (np.abs(Y[:, 1:]) * rest[None, :]).sum(1)
        assert worst.max() <= eta_c * (1 + 1e-9)
        assert worst.max() >= 0.999 * eta_c


def test_adam_group_map_matches_torch_optim_with_six_groups():
    # one learning rate per 3DGS parameter group, all different: the rows of
    # each group are taken from the layout's named views, not from the
    # oracle's row table, and torch's Adam updates each group separately
    rng = np.random.default_rng(12)
    deg = 2
    x0 = rng.normal(size=(G.n_params(deg), 7))
    lrs = dict(mu=1.3e-3, f_dc=2.9e-3, f_rest=3.7e-4, opacity=5.3e-2, scale=7.1e-3, rot=1.1e-2)
    views = G.split(torch.tensor(x0), deg)
    named = dict(mu=views["mu"], scale=views["log_s"], rot=views["quat"], opacity=views["logit"],
                 f_dc=views["sh"][:, 0, :], f_rest=views["sh"][:, 1:, :])
    params = {k: torch.nn.Parameter(v.clone()) for k, v in named.items()}
    opt = torch.optim.Adam([dict(params=[params[k]], lr=lrs[k]) for k in Mth.ADAM_GROUPS], betas=(0.9, 0.999),
                           eps=1e-15)
    x, m, v = x0.copy(), np.zeros_like(x0), np.zeros_like(x0)
    for step in range(1, 6):
        g = rng.normal(size=x0.shape)
        gv = G.split(torch.tensor(g), deg)
        gnamed = dict(mu=gv["mu"], scale=gv["log_s"], rot=gv["quat"], opacity=gv["logit"], f_dc=gv["sh"][:, 0, :],
                      f_rest=gv["sh"][:, 1:, :])
        for k in params:
            params[k].grad = gnamed[k].clone()
        opt.step()
        x, m, v = Mth.adam_step(x, g, m, v, step, lrs, deg)
    xv = G.split(torch.tensor(x), deg)
    got = dict(mu=xv["mu"], scale=xv["log_s"], rot=xv["quat"], opacity=xv["logit"], f_dc=xv["sh"][:, 0, :],
               f_rest=xv["sh"][:, 1:, :])
    for k in params:
        assert np.allclose(got[k].numpy(), params[k].detach().numpy(), rtol=1e-12, atol=1e-15), k
    # every row moved by its own group's rate (the groups are told apart)
    assert len(set(lrs.values())) == 6


# ----------------------------------------------------------------------------
# Algorithm 1 as a loop: pinned on a separable quadratic, where the
# Gauss-Newton matrix is diagonal and known, so every Rademacher probe gives
# z (.) H z = diag(H) exactly


def _quadratic(rng, shape):
    d = rng.uniform(0.5, 3.0, size=shape)
    c = rng.normal(size=shape)
    grad = lambda x, t: d * (x - c)  # noqa: E731
    # Hutchinson on H = diag(d): z (.) (H z) with a probe of the oracle's generator
    hutch = lambda x, t: Mth.probe(77, t, *shape) * (d * Mth.probe(77, t, *shape))  # noqa: E731
    return d, c, grad, hutch


def test_run_tr_one_newton_step_solves_a_quadratic():
    # theta1 = theta2 = 0, l = 1 and no radius: the plain diagonal Gauss-Newton
    # (here Newton) step, which lands on the minimum of a separable quadratic
    rng = np.random.default_rng(20)
    d, c, grad, hutch = _quadratic(rng, (4, 6))
    x1 = rng.normal(size=(4, 6))
    inf = lambda x, eps: np.full(x.shape, np.inf)  # noqa: E731
    x, gh, Dh, log = Mth.run_tr(x1, 3, grad, hutch, inf, l=1, theta1=0.0, theta2=0.0)
    assert np.allclose(log[0]["x"], c, rtol=0, atol=1e-14)
    assert np.allclose(x, c, atol=1e-14) and np.allclose(Dh, d)
    assert all(r["hutch"] for r in log)


def test_run_tr_emas_and_schedule_on_frozen_parameters():
    # a zero radius freezes x, so g_t is constant: the EMAs are geometric sums,
    # ghat_t = (1 - theta1^t) g and, after k Hutchinson iterations,
    # Dhat = (1 - theta2^k) diag(H); Hutchinson runs at t = 1, 1 + l, 1 + 2l, ...
    rng = np.random.default_rng(21)
    d, c, grad, hutch = _quadratic(rng, (3, 5))
    x1 = rng.normal(size=(3, 5))
    seen_eps = []

    def zero(x, eps):
        seen_eps.append(eps)
        return np.zeros(x.shape)

    T, l, th1, th2 = 23, 10, 0.9, 0.999
    x, gh, Dh, log = Mth.run_tr(x1, T, grad, hutch, zero, l=l, theta1=th1, theta2=th2)
    g = d * (x1 - c)
    assert np.array_equal(x, x1)
    assert [r["t"] for r in log if r["hutch"]] == [1, 11, 21]
    for r in log:
        k = (r["t"] - 1) // l + 1
        assert np.allclose(r["ghat"], (1 - th1 ** r["t"]) * g, rtol=1e-12)
        assert np.allclose(r["Dhat"], (1 - th2 ** k) * d, rtol=1e-12)
        assert np.all(r["dx"] == 0)
    # epsilon: 1e-6 at t = 1, 1e-8 at t = T, a constant ratio in between
    assert seen_eps[0] == pytest.approx(1e-6, rel=1e-14) and seen_eps[-1] == pytest.approx(1e-8, rel=1e-14)
    ratios = np.array(seen_eps[1:]) / np.array(seen_eps[:-1])
    assert np.allclose(ratios, (1e-2) ** (1.0 / (T - 1)), rtol=1e-12)


def test_run_tr_clips_to_the_radius_and_reports_it():
    rng = np.random.default_rng(22)
    d, c, grad, hutch = _quadratic(rng, (2, 50))
    x1 = c + rng.choice([-1.0, 1.0], size=c.shape)  # every Newton step has size 1
    eta = lambda x, eps: np.full(x.shape, 0.25)  # noqa: E731
    x, gh, Dh, log = Mth.run_tr(x1, 2, grad, hutch, eta, l=1, theta1=0.0, theta2=0.0)
    assert np.allclose(np.abs(log[0]["dx"]), 0.25) and log[0]["clipped"] == 1.0 and log[0]["nonpos"] == 0.0
    assert np.allclose(np.abs(x - c), 0.5)


def test_run_tr_on_the_objective_matches_its_first_step():
    # the driver on the real objective: iteration 1 is the tr_step of the
    # gradient and Hutchinson estimate at x_1 with eps_1 = 1e-6
    x, prob = tiny_problem(seed=5, n=4, sh_degree=0, size=16)
    S1s, S2s, seeds = [[0], [1]], [[1], [0]], [9, 10]
    xT, gh, Dh, log = Mth.run_tr_problem(x, prob, 2, S1s, S2s, 2, seeds, l=1)
    g1, _ = Mth.gradient(x, prob, [0])
    D1 = Mth.hutchinson(x, prob, [1], 2, 9)
    x2, _, _, dx, _ = Mth.tr_step(x, g1, np.zeros_like(x), np.zeros_like(x), D1, 0.9, 0.999, 1e-6, 0)
    assert np.allclose(log[0]["x"], x2, rtol=0, atol=1e-15) and np.allclose(log[0]["dx"], dx, atol=1e-15)
    assert log[1]["eps"] == pytest.approx(1e-8) and log[1]["hutch"]


def test_trainer_schedules_match_the_oracle():
    # the trainer computes the same epsilon decay and Adam learning rates on
    # the host as the oracle does (two copies of one schedule, tied here)
    from paper_2602_00395_amd import trainer as Tr

    for T in (1, 2, 10, 15000):
        for t in sorted({1, 2, T // 2 + 1, max(T - 1, 1), T}):
            assert Tr.eps_schedule(t, T) == pytest.approx(Mth.eps_schedule(t, T), rel=1e-13), (t, T)
    for t in (0, 1, 500, 29999, 30000):
        a, b = Tr.adam_lrs(t, 30000, 4.4), Mth.adam_lrs(t, 30000, 4.4)
        assert a.keys() == b.keys() and all(a[k] == pytest.approx(b[k], rel=1e-13) for k in a)
