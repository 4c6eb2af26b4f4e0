"""The optimizer of Algorithm 1 (3DGS^2-TR) and its Adam baseline, in FP64.

Paper passages followed (section / equation / algorithm):

* Methodology, "Algorithm Design": stochastic gradient g_t with the scale
  (1/m)(M/|S1|); EMA of g with theta1; Hutchinson estimate D_t with the scale
  (1/m)(M/|S2|)(1/nu) and Rademacher probes; EMA of D with theta2 on every
  l-th iteration; step -D^-1 g; parameter-wise clip by eta = SHD(x, eps).
* Algorithm 1 for the order of the steps; ``run_tr`` is the algorithm as a
  plain loop over t = 1..T (pinned on a separable quadratic, where the
  Gauss-Newton matrix and the EMAs have closed forms).
* Background, Eq. objective: J is the Jacobian of F = sqrt(loss components),
  so J^T F = 1/2 grad(sum of components) and J^T J z is formed from an image
  JVP, the loss Jacobian and an image VJP (Gauss-Newton).
* Methodology, "Trust-Region Based on Squared Hellinger Distance" and the
  appendix derivations: closed-form H^2, scale normalisation by det S, and the
  bounds on mu, S, alpha, colour and the quaternion.

Readings where the paper is silent, ambiguous or garbled:

* GN weight floor: J involves 1/(2 sqrt(l)), singular at l = 0; the weight
  1/(4 l) uses max(l, delta_l) with delta_l = 1e-6.  The gradient stays exact.
* Iteration t is a Hutchinson step when (t - 1) mod l == 0 (the printed
  "t mod l = 1" never fires for l = 1).
* No bias correction of either EMA (Algorithm 1 as printed; initial values 0).
* Where Dhat <= 0 or is not finite, the step is -sign(ghat) * eta when eta is
  finite, else 0 (the limit of a vanishing positive floor on Dhat).
* Hellinger distance H^2 = 1/2 int (sqrt G - sqrt G')^2; the closed form then
  has the -1/8 in the exponent as in the mean-bound derivation.
* The mean bound uses the printed Sigma_cc; the scale, opacity and colour
  bounds are used as printed.  The quaternion constant is
  beta_c = T''(0) = 2 ||S A_c S^-1||_F^2 + 2 tr(R^T d^2R/dq_c^2), A_c = R^T dR/dq_c.
* The colour bound uses the base colour C_c = 0.5 + C0 f_{0,c} floored at
  1/255; every SH coefficient of channel c gets eta_C / C0.
* The clip acts on raw parameters: eta for log-scale is eta_s / s, for the
  opacity logit eta_alpha / (alpha (1 - alpha)).
* epsilon decays log-linearly from 1e-6 to 1e-8 over the T iterations.
* Adam: Kingma-Ba with bias correction, betas (0.9, 0.999), eps 1e-15 and the
  3DGS per-group learning rates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from .gaussians import DT, SH_C0, n_params, rotation, sh_basis, split
from .binning import Bins, bin_view
from .render import render
from .loss import loss_components, ssim_map

GN_FLOOR = 1e-6
COLOUR_FLOOR = 1.0 / 255.0


# ----------------------------------------------------------------------------
# Problem definition


@dataclass
class Problem:
    """Cameras, targets and the constants of the objective (Eq. objective)."""

    cameras: list
    targets: list  # float arrays [H, W, 3]
    sh_degree: int
    lam: float = 0.2
    background: tuple = (0.0, 0.0, 0.0)
    train_ids: list = field(default_factory=list)

    def __post_init__(self):
        if not self.train_ids:
            self.train_ids = list(range(len(self.cameras)))

    @property
    def M(self) -> int:
        return len(self.train_ids)

    @property
    def m(self) -> int:
        return sum(6 * self.cameras[i].height * self.cameras[i].width for i in self.train_ids)


def _t(x) -> torch.Tensor:
    return torch.as_tensor(np.asarray(x, np.float64), dtype=DT)


def bins_for(x, prob: Problem, ids) -> dict:
    x32 = np.asarray(x, np.float32)
    return {j: bin_view(x32, prob.cameras[j]) for j in ids}


def image_loss_sum(x: torch.Tensor, prob: Problem, j: int, bins: Bins) -> torch.Tensor:
    img = render(x, prob.cameras[j], prob.sh_degree, bins, prob.background)
    l1, ls = loss_components(img, _t(prob.targets[j]), prob.lam)
    return l1.sum() + ls.sum()


def objective(x, prob: Problem, ids=None, bins=None) -> float:
    """f = 1/(2m) sum over images of the sum of their loss components."""
    ids = prob.train_ids if ids is None else ids
    xt = _t(x)
    bins = bins or bins_for(x, prob, ids)
    with torch.no_grad():
        tot = sum(float(image_loss_sum(xt, prob, j, bins[j])) for j in ids)
    return tot / (2.0 * prob.m)


def gradient(x, prob: Problem, S1, bins=None):
    """g_t = (1/m)(M/|S1|) sum_{j in S1} J_j^T f_j = (M/(2m|S1|)) grad sum_j sum_k l_jk.

    Returns (g [P, N] float64 numpy, f_S1) where f_S1 = 1/(2m) sum over S1 of
    the loss components (the mini-batch's share of the objective).
    """
    xt = _t(x).requires_grad_(True)
    bins = bins or bins_for(x, prob, S1)
    tot = sum(image_loss_sum(xt, prob, j, bins[j]) for j in S1)
    tot.backward()
    scale = prob.M / (2.0 * prob.m * len(S1))
    return (xt.grad * scale).numpy(), float(tot.detach()) / (2.0 * prob.m)


def loss_cotangent(img: torch.Tensor, tgt: torch.Tensor, lam: float) -> torch.Tensor:
    """d(sum_k l_k)/dC, the image cotangent of the summed loss components."""
    im = img.detach().clone().requires_grad_(True)
    l1, ls = loss_components(im, tgt, lam)
    (l1.sum() + ls.sum()).backward()
    return im.grad


def gn_cotangent(img: torch.Tensor, tgt: torch.Tensor, u: torch.Tensor, lam: float,
                 floor: float = GN_FLOOR) -> torch.Tensor:
    """y = sum_k (dl_k/dC)^T w_k, w_k = (dl_k/dC . u) / (4 max(l_k, floor))."""
    r = img - tgt
    s = torch.sign(r)
    l1 = (1.0 - lam) * torch.abs(r)
    v1 = (1.0 - lam) * s * u
    w1 = v1 / (4.0 * torch.clamp(l1, min=floor))
    y = (1.0 - lam) * s * w1
    if lam > 0.0:
        ssim_fn = lambda im: ssim_map(im, tgt)  # noqa: E731
        S, dS = torch.func.jvp(ssim_fn, (img,), (u,))
        ls = lam * (1.0 - S)
        v2 = -lam * dS
        w2 = v2 / (4.0 * torch.clamp(ls, min=floor))
        _, vjp_fn = torch.func.vjp(ssim_fn, img)
        y = y + vjp_fn(-lam * w2)[0]
    return y


def gn_hvp_image(x, prob: Problem, j: int, z, bins: Bins | None = None, floor: float = GN_FLOOR):
    """h = J_img^T y with u = J_img z and y the Gauss-Newton cotangent (image j)."""
    xt = _t(x)
    zt = _t(z)
    bins = bins or bin_view(np.asarray(x, np.float32), prob.cameras[j])
    f = lambda xx: render(xx, prob.cameras[j], prob.sh_degree, bins, prob.background)  # noqa: E731
    img, u = torch.func.jvp(f, (xt,), (zt,))
    y = gn_cotangent(img, _t(prob.targets[j]), u, prob.lam, floor)
    _, vjp_fn = torch.func.vjp(f, xt)
    return vjp_fn(y)[0].numpy()


# ----------------------------------------------------------------------------
# Rademacher probes: SplitMix64 (Steele, Lea and Flood, 2014) as a counter hash.

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, np.uint64)
    with np.errstate(over="ignore"):
        z = v + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def probe(seed: int, i: int, p: int, n: int) -> np.ndarray:
    """z^(i) in {-1, +1}^{P x N}: +1 when the top bit of the hash of
    (seed, i, component * N + gaussian) is clear."""
    inner = splitmix64(np.array([np.uint64(seed) ^ np.uint64(i)], np.uint64))[0]
    k = np.arange(p * n, dtype=np.uint64)
    h = splitmix64(k ^ inner)
    return np.where((h >> np.uint64(63)) == 0, 1.0, -1.0).reshape(p, n)


def hutchinson(x, prob: Problem, S2, nu: int, seed: int, bins=None, floor: float = GN_FLOOR):
    """D_t = (1/m)(M/|S2|)(1/nu) sum_i z^(i) . sum_{j in S2} J_j^T J_j z^(i)."""
    x = np.asarray(x)
    p, n = x.shape
    bins = bins or bins_for(x, prob, S2)
    acc = np.zeros((p, n))
    for i in range(nu):
        z = probe(seed, i, p, n)
        hsum = np.zeros((p, n))
        for j in S2:
            hsum += gn_hvp_image(x, prob, j, z, bins[j], floor)
        acc += z * hsum
    return acc * (prob.M / (prob.m * len(S2) * nu))


# ----------------------------------------------------------------------------
# Squared Hellinger distance and the trust-region radius


def hellinger2(Z1, mu1, S1, Z2, mu2, S2) -> float:
    """1/2 int (sqrt(G) - sqrt(G'))^2 for G = Z N(mu, S) (any dimension)."""
    mu1, mu2 = np.atleast_1d(np.asarray(mu1, float)), np.atleast_1d(np.asarray(mu2, float))
    S1, S2 = np.atleast_2d(np.asarray(S1, float)), np.atleast_2d(np.asarray(S2, float))
    Sm = 0.5 * (S1 + S2)
    d = mu1 - mu2
    bc = (np.linalg.det(S1) ** 0.25 * np.linalg.det(S2) ** 0.25 / np.sqrt(np.linalg.det(Sm))
          * math.exp(-0.125 * float(d @ np.linalg.solve(Sm, d))))
    return 0.5 * (Z1 + Z2) - math.sqrt(Z1 * Z2) * bc


def quaternion_beta(log_s, q) -> np.ndarray:
    """beta_c = T''(0) for each quaternion component, from the appendix:
    2 ||S dE S^-1||_F^2 + 2 tr(d^2E), dE = R^T dR/dq_c, d^2E = R^T d^2R/dq_c^2."""
    ls = torch.as_tensor(np.asarray(log_s, float), dtype=DT).reshape(-1, 3)
    qq = torch.as_tensor(np.asarray(q, float), dtype=DT).reshape(-1, 4)
    s = torch.exp(ls)
    R = rotation(qq)  # [N,3,3]
    dR = torch.func.vmap(torch.func.jacfwd(rotation))(qq)  # [N,3,3,4]
    d2R = torch.func.vmap(torch.func.jacfwd(torch.func.jacfwd(rotation)))(qq)  # [N,3,3,4,4]
    out = np.zeros((qq.shape[0], 4))
    Rt = R.transpose(-1, -2)
    for c in range(4):
        dE = Rt @ dR[..., c]
        d2E = Rt @ d2R[..., c, c]
        SdES = s[:, :, None] * dE / s[:, None, :]
        t1 = 2.0 * (SdES ** 2).sum((-1, -2))
        t2 = 2.0 * d2E.diagonal(dim1=-2, dim2=-1).sum(-1)
        b = (t1 + t2).numpy()
        # The two terms cancel exactly when S is isotropic in the rotated
        # plane (T is then constant); a sum below their rounding error is 0.
        noise = 64.0 * np.finfo(np.float64).eps * (np.abs(t1.numpy()) + np.abs(t2.numpy()))
        out[:, c] = np.where(np.abs(b) <= noise, 0.0, b)
    return out


def sh_rest_abs_max(sh_degree: int) -> float:
    """max over unit directions d of sum_{k >= 1} |Y_k(d)| (0 at degree 0).

    Found numerically: the best of a dense random sampling of the sphere,
    refined by Nelder-Mead from the best samples (the function is smooth
    away from the zero sets of the Y_k).
    """
    if sh_degree == 0:
        return 0.0
    if sh_degree in _SH_ABS_MAX:
        return _SH_ABS_MAX[sh_degree]
    from scipy.optimize import minimize

    def neg(a):
        th, ph = a
        d = torch.tensor([[math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]],
                         dtype=torch.float64)
        return -float(sh_basis(d, sh_degree)[0, 1:].abs().sum())

    rng = np.random.default_rng(0)
    d = rng.normal(size=(100000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    vals = sh_basis(torch.tensor(d), sh_degree)[:, 1:].abs().sum(1).numpy()
    best = float(vals.max())
    for i in np.argsort(-vals)[:24]:
        a0 = [math.acos(max(-1.0, min(1.0, d[i, 2]))), math.atan2(d[i, 1], d[i, 0])]
        r = minimize(neg, a0, method="Nelder-Mead", options=dict(xatol=1e-12, fatol=1e-15, maxiter=4000))
        best = max(best, -float(r.fun))
    _SH_ABS_MAX[sh_degree] = best
    return best


_SH_ABS_MAX: dict = {}


def shd_eta(x, eps: float, sh_degree: int, colour_floor: float = COLOUR_FLOOR,
            mean_bound: str = "printed", constants: str = "printed", sh_rest: str = "base") -> np.ndarray:
    """eta = SHD(x, eps) in raw-parameter space, [P, N] (inf = unconstrained).

    mean_bound "printed" uses Sigma_cc as the appendix does (exact only for an
    axis-aligned Sigma); "exact" uses 1 / (Sigma^-1)_cc, the exact second-order
    radius of a move along axis c for any rotation.
    constants "printed" keeps the appendix constants, whose Taylor steps make
    the scale, opacity, colour and quaternion radii conservative (the exact
    H^2 at eta is 0.75, 0.5, 0.5 and about 0.5 times eps); "second_order"
    rescales eta^2 by 1/0.75, 2, 2 and 2 (constants 8/3, 8, 8 and 16 in place
    of 2, 4, 4 and 8) so that every class spends eps to second order.
    sh_rest "base" gives every SH coefficient of channel c the base colour's
    radius eta_C / C0; "joint" keeps that for the DC coefficient and gives the
    view-dependent coefficients (k >= 1) the common radius eta_C / S, S the
    maximum over directions of sum_k |Y_k|, so that moving all of them at once
    changes the colour by at most eta_C in every direction.
    """
    xt = _t(x)
    p = split(xt, sh_degree)
    n = xt.shape[1]
    alpha = torch.sigmoid(p["logit"]).numpy()
    s = torch.exp(p["log_s"]).numpy()
    R = rotation(p["quat"]).numpy()
    Sigma = np.einsum("nik,nk,njk->nij", R, s * s, R)
    with np.errstate(divide="ignore", invalid="ignore"):
        L = np.where(eps < alpha, -np.log1p(-eps / alpha), np.inf)
    eta = np.zeros((n_params(sh_degree), n))
    if mean_bound == "exact":
        diag = 1.0 / np.linalg.inv(Sigma).diagonal(axis1=1, axis2=2)
    else:
        diag = Sigma.diagonal(axis1=1, axis2=2)
    if constants == "second_order":
        k_s, k_q, k_a, k_c = 8.0 / 3.0, 16.0, 8.0, 8.0
    else:
        k_s, k_q, k_a, k_c = 2.0, 8.0, 4.0, 4.0
    for c in range(3):
        eta[c] = np.sqrt(8.0 * diag[:, c] * L)
        eta[3 + c] = np.sqrt(k_s * s[:, c] ** 2 * eps / alpha) / s[:, c]
    beta = quaternion_beta(p["log_s"].numpy(), p["quat"].numpy())
    with np.errstate(divide="ignore", invalid="ignore"):
        for c in range(4):
            eta[6 + c] = np.where(beta[:, c] > 0, np.sqrt(k_q * L / beta[:, c]), np.inf)
    eta[10] = np.sqrt(k_a * alpha * eps) / (alpha * (1.0 - alpha))
    base = 0.5 + SH_C0 * p["sh"][:, 0, :].numpy()  # [N, 3]
    eta_C = np.sqrt(k_c * np.maximum(base, colour_floor) * eps / alpha[:, None])
    k = (sh_degree + 1) ** 2
    rest = sh_rest_abs_max(sh_degree) if sh_rest == "joint" else SH_C0
    for kk in range(k):
        for c in range(3):
            eta[11 + 3 * kk + c] = eta_C[:, c] / (SH_C0 if kk == 0 else rest)
    return eta


# ----------------------------------------------------------------------------
# The update of Algorithm 1


def eps_schedule(t: int, T: int, eps0: float = 1e-6, eps1: float = 1e-8) -> float:
    if T <= 1:
        return eps0
    return math.exp(math.log(eps0) + (t - 1) / (T - 1) * (math.log(eps1) - math.log(eps0)))


def is_hutchinson_step(t: int, l: int) -> bool:
    return (t - 1) % l == 0


def tr_step(x, g, ghat, Dhat, D_t, theta1: float, theta2: float, eps: float, sh_degree: int,
            eta=None, mean_bound: str = "printed", constants: str = "printed", sh_rest: str = "base"):
    """One update of Algorithm 1 given g_t (and D_t on a Hutchinson step, else None).

    Returns (x_next, ghat_next, Dhat_next, dx_hat, eta).
    """
    x, g, ghat, Dhat = (np.asarray(a, np.float64) for a in (x, g, ghat, Dhat))
    ghat = theta1 * ghat + (1.0 - theta1) * g
    if D_t is not None:
        Dhat = theta2 * Dhat + (1.0 - theta2) * np.asarray(D_t, np.float64)
    if eta is None:
        eta = shd_eta(x, eps, sh_degree, mean_bound=mean_bound, constants=constants, sh_rest=sh_rest)
    with np.errstate(divide="ignore", invalid="ignore"):
        newton = -ghat / Dhat
        fallback = np.where(np.isfinite(eta), -np.sign(ghat) * eta, 0.0)
        dx = np.where((Dhat > 0) & np.isfinite(Dhat) & np.isfinite(newton), newton, fallback)
    dx_hat = np.minimum(np.maximum(dx, -eta), eta)
    return x + dx_hat, ghat, Dhat, dx_hat, eta


ADAM_GROUPS = ("mu", "f_dc", "f_rest", "opacity", "scale", "rot")


def adam_group_rows(sh_degree: int) -> dict:
    p = n_params(sh_degree)
    return dict(mu=range(0, 3), scale=range(3, 6), rot=range(6, 10), opacity=range(10, 11),
                f_dc=range(11, 14), f_rest=range(14, p))


def adam_lrs(t: int, T: int, extent: float) -> dict:
    """3DGS per-group learning rates; the mean's decays log-linearly."""
    frac = min(max(t / max(T, 1), 0.0), 1.0)
    lr_mu = math.exp((1 - frac) * math.log(1.6e-4 * extent) + frac * math.log(1.6e-6 * extent))
    return dict(mu=lr_mu, f_dc=2.5e-3, f_rest=2.5e-3 / 20.0, opacity=0.05, scale=5e-3, rot=1e-3)


def adam_step(x, g, m, v, step: int, lrs: dict, sh_degree: int, b1=0.9, b2=0.999, eps=1e-15):
    """Kingma-Ba Adam with bias correction and per-group learning rates."""
    x, g, m, v = (np.asarray(a, np.float64).copy() for a in (x, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    rows = adam_group_rows(sh_degree)
    for name, rr in rows.items():
        rr = list(rr)
        x[rr] -= lrs[name] * mhat[rr] / (np.sqrt(vhat[rr]) + eps)
    return x, m, v


# ----------------------------------------------------------------------------
# Algorithm 1 as a plain loop


def run_tr(x1, T: int, grad_fn, hutch_fn, eta_fn, l: int = 10, theta1: float = 0.9, theta2: float = 0.999,
           eps0: float = 1e-6, eps1: float = 1e-8, keep_x: bool = True):
    """Algorithm 1 for t = 1..T, with the iteration's pieces passed in.

    grad_fn(x, t)  -> g_t, the stochastic gradient on iteration t's batch S1;
    hutch_fn(x, t) -> D_t = Hutch(x_t, S2, nu) on iteration t's batch S2,
                      called only on Hutchinson iterations, (t - 1) mod l = 0;
    eta_fn(x, eps) -> eta = SHD(x, eps) at the current parameters.
    The budget of iteration t is eps_schedule(t, T, eps0, eps1) (the
    evaluation's decay of epsilon over the run).  Both EMAs start at zero and
    are not bias-corrected; on other iterations Dhat is kept.

    Returns (x_{T+1}, ghat_T, Dhat_T, log): one record per iteration with t,
    eps, whether it was a Hutchinson iteration, copies of x_{t+1}, ghat_t,
    Dhat_t and the clipped step (x_{t+1} only when keep_x), and the step's
    diagnostics: the share of coordinates whose step was clipped to the
    radius, the share taking the rule for Dhat <= 0, and the step norm.
    """
    x = np.asarray(x1, np.float64).copy()
    ghat = np.zeros_like(x)
    Dhat = np.zeros_like(x)
    log = []
    for t in range(1, T + 1):
        eps = eps_schedule(t, T, eps0, eps1)
        g = np.asarray(grad_fn(x, t), np.float64)
        D = np.asarray(hutch_fn(x, t), np.float64) if is_hutchinson_step(t, l) else None
        eta = np.asarray(eta_fn(x, eps), np.float64)
        x_next, ghat, Dhat, dx_hat, _ = tr_step(x, g, ghat, Dhat, D, theta1, theta2, eps, 0, eta=eta)
        with np.errstate(divide="ignore", invalid="ignore"):
            newton = -ghat / Dhat
            curved = (Dhat > 0) & np.isfinite(Dhat) & np.isfinite(newton)
            clipped = curved & (np.abs(newton) > eta)
        log.append(dict(t=t, eps=eps, hutch=D is not None, x=x_next.copy() if keep_x else None, ghat=ghat.copy(),
                        Dhat=Dhat.copy(), dx=dx_hat.copy(), clipped=float(clipped.mean()),
                        nonpos=float((~curved).mean()), step_norm=float(np.linalg.norm(dx_hat))))
        x = x_next
    return x, ghat, Dhat, log


def run_tr_problem(x1, prob: Problem, T: int, S1s, S2s, nu: int, seeds, l: int = 10, theta1: float = 0.9,
                   theta2: float = 0.999, eps0: float = 1e-6, eps1: float = 1e-8, mean_bound: str = "printed",
                   constants: str = "printed", sh_rest: str = "base"):
    """run_tr on the objective of Eq. objective: S1s[t-1] and S2s[t-1] are
    iteration t's image batches, seeds[t-1] its probe seed (only Hutchinson
    iterations use S2 and the seed)."""
    return run_tr(x1, T,
                  lambda x, t: gradient(x, prob, S1s[t - 1])[0],
                  lambda x, t: hutchinson(x, prob, S2s[t - 1], nu, seeds[t - 1]),
                  lambda x, eps: shd_eta(x, eps, prob.sh_degree, mean_bound=mean_bound, constants=constants,
                                         sh_rest=sh_rest),
                  l=l, theta1=theta1, theta2=theta2, eps0=eps0, eps1=eps1)
