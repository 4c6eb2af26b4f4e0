"""Host-side drivers of the optimizer loop (Algorithm 1) and the Adam baseline.

Paper: Algorithm 1 (order of the steps), Methodology ("Algorithm Design":
mini-batches S1, S2 and the Hutchinson interval l) and the evaluation
settings: l = 10, theta1 = 0.9, theta2 = 0.999, |S1| = |S2| = nu = 1, epsilon
decaying exponentially from 1e-6 to 1e-8 over the run.  Readings: iteration t
is a Hutchinson step when (t - 1) mod l == 0; the decay is log-linear in t.
Adam uses the 3DGS per-group learning rates, the mean's decaying
log-linearly from 1.6e-4 to 1.6e-6 times the scene extent.

Every iteration runs entirely in the HIP library; this module only picks
cameras and schedules.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from .api import Scene


def eps_schedule(t: int, T: int, eps0: float = 1e-6, eps1: float = 1e-8) -> float:
    if T <= 1:
        return eps0
    f = min(max((t - 1) / (T - 1), 0.0), 1.0)
    return math.exp(math.log(eps0) + f * (math.log(eps1) - math.log(eps0)))


def adam_lrs(t: int, T: int, extent: float) -> dict:
    f = min(max(t / max(T, 1), 0.0), 1.0)
    lr_mu = math.exp((1 - f) * math.log(1.6e-4 * extent) + f * math.log(1.6e-6 * extent))
    return dict(mu=lr_mu, f_dc=2.5e-3, f_rest=2.5e-3 / 20.0, opacity=0.05, scale=5e-3, rot=1e-3)


@dataclass
class TRConfig:
    l: int = 10
    theta1: float = 0.9
    theta2: float = 0.999
    nu: int = 1
    s1: int = 1
    s2: int = 1
    budget: int = 30000
    seed: int = 4002
    probe_seed: int = 5002
    # trust-region radius variant bits; default TR_SH_JOINT: the view-dependent
    # SH coefficients share the radius that bounds the colour change of moving
    # all of them at once (the printed radius gives each of them the base
    # colour's, which lets the colour move by many times eta_C)
    variant: int = 4
    fused: bool = True  # one gs3_tr_iteration call per step (else grad / hvp_diag / tr_step)


class TRTrainer:
    """Algorithm 1 on a resident Scene."""

    def __init__(self, scene: Scene, train_ids, cfg: TRConfig | None = None):
        self.scene = scene
        self.train = list(train_ids)
        self.cfg = cfg or TRConfig()
        self.rng = np.random.default_rng(self.cfg.seed)
        # gradient and D_t buffers only for the unfused path (the fused
        # iteration keeps them inside the scene)
        self.g = None if self.cfg.fused else scene._empty_like_params()
        self.D = None if self.cfg.fused else scene._empty_like_params()
        self.t = 0
        # the last iteration's choices: (t, S1, S2, probe seed, epsilon)
        self.last = None

    def step(self):
        c = self.cfg
        self.t += 1
        t = self.t
        S1 = [self.train[i] for i in self.rng.integers(len(self.train), size=c.s1)]
        eps = eps_schedule(t, c.budget)
        S2 = []
        if (t - 1) % c.l == 0:
            S2 = [self.train[i] for i in self.rng.integers(len(self.train), size=c.s2)]
        self.last = (t, S1, S2, c.probe_seed + t, eps)
        if c.fused:
            self.scene.tr_iteration(S1, S2, c.nu, c.probe_seed + t, c.theta1, c.theta2, eps, variant=c.variant)
            return
        self.scene.grad(S1, out=self.g)
        if S2:
            self.scene.hvp_diag(S2, c.nu, c.probe_seed + t, out=self.D)
            self.scene.tr_step(self.g, self.D, c.theta1, c.theta2, eps, variant=c.variant)
        else:
            self.scene.tr_step(self.g, None, c.theta1, c.theta2, eps, variant=c.variant)


class AdamTrainer:
    """The Adam baseline (optionally ADAM-TR: clipped by the Hellinger radius)."""

    def __init__(self, scene: Scene, train_ids, extent: float, budget: int = 30000, seed: int = 4002,
                 trust_region: bool = False):
        self.scene = scene
        self.train = list(train_ids)
        self.extent = extent
        self.budget = budget
        self.trust_region = trust_region
        self.rng = np.random.default_rng(seed)
        self.g = scene._empty_like_params()
        self.t = 0

    def step(self):
        self.t += 1
        j = self.train[int(self.rng.integers(len(self.train)))]
        self.scene.grad([j], out=self.g)
        eps = eps_schedule(self.t, self.budget) if self.trust_region else None
        self.scene.adam_step(self.g, adam_lrs(self.t, self.budget, self.extent), self.t, epsilon=eps)


def mean_psnr(scene: Scene, ids) -> float:
    return float(np.mean([scene.psnr(j) for j in ids]))


def fit(trainer, scene: Scene, test_ids, iters: int, eval_every: int = 500, target_psnr: float | None = None,
        log=None, interpolate: bool = False):
    """Run `iters` iterations; evaluate the held-out PSNR every `eval_every`.
    The clock counts training only (evaluation excluded).  Returns (history,
    seconds to target): the training time of the first evaluation at or above
    the target, or with `interpolate` the time at which the PSNR line between
    that evaluation and the one before it crosses the target."""
    hist = []
    train_s = 0.0
    reached = None
    done = 0
    prev = (0, 0.0, mean_psnr(scene, test_ids)) if interpolate else None
    while done < iters:
        n = min(eval_every, iters - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            trainer.step()
        torch.cuda.synchronize()
        train_s += time.perf_counter() - t0
        done += n
        p = mean_psnr(scene, test_ids)
        hist.append((done, train_s, p))
        if log:
            log(f"iter {done} train_s {train_s:.2f} psnr {p:.3f}")
        if target_psnr is not None and reached is None and p >= target_psnr:
            reached = train_s
            if interpolate and prev is not None and prev[2] < target_psnr:
                f = (target_psnr - prev[2]) / (p - prev[2])
                reached = prev[1] + f * (train_s - prev[1])
        prev = (done, train_s, p)
    return hist, reached
