"""Shared test helpers (test infrastructure; no method arithmetic)."""
import numpy as np
import torch

from oracle import render as R

GROUPS = {"mu": slice(0, 3), "scale": slice(3, 6), "rot": slice(6, 10), "opacity": slice(10, 11),
          "f_dc": slice(11, 14), "f_rest": slice(14, None)}


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def group_errors(a, b, p):
    """Relative L2 error per parameter group.  A group whose reference is
    (numerically) zero -- e.g. the rotation gradient of isotropic Gaussians --
    is measured against the norm of the whole vector instead."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    total = np.linalg.norm(b)
    out = {}
    for k, sl in GROUPS.items():
        rows = range(p)[sl]
        if len(rows) == 0:
            continue
        nb = np.linalg.norm(b[sl])
        denom = nb if nb > 1e-6 * total else total
        out[k] = float(np.linalg.norm(a[sl] - b[sl]) / denom) if denom > 0 else float(np.linalg.norm(a[sl]))
    return out


def offset_targets(x, cams, sh_degree, seed, lo=0.05, hi=0.15):
    """Oracle render of x plus a random +-U[lo, hi] per pixel and channel, so
    every residual is at least `lo` away from the L1 kink and SSIM stays far
    from 1 (the Gauss-Newton weights are then well conditioned)."""
    rng = np.random.default_rng(seed)
    out = []
    for cam in cams:
        img = R.render(torch.tensor(np.asarray(x, np.float64)), cam, sh_degree).numpy()
        sgn = rng.choice([-1.0, 1.0], size=img.shape)
        out.append((img + sgn * rng.uniform(lo, hi, size=img.shape)).astype(np.float32))
    return out


def group_max_abs(a, b, p):
    """Largest elementwise error per parameter group, relative to the group's
    largest reference entry (the whole vector's when the group is ~zero):
    a few bad entries can hide inside a group's L2 norm, not here."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    top = np.abs(b).max() if b.size else 0.0
    out = {}
    for k, sl in GROUPS.items():
        if len(range(p)[sl]) == 0:
            continue
        ref = np.abs(b[sl]).max()
        denom = ref if ref > 1e-6 * top else top
        err = np.abs(a[sl] - b[sl]).max()
        out[k] = float(err / denom) if denom > 0 else float(err)
    return out


def view_flips(x, cams, ids, sh_degree, tiles=None):
    """Summed float32-vs-float64 decision flips (skip, clamp, stop) over views."""
    from oracle import render as R

    tot = dict(skip=0, clamp=0, stop=0, evaluations=0, pixels=0)
    for j in ids:
        r = R.decision_flips(np.asarray(x, np.float64), cams[j], sh_degree, tiles=tiles)
        for k in tot:
            tot[k] += r[k]
    return tot
