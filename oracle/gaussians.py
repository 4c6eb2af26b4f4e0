"""Gaussian primitive, parameterisation and view-dependent colour (FP64).

Paper: Background, "Review of Gaussian Splatting" (Eq. gaussian-primitive);
rotation matrix of an unnormalised quaternion from the appendix "Bound on the
rotation R".  Readings taken where the paper is silent or garbled:

* Sigma = R diag(s)^2 R^T.  The paper prints R^T S^T S R, but its rotation
  derivation composes R' = R dR with dR = R^-1 R', which is the R S^2 R^T
  form; the two differ only by conjugating the quaternion.
* Raw parameters are stored: log-scale, quaternion (unnormalised), opacity
  logit and SH coefficients; s = exp(log-scale), alpha = sigmoid(logit).
* Colour: real spherical harmonics up to degree 3 evaluated at the unit
  direction from the camera centre to the mean, plus 0.5, clamped at zero.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64

# Real spherical-harmonic normalisation constants, from their closed forms.
SH_C0 = 0.5 * math.sqrt(1.0 / math.pi)
_K1 = math.sqrt(3.0 / (4.0 * math.pi))
_K2a = 0.5 * math.sqrt(15.0 / math.pi)
_K2b = 0.25 * math.sqrt(5.0 / math.pi)
_K2c = 0.25 * math.sqrt(15.0 / math.pi)
_K3a = 0.25 * math.sqrt(35.0 / (2.0 * math.pi))
_K3b = 0.5 * math.sqrt(105.0 / math.pi)
_K3c = 0.25 * math.sqrt(21.0 / (2.0 * math.pi))
_K3d = 0.25 * math.sqrt(7.0 / math.pi)
_K3e = 0.25 * math.sqrt(105.0 / math.pi)


def n_coeffs(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def n_params(sh_degree: int) -> int:
    return 11 + 3 * n_coeffs(sh_degree)


def split(x: torch.Tensor, sh_degree: int) -> dict:
    """Views of the raw parameter rows of ``x`` (shape [P, N])."""
    k = n_coeffs(sh_degree)
    n = x.shape[1]
    return dict(
        mu=x[0:3].T,
        log_s=x[3:6].T,
        quat=x[6:10].T,  # (q_x, q_y, q_z, q_w)
        logit=x[10],
        sh=x[11:11 + 3 * k].T.reshape(n, k, 3),
    )


def rotation_unnormalised(q: torch.Tensor) -> torch.Tensor:
    """R~(q) of the appendix: homogeneous quadratic in q, R = R~ / |q|^2."""
    qx, qy, qz, qw = q.unbind(-1)
    r2 = qx * qx + qy * qy + qz * qz + qw * qw
    rows = [
        [r2 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)],
        [2 * (qx * qy + qw * qz), r2 - 2 * (qz * qz + qx * qx), 2 * (qy * qz - qw * qx)],
        [2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), r2 - 2 * (qx * qx + qy * qy)],
    ]
    return torch.stack([torch.stack(r, -1) for r in rows], -2)


def rotation(q: torch.Tensor) -> torch.Tensor:
    r2 = (q * q).sum(-1)
    return rotation_unnormalised(q) / r2[..., None, None]


def covariance(log_s: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """Sigma = R diag(s^2) R^T with s = exp(log_s)."""
    R = rotation(q)
    M = R * torch.exp(log_s)[..., None, :]
    return M @ M.transpose(-1, -2)


def sh_basis(d: torch.Tensor, sh_degree: int) -> torch.Tensor:
    """Real SH basis values Y_k(d) for unit directions d [..., 3] -> [..., K]."""
    x, y, z = d.unbind(-1)
    out = [torch.full_like(x, SH_C0)]
    if sh_degree >= 1:
        out += [-_K1 * y, _K1 * z, -_K1 * x]
    if sh_degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [_K2a * x * y, -_K2a * y * z, _K2b * (2 * zz - xx - yy), -_K2a * x * z, _K2c * (xx - yy)]
    if sh_degree >= 3:
        out += [
            -_K3a * y * (3 * xx - yy),
            _K3b * x * y * z,
            -_K3c * y * (4 * zz - xx - yy),
            _K3d * z * (2 * zz - 3 * xx - 3 * yy),
            -_K3c * x * (4 * zz - xx - yy),
            _K3e * z * (xx - yy),
            -_K3a * x * (xx - 3 * yy),
        ]
    return torch.stack(out, -1)


def colour(sh: torch.Tensor, mu: torch.Tensor, cam_centre: torch.Tensor, sh_degree: int) -> torch.Tensor:
    """View-dependent RGB: sum_k f_k Y_k(dir) + 0.5, clamped at 0 (zero gradient when clamped)."""
    d = mu - cam_centre[None, :]
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    Y = sh_basis(d, sh_degree)
    rgb = (Y[..., None] * sh).sum(-2) + 0.5
    return torch.clamp(rgb, min=0.0)


def activations(x: torch.Tensor, sh_degree: int) -> dict:
    p = split(x, sh_degree)
    return dict(
        mu=p["mu"],
        s=torch.exp(p["log_s"]),
        R=rotation(p["quat"]),
        alpha=torch.sigmoid(p["logit"]),
        sh=p["sh"],
        quat=p["quat"],
    )
