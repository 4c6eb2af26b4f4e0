"""Pins of the oracle's Gaussian primitive: rotation, covariance and SH colour."""
import math

import numpy as np
import torch

from oracle import gaussians as G


def test_rotation_is_orthonormal_for_unnormalised_quaternions():
    rng = np.random.default_rng(0)
    q = torch.tensor(rng.normal(size=(64, 4)) * rng.uniform(0.1, 5.0, size=(64, 1)))
    R = G.rotation(q)
    eye = torch.eye(3, dtype=torch.float64).expand(64, 3, 3)
    assert torch.allclose(R @ R.transpose(-1, -2), eye, atol=1e-14)
    assert torch.allclose(torch.linalg.det(R), torch.ones(64, dtype=torch.float64), atol=1e-14)
    # scale invariance: R(c q) = R(q)
    assert torch.allclose(G.rotation(3.7 * q), R, atol=1e-14)


def test_rotation_about_z_matches_textbook():
    th = 0.7
    q = torch.tensor([0.0, 0.0, math.sin(th / 2), math.cos(th / 2)], dtype=torch.float64)
    R = G.rotation(q)
    want = torch.tensor([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0, 0, 1.0]],
                        dtype=torch.float64)
    assert torch.allclose(R, want, atol=1e-15)
    # rotating e_x by R gives (cos, sin, 0)
    assert torch.allclose(R @ torch.tensor([1.0, 0, 0], dtype=torch.float64),
                          torch.tensor([math.cos(th), math.sin(th), 0.0], dtype=torch.float64))


def test_covariance_eigen_decomposition():
    rng = np.random.default_rng(1)
    ls = torch.tensor(rng.normal(-2, 0.5, size=(16, 3)))
    q = torch.tensor(rng.normal(size=(16, 4)))
    S = G.covariance(ls, q)
    R = G.rotation(q)
    ev = torch.linalg.eigvalsh(S)
    want = torch.sort(torch.exp(2 * ls), dim=-1).values
    assert torch.allclose(ev, want, rtol=1e-12)
    # columns of R are the principal axes: S R e_k = s_k^2 R e_k
    for k in range(3):
        axis = R[:, :, k]
        assert torch.allclose((S @ axis[..., None])[..., 0], torch.exp(2 * ls[:, k])[:, None] * axis, atol=1e-14)


def _sphere_quadrature(n_theta=64, n_phi=128):
    # Gauss-Legendre in cos(theta) times uniform in phi is exact for these polynomials
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).reshape(-1)
    return torch.tensor(d), torch.tensor(wt)


def test_sh_basis_is_orthonormal_on_the_sphere():
    d, w = _sphere_quadrature()
    Y = G.sh_basis(d, 3)  # [Q, 16]
    gram = (Y * w[:, None]).T @ Y
    assert torch.allclose(gram, torch.eye(16, dtype=torch.float64), atol=1e-12)


def test_sh_degree1_is_linear_in_direction():
    d, _ = _sphere_quadrature(8, 8)
    Y = G.sh_basis(d, 1)
    k = math.sqrt(3 / (4 * math.pi))
    assert torch.allclose(Y[:, 1:4].abs(), k * torch.stack([d[:, 1], d[:, 2], d[:, 0]], 1).abs(), atol=1e-15)


def test_degree0_colour_and_clamp():
    sh = torch.tensor([[[1.0, -3.0, 0.2]]], dtype=torch.float64)
    mu = torch.tensor([[0.3, 0.1, -0.2]], dtype=torch.float64)
    c = G.colour(sh, mu, torch.zeros(3, dtype=torch.float64), 0)
    want = torch.tensor([[G.SH_C0 * 1.0 + 0.5, max(G.SH_C0 * -3.0 + 0.5, 0.0), G.SH_C0 * 0.2 + 0.5]],
                        dtype=torch.float64)
    assert torch.allclose(c, want, atol=1e-15)
    assert abs(G.SH_C0 - 0.28209479177387814) < 1e-16


def test_split_layout():
    x = torch.arange(14 * 2, dtype=torch.float64).reshape(14, 2)
    p = G.split(x, 0)
    assert p["mu"][1].tolist() == [1.0, 3.0, 5.0]
    assert p["quat"][0].tolist() == [12.0, 14.0, 16.0, 18.0]
    assert float(p["logit"][1]) == 21.0
    assert p["sh"][0, 0].tolist() == [22.0, 24.0, 26.0]
    assert G.n_params(3) == 59
