"""Seeded scene, camera and request generators.

Raw parameters are stored structure-of-arrays, ``float32[P][N]`` with
P = 11 + 3K and K = (d+1)^2 spherical-harmonic coefficients per colour
channel.  Row order: mu_x, mu_y, mu_z, log-scale 0..2, quaternion
(q_x, q_y, q_z, q_w), opacity logit, then SH coefficient k, channel c at row
11 + 3k + c.  Cameras are OpenCV pinholes (x right, y down, z forward) given
as a world-to-camera rotation ``R`` and translation ``t``.

Seed convention: ground truth 1000+c, init noise 2000+c, cameras 3000+c,
mini-batches 4000+c, probes 5000+c, where c is the workload number.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Half-width of the uniform draw of DC coefficients that spans base colours
# in [0, 1]: the DC basis value of real SH is 1/(2 sqrt(pi)).
_DC_HALF_RANGE = 0.5 * 2.0 * math.sqrt(math.pi)


def n_params(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # float32[3,3], world -> camera
    t: np.ndarray  # float32[3]

    def centre(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclass
class SceneInputs:
    name: str
    sh_degree: int
    gt: np.ndarray  # float32[P][N]
    init: np.ndarray  # float32[P][N]
    cameras: list = field(default_factory=list)
    test_every: int = 8  # cameras with index % test_every == 0 are held out

    @property
    def n(self) -> int:
        return self.gt.shape[1]

    @property
    def p(self) -> int:
        return self.gt.shape[0]

    def train_ids(self):
        return [i for i in range(len(self.cameras)) if i % self.test_every != 0]

    def test_ids(self):
        return [i for i in range(len(self.cameras)) if i % self.test_every == 0]


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """World-to-camera (R, t) for a camera at ``eye`` looking at ``target``."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, np.float64)
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float64)
    t = -R @ eye
    return R.astype(np.float32), t.astype(np.float32)


def make_camera(eye, width, height, fov_x_deg=60.0, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    R, t = look_at(eye, target, up)
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(int(width), int(height), float(np.float32(f)), float(np.float32(f)),
                  float(width) / 2.0, float(height) / 2.0, R, t)


def fibonacci_sphere(n: int, radius: float, hemisphere: bool = False) -> np.ndarray:
    """Golden-angle spiral points; with ``hemisphere`` only z >= 0 is covered."""
    i = np.arange(n, dtype=np.float64) + 0.5
    if hemisphere:
        z = 1.0 - i / n
    else:
        z = 1.0 - 2.0 * i / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = math.pi * (3.0 - math.sqrt(5.0)) * i
    return radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def _unit_quaternions(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _assemble(mu, log_s, quat, logit_a, f):
    """Pack per-Gaussian arrays into the float32[P][N] layout."""
    n = mu.shape[0]
    k = f.shape[1]
    x = np.empty((11 + 3 * k, n), np.float32)
    x[0:3] = mu.T
    x[3:6] = log_s.T
    x[6:10] = quat.T
    x[10] = logit_a
    x[11:] = f.reshape(n, 3 * k).T
    return x


def random_scene(rng, n, sh_degree, mu_lo=-1.0, mu_hi=1.0, log_scale_mean=math.log(0.05),
                 log_scale_std=0.3, sh_rest_std=0.2):
    """Ground-truth draw shared by several workloads."""
    k = (sh_degree + 1) ** 2
    mu = rng.uniform(mu_lo, mu_hi, size=(n, 3))
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quat = _unit_quaternions(rng, n)
    logit_a = rng.normal(0.0, 1.0, size=n)
    f = np.zeros((n, k, 3))
    f[:, 0, :] = rng.uniform(-_DC_HALF_RANGE, _DC_HALF_RANGE, size=(n, 3))
    if k > 1:
        f[:, 1:, :] = rng.normal(0.0, sh_rest_std, size=(n, k - 1, 3))
    return _assemble(mu, log_s, quat, logit_a, f)


def config1_scene() -> SceneInputs:
    """2,000 Gaussians, SH degree 0, eight 64x64 cameras on a radius-4 sphere."""
    c = 1
    gt = random_scene(np.random.default_rng(1000 + c), 2000, 0)
    noise = np.random.default_rng(2000 + c).normal(0.0, 0.05, size=gt.shape)
    init = (gt + noise).astype(np.float32)
    cams = [make_camera(e, 64, 64) for e in fibonacci_sphere(8, 4.0)]
    return SceneInputs("plain-2k-sh0-8x64", 0, gt, init, cams)


def _knn_mean_dist(points, k=3):
    from scipy.spatial import cKDTree

    tree = cKDTree(points)
    d, _ = tree.query(points, k=k + 1)
    return np.maximum(d[:, 1:].mean(axis=1), 1e-7)


def _object_init(rng, gt, sh_degree, mu_noise=0.05, dc_noise=0.05):
    """Init from noisy ground-truth means: isotropic scales, identity rotation."""
    n = gt.shape[1]
    k = (sh_degree + 1) ** 2
    mu = gt[0:3].T.astype(np.float64) + rng.normal(0.0, mu_noise, size=(n, 3))
    log_s = np.repeat(np.log(_knn_mean_dist(mu))[:, None], 3, axis=1)
    quat = np.tile(np.array([0.0, 0.0, 0.0, 1.0]), (n, 1))
    logit_a = np.full(n, math.log(0.1 / 0.9))
    f = np.zeros((n, k, 3))
    f[:, 0, :] = gt[11:14].T + rng.normal(0.0, dc_noise, size=(n, 3))
    return _assemble(mu, log_s, quat, logit_a, f)


def config2_scene(n=100_000, n_cams=48, res=800) -> SceneInputs:
    """Object scale: 100k Gaussians, SH degree 3, 48 cameras at 800x800 on a hemisphere."""
    c = 2
    gt = random_scene(np.random.default_rng(1000 + c), n, 3)
    init = _object_init(np.random.default_rng(2000 + c), gt, 3)
    cams = [make_camera(e, res, res) for e in fibonacci_sphere(n_cams, 4.0, hemisphere=True)]
    return SceneInputs(f"object-{n // 1000}k-sh3-{n_cams}x{res}", 3, gt, init, cams)


def config3_scene(n=1_000_000, n_cams=200) -> SceneInputs:
    """Unbounded outdoor shape: a 20-component mixture foreground plus a far shell."""
    c = 3
    rng = np.random.default_rng(1000 + c)
    n_fg = int(round(0.7 * n))
    n_bg = n - n_fg
    centres = rng.normal(size=(20, 3))
    centres *= (2.0 * rng.uniform(0, 1, size=(20, 1)) ** (1.0 / 3.0)) / np.linalg.norm(centres, axis=1, keepdims=True)
    sig = rng.uniform(0.1, 0.4, size=20)
    comp = rng.integers(0, 20, size=n_fg)
    fg = centres[comp] + rng.normal(size=(n_fg, 3)) * sig[comp, None]
    dirs = rng.normal(size=(n_bg, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    bg = dirs * rng.uniform(20.0, 50.0, size=(n_bg, 1))
    mu = np.concatenate([fg, bg])
    log_s = np.concatenate([rng.normal(math.log(0.05), 0.3, size=(n_fg, 3)),
                            rng.normal(math.log(0.5), 0.3, size=(n_bg, 3))])
    k = 16
    f = np.zeros((n, k, 3))
    f[:, 0, :] = rng.uniform(-_DC_HALF_RANGE, _DC_HALF_RANGE, size=(n, 3))
    f[:, 1:, :] = rng.normal(0.0, 0.2, size=(n, k - 1, 3))
    gt = _assemble(mu, log_s, _unit_quaternions(rng, n), rng.normal(0.0, 1.0, size=n), f)
    init = _object_init(np.random.default_rng(2000 + c), gt, 3)
    crng = np.random.default_rng(3000 + c)
    th = 2.0 * math.pi * np.arange(n_cams) / n_cams
    eyes = np.stack([6.0 * np.cos(th), 4.0 * np.sin(th), np.ones(n_cams)], axis=1)
    eyes += crng.normal(0.0, 0.2, size=eyes.shape)
    cams = [make_camera(e, 1600, 1000) for e in eyes]
    return SceneInputs(f"unbounded-{n // 1000}k-sh3-{n_cams}x1600x1000", 3, gt, init, cams)


def config4_scene(n=6_000_000, n_cams=1000) -> SceneInputs:
    """City-block grid: Gaussians over a 200x200 square, cameras on straight tracks."""
    c = 4
    rng = np.random.default_rng(1000 + c)
    xy = rng.uniform(-100.0, 100.0, size=(n, 2))
    z = rng.lognormal(math.log(3.0), 1.0, size=(n, 1))
    mu = np.concatenate([xy, z], axis=1)
    log_s = rng.normal(math.log(0.3), 0.3, size=(n, 3))
    k = 16
    f = np.zeros((n, k, 3), np.float32)
    f[:, 0, :] = rng.uniform(-_DC_HALF_RANGE, _DC_HALF_RANGE, size=(n, 3))
    f[:, 1:, :] = rng.normal(0.0, 0.2, size=(n, k - 1, 3))
    gt = _assemble(mu, log_s, _unit_quaternions(rng, n), rng.normal(0.0, 1.0, size=n), f)
    init = gt.copy()
    init[0:3] += np.random.default_rng(2000 + c).normal(0.0, 0.05, size=(3, n)).astype(np.float32)
    per_track = max(1, n_cams // 20)
    cams = []
    pitch = math.radians(30.0)
    for track in range(20):
        along_x = track < 10
        off = -90.0 + 20.0 * (track % 10)
        for j in range(per_track):
            s = -100.0 + 200.0 * (j + 0.5) / per_track
            eye = np.array([s, off, 30.0]) if along_x else np.array([off, s, 30.0])
            head = np.array([1.0, 0.0, 0.0]) if along_x else np.array([0.0, 1.0, 0.0])
            look = eye + head * math.cos(pitch) - np.array([0.0, 0.0, math.sin(pitch)])
            cams.append(make_camera(eye, 1920, 1080, target=look))
    return SceneInputs(f"city-{n // 1000}k-sh3-{len(cams)}x1920x1080", 3, gt, init, cams)


def serving_requests(n_req=64, rate=2.0, seed=5):
    """Poisson arrivals of scene-fit requests with log-uniform Gaussian counts."""
    rng = np.random.default_rng(6000 + seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    out = []
    for i in range(n_req):
        n = int(math.floor(math.exp(rng.uniform(math.log(1e4), math.log(5e5)))))
        out.append(dict(
            arrival_s=float(np.cumsum(gaps)[i]),
            n=n,
            n_cams=int(rng.integers(16, 129)),
            res=int(16 * rng.integers(16, 51)),
            sh_degree=int(rng.integers(0, 4)),
            seed=int(rng.integers(0, 2**31 - 1)),
        ))
    return out


def request_scene(req) -> SceneInputs:
    rng = np.random.default_rng(req["seed"])
    gt = random_scene(rng, req["n"], req["sh_degree"])
    init = _object_init(rng, gt, req["sh_degree"])
    cams = [make_camera(e, req["res"], req["res"]) for e in fibonacci_sphere(req["n_cams"], 4.0, hemisphere=True)]
    return SceneInputs(f"req-{req['n']}", req["sh_degree"], gt, init, cams)


def tiny_scene(seed, n=8, sh_degree=0, width=32, height=32, n_cams=2, spread=0.6,
               log_scale_mean=math.log(0.12), log_scale_std=0.2, dist=3.0):
    """A handful of well-resolved Gaussians in front of a few cameras (test scenes)."""
    rng = np.random.default_rng(seed)
    gt = random_scene(rng, n, sh_degree, -spread, spread, log_scale_mean, log_scale_std, 0.1)
    eyes = fibonacci_sphere(max(n_cams, 1), dist)
    if n_cams == 1:
        eyes = np.array([[0.0, -dist, 0.3]])
    cams = [make_camera(e, width, height) for e in eyes]
    return SceneInputs(f"tiny-{seed}", sh_degree, gt, gt.copy(), cams)
