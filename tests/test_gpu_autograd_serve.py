"""GPU tests of the two adopted patterns: the torch.autograd.Function wrapper
(backward and forward mode checked against the FP64 oracle and its central
finite differences; the torch.func Gauss-Newton product checked against
gs3_hvp_diag) and the continuous-batching server (a scene fitted alone and in
a mix of concurrent fits ends bitwise identical)."""
import sys

import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import binning as B
from oracle import method as Mth
from oracle import render as R
from tests.helpers import group_errors, offset_targets, rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def crop():
    """The 500 Gaussians nearest the origin of the object-scale scene, SH 3,
    rendered at 800x800 from two cameras."""
    sc = syn.config2_scene()
    d = np.linalg.norm(sc.init[0:3].T, axis=1)
    keep = np.argsort(d)[:500]
    x = sc.init[:, keep].copy()
    x[14:] = sc.gt[14:, keep]
    x[6:10] = sc.gt[6:10, keep]  # non-trivial rotations
    x[3:6] = sc.gt[3:6, keep]
    cams = [sc.cameras[0], sc.cameras[17]]
    return x.astype(np.float32), cams


def _scene(x, cams, targets=None, lam=0.2):
    from paper_2602_00395_amd import Scene

    tg = targets or [np.zeros((c.height, c.width, 3), np.float32) for c in cams]
    return Scene(torch.tensor(x, device=DEV), [torch.tensor(t, device=DEV) for t in tg], cams, 3, lam=lam)


def test_autograd_backward_matches_oracle_and_fd(crop):
    from paper_2602_00395_amd.autograd import rasterize

    x, cams = crop
    s = _scene(x, cams)
    cam = cams[1]
    rng = np.random.default_rng(1)
    w = rng.normal(size=(cam.height, cam.width, 3))
    xp = torch.tensor(x, device=DEV, requires_grad=True)
    img = rasterize(xp, s, 1)
    (img * torch.tensor(w, dtype=torch.float32, device=DEV)).sum().backward()
    got = xp.grad.cpu().numpy()
    bins = B.bin_view(x, cam)
    f = lambda xx: (R.render(xx, cam, 3, bins) * torch.tensor(w)).sum()  # noqa: E731
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    f(xt).backward()
    want = xt.grad.numpy()
    errs = group_errors(got, want, 59)
    say("autograd backward vs oracle", errs)
    assert all(e <= TOL for e in errs.values()), errs
    # central finite differences of the FP64 oracle along random directions
    # (bins fixed; directions with a flipped blend decision are skipped)
    n_ok = 0
    with torch.no_grad():
        _, aux0 = R.render(torch.tensor(x, dtype=torch.float64), cam, 3, bins, return_aux=True)
        for k in range(6):
            v = rng.normal(size=x.shape) * 1e-2
            h = 1e-4
            fp, ap = R.render(torch.tensor(x + h * v), cam, 3, bins, return_aux=True)
            fm, am = R.render(torch.tensor(x - h * v), cam, 3, bins, return_aux=True)
            if not (R.decisions_equal(ap["decisions"], aux0["decisions"])
                    and R.decisions_equal(am["decisions"], aux0["decisions"])):
                continue
            fd = float(((fp - fm) * torch.tensor(w)).sum()) / (2 * h)
            an = float((got.astype(np.float64) * v).sum())
            say("  fd", fd, "autograd", an)
            assert abs(fd - an) <= 1e-4 * float(np.abs(got.astype(np.float64) * v).sum())
            n_ok += 1
    assert n_ok >= 3
    s.close()


def test_autograd_forward_mode_matches_oracle(crop):
    from paper_2602_00395_amd.autograd import rasterize

    x, cams = crop
    s = _scene(x, cams)
    rng = np.random.default_rng(2)
    tan = rng.normal(size=x.shape).astype(np.float32)
    import torch.autograd.forward_ad as fwAD

    with fwAD.dual_level():
        dual = fwAD.make_dual(torch.tensor(x, device=DEV), torch.tensor(tan, device=DEV))
        img, jt = fwAD.unpack_dual(rasterize(dual, s, 0))
    bins = B.bin_view(x, cams[0])
    _, want = torch.func.jvp(lambda xx: R.render(xx, cams[0], 3, bins), (torch.tensor(x, dtype=torch.float64),),
                             (torch.tensor(tan, dtype=torch.float64),))
    e = rel_l2(jt.cpu().numpy(), want.numpy())
    say("autograd jvp vs oracle", e)
    assert e <= TOL
    s.close()


def test_torch_func_gauss_newton_product_equals_hvp_diag(crop):
    """u = J z by torch forward-mode AD, y = GN-weighted L1 cotangent in torch,
    h = J^T y by reverse mode; s z . h must equal gs3_hvp_diag with the same probe."""
    import torch.autograd.forward_ad as fwAD

    from paper_2602_00395_amd.autograd import rasterize

    x, cams = crop
    targets = offset_targets(x, cams, 3, seed=9)
    s = _scene(x, cams, targets, lam=0.0)
    seed, j = 77, 1
    z = torch.tensor(Mth.probe(seed, 0, *x.shape), dtype=torch.float32, device=DEV)
    xp = torch.tensor(x, device=DEV)
    with fwAD.dual_level():
        img, u = fwAD.unpack_dual(rasterize(fwAD.make_dual(xp, z), s, j))
    r = img - torch.tensor(targets[j], device=DEV)
    sg = torch.sign(r)
    y = sg * (sg * u) / (4.0 * torch.clamp(r.abs(), min=1e-6))
    xg = xp.clone().requires_grad_(True)
    (h,) = torch.autograd.grad(rasterize(xg, s, j), xg, grad_outputs=y)
    m = 6 * sum(c.height * c.width for c in cams)
    d_torch = (z * h * (len(cams) / m)).cpu().numpy()
    d_lib = s.hvp_diag([j], 1, seed).cpu().numpy()
    errs = group_errors(d_lib, d_torch, 59)
    say("hvp_diag vs torch.func GN product", errs)
    assert all(e <= TOL for e in errs.values()), errs
    s.close()


def _fit_requests(k, iters):
    from paper_2602_00395_amd import Scene
    from paper_2602_00395_amd.serve import FitRequest

    reqs = []
    for i in range(k):
        sc = syn.tiny_scene(100 + i, n=300 + 200 * i, sh_degree=i % 2, width=96, height=80, n_cams=9,
                            log_scale_mean=np.log(0.06))
        rng = np.random.default_rng(i)
        init = sc.gt.copy()
        init[0:3] += rng.normal(0, 0.03, size=init[0:3].shape).astype(np.float32)
        gt_t = torch.tensor(sc.gt, device=DEV)
        blank = [torch.zeros((c.height, c.width, 3), device=DEV) for c in sc.cameras]
        g = Scene(gt_t, blank, sc.cameras, sc.sh_degree, lam=0.2)
        targets = [g.render(jj).clone() for jj in range(len(sc.cameras))]
        torch.cuda.synchronize()
        g.close()
        mask = [jj % 8 != 0 for jj in range(len(sc.cameras))]

        def make(stream, init=init, targets=targets, sc=sc, mask=mask):
            return Scene(torch.tensor(init, device=DEV), targets, sc.cameras, sc.sh_degree, lam=0.2,
                         train_mask=mask, stream=stream)

        reqs.append(FitRequest(rid=i, arrival_s=0.05 * i, n=sc.n, sh_degree=sc.sh_degree, make_scene=make,
                               train_ids=sc.train_ids(), test_ids=sc.test_ids(), target_psnr=1e9,
                               max_iters=iters, check_every=iters // 2, bytes_needed=1, seed=1234 + i))
    return reqs


def test_served_fits_are_identical_alone_and_in_the_mix():
    from paper_2602_00395_amd.serve import Server

    reqs = _fit_requests(3, 40)
    alone = {}
    for r in reqs:
        st = Server(hbm_budget=10, max_active=1, keep_params=True).run([r])
        alone[r.rid] = st.results[0].final_params
    st = Server(hbm_budget=10, max_active=3, keep_params=True).run(reqs)
    assert st.peak_bytes <= 10
    for res in st.results:
        say("request", res.rid, "iters", res.iters, "psnr", round(res.psnr, 3))
        assert res.iters == 40
        assert torch.equal(res.final_params, alone[res.rid]), res.rid
