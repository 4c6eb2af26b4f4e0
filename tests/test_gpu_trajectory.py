"""Algorithm 1 end to end: the trainer's fused iterations (gs3_tr_iteration)
against the oracle's plain loop (run_tr) on the plain CPU-sized workload
(2,000 Gaussians, SH degree 0, eight 64x64 views, 10 iterations, 4
Hutchinson probes), iteration by iteration: parameters, gradient EMA and
Hessian-diagonal EMA per parameter group at relative L2 <= 1e-4, with the
largest elementwise error and the float32-vs-float64 decision flips of the
views used reported beside them."""
import sys

import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import method as Mth
from tests.helpers import group_errors, group_max_abs, offset_targets, view_flips

pytestmark = pytest.mark.gpu
TOL = 1e-4
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("T,l,nu,s1,s2", [(10, 10, 4, 1, 1), (6, 2, 2, 2, 2)])
def test_trajectory_matches_oracle_algorithm1(T, l, nu, s1, s2):
    from paper_2602_00395_amd import Scene
    from paper_2602_00395_amd.trainer import TRConfig, TRTrainer

    sc = syn.config1_scene()
    x1 = sc.init.astype(np.float32)
    targets = offset_targets(x1, sc.cameras, 0, seed=4001)
    s = Scene(torch.tensor(x1, device=DEV), [torch.tensor(t, device=DEV) for t in targets], sc.cameras, 0, lam=0.2)
    cfg = TRConfig(l=l, nu=nu, s1=s1, s2=s2, budget=T, seed=4001, probe_seed=5001)
    tr = TRTrainer(s, range(len(sc.cameras)), cfg)
    P, N = x1.shape
    got, picks = [], []
    for _ in range(T):
        tr.step()
        t, S1, S2, seed, eps = tr.last
        picks.append((S1, S2, seed, eps))
        xs, gh, dh = (torch.empty((P, N), device=DEV) for _ in range(3))
        s.export(x=xs, ghat=gh, dhat=dh)
        got.append(tuple(v.cpu().numpy() for v in (xs, gh, dh)))
    s.close()
    say("trajectory T", T, "l", l, "nu", nu, "picks", [(p[0], p[1]) for p in picks])
    prob = Mth.Problem(sc.cameras, targets, 0, lam=0.2)
    S1s = [p[0] for p in picks]
    S2s = [p[1] for p in picks]
    seeds = [p[2] for p in picks]
    _, _, _, log = Mth.run_tr_problem(x1, prob, T, S1s, S2s, nu, seeds, l=l)
    x_prev = x1.astype(np.float64)
    for r, (gx, gg, gd), p in zip(log, got, picks):
        assert r["hutch"] == bool(p[1]) and abs(r["eps"] - p[3]) <= 1e-12 * r["eps"]
        ex, eg, ed = group_errors(gx, r["x"], P), group_errors(gg, r["ghat"], P), group_errors(gd, r["Dhat"], P)
        mg, md = group_max_abs(gg, r["ghat"], P), group_max_abs(gd, r["Dhat"], P)
        flips = view_flips(x_prev, sc.cameras, sorted(set(p[0]) | set(p[1])), 0)
        x_prev = r["x"]
        say(f"  t={r['t']} eps={r['eps']:.3g} clipped={r['clipped']:.3f} nonpos={r['nonpos']:.3f}",
            "x", max(ex.values()), "ghat", max(eg.values()), "max-abs", max(mg.values()),
            "Dhat", max(ed.values()), "max-abs", max(md.values()), "flips", flips)
        for name, e in (("x", ex), ("ghat", eg), ("Dhat", ed)):
            assert all(v <= TOL for v in e.values()), (r["t"], name, e)
