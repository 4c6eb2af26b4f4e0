"""Binning parity at the large single-GPU workloads: one view of the city
workload (6M Gaussians, 1920x1080) and one of the unbounded workload (1M
Gaussians, 1600x1000).  Tile keys, the sorted Gaussian order and per-tile
ranges bit-exact against the oracle's float32 binning.  These sizes run the
multi-round paths of the scans (more than 256 scan blocks of Gaussians, more
than 2,048 radix blocks of pairs) that smaller views never reach."""
import sys

import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import binning as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bin_parity(sc, cam_ids, tag):
    from paper_2602_00395_amd import Scene

    cams = [sc.cameras[j] for j in cam_ids]
    x = sc.init.astype(np.float32)
    zeros = [torch.zeros((c.height, c.width, 3), device=DEV) for c in cams]
    s = Scene(torch.tensor(x, device=DEV), zeros, cams, sc.sh_degree, lam=0.2)
    try:
        for k, j in enumerate(cam_ids):
            say(tag, "camera", j, "binning on the GPU")
            keys, gids, ranges = s.bin(k)
            k_gpu = keys.cpu().numpy().view(np.uint64)
            g_gpu = gids.cpu().numpy().astype(np.int64)
            r_gpu = ranges.cpu().numpy().astype(np.int64)
            ob = B.bin_view(x, cams[k])
            say(tag, "camera", j, "pairs", len(ob.keys), "visible", int(ob.visible.sum()))
            assert len(ob.keys) > 2048 * 1024, len(ob.keys)  # more than one round of radix blocks
            assert len(k_gpu) == len(ob.keys)
            assert np.array_equal(k_gpu, ob.keys), tag
            assert np.array_equal(g_gpu, ob.gids), tag
            empty = ob.ranges[:, 0] == ob.ranges[:, 1]
            assert np.array_equal(r_gpu[~empty], ob.ranges[~empty]), tag
            assert np.all(r_gpu[empty, 0] == r_gpu[empty, 1]), tag
    finally:
        s.close()


def test_binning_bit_exact_city_view():
    sc = syn.config4_scene()
    assert sc.n > 256 * 4096  # more Gaussians than one round of the scan's top level
    _bin_parity(sc, [0, 517], "city")


def test_binning_bit_exact_unbounded_view():
    sc = syn.config3_scene()
    _bin_parity(sc, [0, 101], "unbounded")
