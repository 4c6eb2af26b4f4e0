"""Continuous-batching scene-fit server on one GPU.

Requests (a scene to fit to a PSNR target) arrive over time.  A request is
admitted as soon as its device footprint (gs3_scene_bytes: resident state plus
per-view scratch) fits in the free part of an HBM budget and an active slot is
free; it then runs Algorithm 1 iterations on its own HIP stream from its own
host thread, so the work of all active scenes overlaps on the device (the
ctypes calls release the GIL).  Every `check_every` iterations it measures the
held-out PSNR; it completes when the target is reached or its iteration cap is
hit, releases its memory and frees its slot, and the next queued request is
admitted.  Reported: per-request time-to-fit (arrival to completion, so
queueing counts), p50/p99, and aggregate Gaussian-updates/s.

The kernels are deterministic (no float atomics) and every request draws its
mini-batches from its own seeded generator, so a scene's trajectory does not
depend on what else is running: results alone and in the mix are identical.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable

import numpy as np


@dataclass
class FitRequest:
    rid: int
    arrival_s: float
    n: int
    sh_degree: int
    make_scene: Callable  # (stream) -> Scene
    train_ids: list
    test_ids: list
    target_psnr: float
    max_iters: int = 3000
    check_every: int = 100
    bytes_needed: int = 0
    seed: int = 0


@dataclass
class FitResult:
    rid: int
    arrival_s: float
    start_s: float
    end_s: float
    iters: int
    psnr: float
    reached: bool
    n: int
    final_params: object = None
    error: str | None = None  # set when the fit raised; such a request counts as failed

    @property
    def latency_s(self) -> float:
        return self.end_s - self.arrival_s


@dataclass
class ServerStats:
    results: list = field(default_factory=list)
    peak_bytes: int = 0
    budget: int = 0
    wall_s: float = 0.0

    @property
    def failed(self) -> list:
        return [r for r in self.results if r.error is not None]

    def percentile(self, q: float) -> float:
        """Latency percentile over every request; a failed request counts as
        never finishing (+inf), so failures can only raise the figure (with
        failures present the percentile takes the next sample up instead of
        interpolating, which would mix inf into finite values)."""
        lat = np.array([r.latency_s if r.error is None else np.inf for r in self.results])
        if not len(lat):
            return float("nan")
        return float(np.percentile(lat, q, method="higher" if np.isinf(lat).any() else "linear"))

    def gaussian_updates_per_s(self) -> float:
        tot = sum(r.iters * r.n for r in self.results)
        return tot / self.wall_s if self.wall_s > 0 else 0.0


def run_fit(req: FitRequest, stream, keep_params: bool, trainer_factory) -> tuple:
    """Fit one request on `stream`; returns (iters, psnr, reached, params)."""
    import torch

    with torch.cuda.stream(stream):
        scene = req.make_scene(stream)
        tr = trainer_factory(scene, req)
        it, psnr, reached = 0, float("-inf"), False
        while it < req.max_iters:
            n = min(req.check_every, req.max_iters - it)
            for _ in range(n):
                tr.step()
            it += n
            psnr = float(np.mean([scene.psnr(j) for j in req.test_ids]))
            if psnr >= req.target_psnr:
                reached = True
                break
        params = scene.params().cpu() if keep_params else None
        stream.synchronize()
        scene.close()
    return it, psnr, reached, params


class Server:
    """Admission by HBM budget, one stream and host thread per active scene."""

    def __init__(self, hbm_budget: int, max_active: int = 8, keep_params: bool = False,
                 trainer_factory=None, clock=time.perf_counter, stream_factory=None):
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.keep_params = keep_params
        self.trainer_factory = trainer_factory or default_trainer
        self.clock = clock
        self.stream_factory = stream_factory or _torch_stream
        self._lock = threading.Lock()
        self._cv = threading.Condition(self._lock)
        self._in_use = 0
        self._active = 0

    def run(self, requests: list, fit_fn=run_fit) -> ServerStats:
        """Serve `requests` (arrival_s relative to the start); returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        for r in reqs:
            if r.bytes_needed > self.budget:
                raise ValueError(f"request {r.rid} needs {r.bytes_needed} B, more than the whole budget")
        stats = ServerStats(budget=self.budget)
        t0 = self.clock()
        threads = []
        queue = list(reqs)

        def worker(req: FitRequest, start_s: float):
            try:
                stream = self.stream_factory()
                it, psnr, reached, params = fit_fn(req, stream, self.keep_params, self.trainer_factory)
                end = self.clock() - t0
                res = FitResult(req.rid, req.arrival_s, start_s, end, it, psnr, reached, req.n, params)
            except Exception as e:  # recorded, not dropped: the stats count it as a failure
                res = FitResult(req.rid, req.arrival_s, start_s, self.clock() - t0, 0, float("nan"), False, req.n,
                                None, error=f"{type(e).__name__}: {e}")
            finally:
                with self._cv:
                    self._in_use -= req.bytes_needed
                    self._active -= 1
                    self._cv.notify_all()
            with self._cv:
                stats.results.append(res)

        while queue:
            req = queue[0]
            with self._cv:
                while True:
                    now = self.clock() - t0
                    arrived = now >= req.arrival_s
                    fits = self._in_use + req.bytes_needed <= self.budget and self._active < self.max_active
                    if arrived and fits:
                        break
                    wait = max(req.arrival_s - now, 0.0) if not arrived else None
                    self._cv.wait(timeout=wait if wait is not None else 0.05)
                self._in_use += req.bytes_needed
                self._active += 1
                stats.peak_bytes = max(stats.peak_bytes, self._in_use)
                start = self.clock() - t0
            queue.pop(0)
            th = threading.Thread(target=worker, args=(req, start), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        stats.wall_s = self.clock() - t0
        stats.results.sort(key=lambda r: r.rid)
        return stats


def _torch_stream():
    import torch

    return torch.cuda.Stream()


def default_trainer(scene, req: FitRequest):
    from .trainer import TRConfig, TRTrainer

    return TRTrainer(scene, req.train_ids, TRConfig(budget=req.max_iters, seed=req.seed, probe_seed=req.seed + 1))
