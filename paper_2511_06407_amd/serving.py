"""Serving loop: sampling requests of mixed dimension arrive over time and are
run concurrently on the GPU with continuous admission.

A request is a latent-GP model (GP-logistic with an isotropic SE kernel, or
the multiple-kernel propensity model) and a number of RMHMC moves.  The
scheduler admits an arrived request as soon as (a) an executor slot is free
and (b) its device-memory footprint fits the HBM budget next to the requests
already running; it never reorders arrivals (FIFO, head-of-line blocking on
memory).  Chain state stays on the device for the request's lifetime.
Latency = completion time - arrival time.

The scheduler talks to an executor with three calls (start, done, release),
so its logic is tested on the CPU with a simulated executor; ``PoolExecutor``
drives the HIP worker pool.
"""
from __future__ import annotations

import dataclasses
import heapq
import math
import time
from typing import List, Optional

import numpy as np

from . import workloads as wl


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str          # "gp_logistic" or "mkl"
    D: int
    n_moves: int
    seed: int
    # filled by the scheduler
    admit_s: Optional[float] = None
    done_s: Optional[float] = None
    leapfrogs: int = 0
    accepted: int = 0

    @property
    def latency_s(self):
        return None if self.done_s is None else self.done_s - self.arrival_s


def make_requests(rate_per_s, duration_s, d_min=34, d_max=1038, moves=(200, 2000), seed=0):
    """Poisson arrivals; D log-uniform in [d_min, d_max]; model type fair coin."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t > duration_s:
            break
        kind = "gp_logistic" if rng.uniform() < 0.5 else "mkl"
        D = int(round(math.exp(rng.uniform(math.log(d_min), math.log(d_max)))))
        if kind == "mkl":
            D = max(D, 14 + 8)
        n_moves = int(rng.integers(moves[0], moves[1] + 1))
        out.append(Request(len(out), t, kind, D, n_moves, seed=len(out)))
    return out


def request_spec(req: Request):
    if req.kind == "gp_logistic":
        spec, _, _ = wl.gp_logistic_2d(req.D - 2, req.seed)
        eps = 0.01
    else:
        spec, _, _ = wl.propensity_mkl(req.D - 14, req.seed)
        # the posterior of the multiple-kernel model sharpens with N: the
        # step of the D = 1038 workload above 512 dimensions
        eps = 0.003 if req.D < 512 else 0.001
    return spec, eps


def footprint_bytes(N, P):
    """Device memory of one model plus its chain state (four per-point caches
    and the model scratch), as allocated by librmhmc."""
    D = N + P
    Dp = ((D + 63) // 64) * 64
    nn = N * N
    h1, h2 = (P + 1) // 2, P // 2
    ny = h1 * (h1 + 1) // 2 + h2 * (h2 + 1) // 2   # Y_lm products formed (pairs within a half)
    point = (2 + 4 * P + ny) * nn + 2 * Dp * Dp + (2 * P * P + 8) * N + P ** 3
    # generated second derivatives of K: at most one per pair (l <= m), 64 at a time
    model_scratch = 3 * nn + 6 * Dp * Dp + min(P * (P + 1) // 2, 64) * nn
    return 8 * (4 * point + model_scratch)


def request_footprint(req: Request):
    P = 2 if req.kind == "gp_logistic" else 14
    return footprint_bytes(req.D - P, P)


class Scheduler:
    def __init__(self, executor, hbm_budget_bytes, n_slots, clock=time.perf_counter):
        self.ex = executor
        self.budget = hbm_budget_bytes
        self.n_slots = n_slots
        self.clock = clock
        self.in_use = 0
        self.max_in_use = 0
        self.max_running = 0
        self.queue_depth = []      # (t, waiting, running)

    def run(self, requests: List[Request], poll_s=0.002):
        pending = sorted(requests, key=lambda r: r.arrival_s)
        for r in pending:
            if request_footprint(r) > self.budget:
                raise ValueError(f"request {r.rid} needs more memory than the whole budget")
        t0 = self.clock()
        running = {}
        i = 0
        waiting = []
        while i < len(pending) or waiting or running:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival_s <= now:
                waiting.append(pending[i])
                i += 1
            # continuous admission, FIFO
            while waiting and len(running) < self.n_slots:
                r = waiting[0]
                fp = request_footprint(r)
                if self.in_use + fp > self.budget:
                    break
                waiting.pop(0)
                r.admit_s = now
                self.in_use += fp
                self.max_in_use = max(self.max_in_use, self.in_use)
                running[r.rid] = (r, self.ex.start(r), fp)
            self.max_running = max(self.max_running, len(running))
            self.queue_depth.append((now, len(waiting), len(running)))
            for rid in list(running):
                r, h, fp = running[rid]
                res = self.ex.done(h)
                if res is not None:
                    r.done_s = self.clock() - t0
                    r.leapfrogs, r.accepted = res
                    self.ex.release(h)
                    self.in_use -= fp
                    del running[rid]
            if not running and waiting and len(running) < self.n_slots and \
                    self.in_use + request_footprint(waiting[0]) > self.budget:
                raise RuntimeError("admission deadlock")
            if i < len(pending) and not waiting and not running:
                # idle until the next arrival
                time_to_next = pending[i].arrival_s - (self.clock() - t0)
                if time_to_next > 0:
                    self.ex.idle(time_to_next)
            else:
                self.ex.idle(poll_s)
        return requests


def summarize(requests: List[Request], wall_s, queue_depth=None, bin_s=1.0):
    """Latency percentiles (completion - arrival), the aggregate completed
    leapfrogs per second of wall time and, given the scheduler's trace of
    (time, waiting, running), the largest waiting depth and, at the end of
    each bin_s window, the waiting depth and the requests in the system."""
    lat = np.array([r.latency_s for r in requests])
    lf = sum(r.leapfrogs for r in requests)
    out = {"requests": len(requests), "p50_latency_s": float(np.percentile(lat, 50)),
           "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
           "max_latency_s": float(lat.max()), "aggregate_leapfrogs_per_s": lf / wall_s,
           "accept_rate": float(sum(r.accepted for r in requests)
                                / max(1, sum(r.n_moves for r in requests))),
           "wall_s": wall_s}
    if queue_depth:
        t = np.array([x[0] for x in queue_depth])
        d = np.array([x[1] for x in queue_depth])
        r = np.array([x[2] for x in queue_depth])
        edges = np.arange(bin_s, t[-1] + bin_s, bin_s)
        idx = np.clip(np.searchsorted(t, edges, side="right") - 1, 0, len(d) - 1)
        out["max_queue_depth"] = int(d.max())
        out["queue_depth_trace"] = [int(x) for x in d[idx]]
        out["in_system_trace"] = [int(x) for x in (d + r)[idx]]
    return out


class PoolExecutor:
    """Runs requests on the HIP worker pool; the model and its chain state
    live on the device from admission to release."""

    def __init__(self, n_workers=4, n_leapfrog=10, n_fixed_point=6, alpha=1e6, precision=None):
        from . import rmhmc
        self.rm = rmhmc
        self.pool = rmhmc.Pool(n_workers)
        self.n_leapfrog, self.K, self.alpha = n_leapfrog, n_fixed_point, alpha
        self.precision = rmhmc.FP64 if precision is None else precision

    def start(self, req: Request):
        import torch
        spec, eps = request_spec(req)
        model = self.rm.Model(spec, self.precision)
        q0 = torch.zeros(spec.D, dtype=torch.float64, device="cuda")
        job = self.pool.submit(model, q0, eps, self.n_leapfrog, self.K, req.n_moves,
                               seed=req.seed, stream_id=req.rid, alpha=self.alpha)
        return job

    def done(self, job):
        if self.pool.poll(job):
            return job.stats.leapfrogs, job.stats.accepted
        return None

    def release(self, job):
        job.model.close()

    def idle(self, s):
        time.sleep(min(s, 0.01))

    def close(self):
        self.pool.close()


class SimulatedExecutor:
    """CPU stand-in: a request takes service_s(req) seconds of simulated time."""

    def __init__(self, service_s, clock):
        self.service_s = service_s
        self.clock = clock         # a SimClock
        self.started = {}

    def start(self, req):
        self.started[req.rid] = (req, self.clock.t + self.service_s(req))
        return req.rid

    def done(self, h):
        req, t_end = self.started[h]
        if self.clock.t >= t_end:
            return (req.n_moves * 10, req.n_moves)
        return None

    def release(self, h):
        del self.started[h]

    def idle(self, s):
        # advance simulated time to the next event
        nxt = [t for _, t in self.started.values() if t > self.clock.t]
        self.clock.t += min([s] + [t - self.clock.t for t in nxt]) if nxt else s


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t
