"""Serving loop with continuous batching on one GPU.

Requests (one instance of the space-homogeneous Boltzmann–Nordheim equation
each: dimension d, modes N, statistics eps, initial datum, end time) arrive
over time.  The server keeps one running batch (libbnq's bnq_batch_*): every
tick advances all admitted instances by one RK4 step in a single captured
HIP-graph replay.  Arrivals are admitted at tick boundaries, first come first
served, while the device-memory budget allows (plan workspace + state, the
shared kernel-mode tables counted once per (d, N)); an instance leaves the
batch when it reaches its end time, and the batch is rebuilt (graph
recaptured) whenever its membership changes.  Each instance's trajectory is
bitwise the one its own plan computes alone, whatever else shares the batch.

All arithmetic runs in libbnq's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import RK4, Batch, Params, Plan, footprint, terms_per_eval


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    d: int
    N: int
    eps: int
    t_end: float
    seed: int
    # filled in by the server
    admitted: float | None = None
    done: float | None = None
    steps: int = 0
    terms: float = 0.0
    result: np.ndarray | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_requests(n: int, rate: float, seed: int, cells, eps_choices=(-1, 1), t_end=(0.05, 0.5)):
    """n requests with exponential inter-arrival times (mean 1/rate s).
    cells: list of ((d, N), weight); eps uniform in eps_choices; t_end uniform
    in the given range; each request carries its own input seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.array([c[1] for c in cells], dtype=float)
    w /= w.sum()
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        d, N = cells[int(rng.choice(len(cells), p=w))][0]
        eps = int(eps_choices[int(rng.integers(len(eps_choices)))])
        te = float(rng.uniform(*t_end))
        out.append(Request(i, t, d, N, eps, te, seed=1000 + i))
    return out


class _Active:
    __slots__ = ("req", "plan", "f", "nsteps", "bytes", "terms_step")

    def __init__(self, req, plan, f, nsteps, nbytes, terms_step):
        self.req, self.plan, self.f, self.nsteps, self.bytes, self.terms_step = req, plan, f, nsteps, nbytes, terms_step


class Server:
    """Continuous-batching server.  make_input(req) -> (f0 ndarray, L)."""

    def __init__(self, make_input, budget_bytes: int, dt: float = 0.01, keep_results: bool = False,
                 max_active: int = 256, precision: int = 0):
        import torch
        self.torch = torch
        self.make_input = make_input
        self.budget = int(budget_bytes)
        self.dt = float(dt)
        self.keep = keep_results
        self.max_active = max_active
        self.precision = int(precision)  # FP64 (0) or FP32C (1) for every request
        self.dev = torch.device("cuda:0")
        self.stream = torch.cuda.Stream()
        self.anchors = {}  # (d, N) -> plan that keeps the shared tables resident
        self.table_bytes = 0

    def _admit(self, req: Request, used: int):
        f0, L = self.make_input(req)
        p = Params(d=req.d, N=req.N, eps=req.eps, L=L, precision=self.precision)
        plan_b, table_b = footprint(p)
        state_b = f0.nbytes
        need = plan_b + state_b + (table_b if (req.d, req.N) not in self.anchors else 0)
        if used + need > self.budget:
            return None
        if (req.d, req.N) not in self.anchors:
            self.anchors[(req.d, req.N)] = Plan(Params(d=req.d, N=req.N, eps=0, L=L, precision=self.precision))
            self.table_bytes += table_b
            need -= table_b
        plan = Plan(p)
        f = self.torch.tensor(f0, device=self.dev)
        nsteps = max(1, int(math.ceil(req.t_end / self.dt - 1e-9)))
        terms = 4.0 * terms_per_eval(p, plan.counts())
        return _Active(req, plan, f, nsteps, need, terms)

    def run(self, requests, max_wall: float | None = None) -> dict:
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active: list[_Active] = []
        used = 0
        batch = None
        dirty = True
        ticks = rebuilds = 0
        terms_done = 0.0
        busy = 0.0
        start = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - start
            if max_wall is not None and now > max_wall:
                break
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                a = self._admit(pending[0], used + self.table_bytes)
                if a is None:
                    if not active:
                        raise RuntimeError(f"request {pending[0].rid} does not fit the memory budget alone")
                    break
                a.req.admitted = now
                active.append(a)
                used += a.bytes
                pending.popleft()
                dirty = True
            if not active:
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - start)))
                continue
            if dirty:
                if batch is not None:
                    batch.close()
                batch = Batch([a.plan for a in active], [a.f for a in active])
                rebuilds += 1
                dirty = False
            t0 = time.perf_counter()
            batch.step(self.dt, RK4, graph=True, stream=self.stream)
            self.stream.synchronize()
            busy += time.perf_counter() - t0
            ticks += 1
            now = time.perf_counter() - start
            still = []
            for a in active:
                a.req.steps += 1
                a.req.terms += a.terms_step
                terms_done += a.terms_step
                if a.req.steps >= a.nsteps:
                    a.req.done = now
                    if self.keep:
                        a.req.result = a.f.cpu().numpy()
                    used -= a.bytes
                    dirty = True
                else:
                    still.append(a)
            if dirty:
                if batch is not None:
                    batch.close()
                    batch = None
                for a in active:
                    if a.req.done is not None:
                        a.plan.close()
            active = still
        if batch is not None:
            batch.close()
        for a in active:
            a.plan.close()
        elapsed = time.perf_counter() - start
        done = [r for r in requests if r.done is not None]
        lat = np.array([r.latency for r in done]) if done else np.array([np.nan])
        return {"completed": len(done), "requests": len(requests), "elapsed_s": elapsed, "ticks": ticks,
                "rebuilds": rebuilds, "busy_s": busy, "terms": terms_done,
                "terms_per_s": terms_done / elapsed if elapsed > 0 else 0.0,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in done])) if done else float("nan")}

    def close(self):
        for p in self.anchors.values():
            p.close()
        self.anchors.clear()
