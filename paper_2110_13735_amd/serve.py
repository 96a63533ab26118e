"""Serving loop with continuous batching on one GPU.

Requests (one instance of the space-homogeneous Boltzmann–Nordheim equation
each: dimension d, modes N, statistics eps, initial datum, end time) arrive
over time.  The admitted requests of one (d, N) cell form a lane with one
running batch (libbnq's bnq_batch_*): a tick advances all of the lane's
instances by one RK4 step in a single captured HIP-graph replay.  Lanes take
turns by start-time fair queuing on measured device time, so each active
request gets about the same share of the device.

* Admission: at tick boundaries, first come first served, while the
  device-memory budget allows (plan workspace + state per request, the
  shared kernel-mode tables counted once per (d, N) and kept resident while
  requests of that cell are admitted or recently served; idle cells' tables
  are evicted when an admission needs the room).  A request that cannot fit
  even alone is refused, and so is one whose estimated service time (from the
  measured device time per step of its cell) exceeds an optional limit.
* Ticks are pipelined: the host enqueues a tick and goes on admitting and
  bookkeeping while the device runs; it waits only when `depth` ticks are in
  flight, or when a membership change must retire the previous batch.  A
  request's completion time is its last tick's end on the device clock.
* Health: each step records non-finite values or Fermi–Dirac values >= 1/|alpha|
  in its plan's host-visible flags (bnq_step health); the server reads them
  without waiting, marks such a request failed, frees its slot and steps the
  others on (a batch whose member has failed refuses to step until rebuilt).
* Cancellation: Server.cancel(rid) removes a pending request, or an active
  one at the next tick boundary.
* Each instance's trajectory is bitwise the one its own plan computes alone,
  whatever else shares the batch.

All arithmetic runs in libbnq's kernels; this module only schedules.  The
scheduling is written against a small executor interface (GpuExecutor here;
the tests drive it with a CPU fake as well).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import (BNQ_EBOUND, BNQ_ENONFINITE, CORR_MASS, CORR_NONE, FP32C, HEALTH_BOUND, HEALTH_NONFINITE, RK4, Batch,
               BnqError, Params, Plan, footprint, terms_per_eval)


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    d: int
    N: int
    eps: int
    t_end: float
    seed: int
    cancel_at: float | None = None  # the client cancels at this time after the start (tests)
    # filled in by the server
    status: str = "pending"  # pending, active, done, failed, cancelled, refused
    reason: str = ""
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


# ---------------------------------------------------------------------------
class GpuExecutor:
    """libbnq plans, batches and HIP events on one GPU."""

    def __init__(self, make_input, dt: float, precision: int = 0, keep_results: bool = False):
        import torch
        self.torch = torch
        self.make_input = make_input
        self.dt = float(dt)
        self.precision = int(precision)
        self.keep = keep_results
        self.dev = torch.device("cuda:0")
        self.stream = torch.cuda.Stream()  # ticks
        self.admin = torch.cuda.Stream()   # plan builds and uploads of admitted requests
        self.anchors = {}                  # (d, N) -> plan that keeps the shared tables resident
        self.batches = {}                  # lane (d, N) -> Batch of its members
        self.retired = []                  # (event, [objects to close]) once the event has completed
        self.t0_evt = torch.cuda.Event(enable_timing=True)

    def begin(self):
        """Start of a run: the origin of the device-clock completion times."""
        self.stream.synchronize()
        self.t0_evt.record(self.stream)

    # sizes -------------------------------------------------------------
    def params(self, req, L):
        # FP32c solves keep their mass to rounding with the mass correction
        return Params(d=req.d, N=req.N, eps=req.eps, L=L, precision=self.precision,
                      correction=CORR_MASS if self.precision == FP32C else CORR_NONE)

    def footprint(self, req):
        """(bytes of the request's own workspace and state, bytes of its cell's
        shared tables if they are not resident)."""
        f0, L = self.make_input(req)
        plan_b, table_b = footprint(self.params(req, L))
        key = (req.d, req.N)
        return plan_b + f0.nbytes, (0 if key in self.anchors else table_b)

    def resident_cells(self):
        return list(self.anchors)

    def evict(self, key):
        """Release an idle cell's tables (its anchor plan)."""
        plan = self.anchors.pop(key)
        self._close_later([plan])

    # instances ---------------------------------------------------------
    def admit(self, req):
        torch = self.torch
        f0, L = self.make_input(req)
        p = self.params(req, L)
        key = (req.d, req.N)
        if key not in self.anchors:
            self.anchors[key] = Plan(Params(d=req.d, N=req.N, eps=0, L=L, precision=self.precision), stream=self.admin)
        plan = Plan(p, stream=self.admin)
        with torch.cuda.stream(self.admin):
            f = torch.tensor(f0, device=self.dev)
        ev = torch.cuda.Event()
        ev.record(self.admin)
        self.stream.wait_event(ev)
        nsteps = max(1, int(math.ceil(req.t_end / self.dt - 1e-9)))
        return {"req": req, "plan": plan, "f": f, "nsteps": nsteps, "terms_step": 4.0 * terms_per_eval(p, plan.counts())}

    def health(self, inst):
        fl = inst["plan"].health(wait=False)
        if fl & HEALTH_NONFINITE:
            return "non-finite state"
        if fl & HEALTH_BOUND:
            return "Fermi-Dirac bound reached"
        return ""

    def set_members(self, lane, insts):
        """A new batch for this lane's instances; the previous one is retired
        after its last enqueued tick."""
        old = self.batches.pop(lane, None)
        if old is not None:
            self._close_later([old])
        if insts:
            self.batches[lane] = Batch([i["plan"] for i in insts], [i["f"] for i in insts])

    def step(self, lane):
        """Enqueue one RK4 tick of the lane's batch; returns its (start, end) events."""
        torch = self.torch
        t0 = torch.cuda.Event(enable_timing=True)
        t0.record(self.stream)
        self.batches[lane].step(self.dt, RK4, graph=True, stream=self.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return t0, ev

    def done(self, ev) -> bool:
        return ev[1].query()

    def wait(self, ev):
        ev[1].synchronize()

    def time_of(self, ev) -> float:
        """Seconds after the start of the run at which the tick ended (device clock)."""
        return self.t0_evt.elapsed_time(ev[1]) * 1e-3

    def duration(self, ev) -> float:
        """Device seconds the tick took."""
        return ev[0].elapsed_time(ev[1]) * 1e-3

    def finish(self, inst):
        """The request's last tick has completed: keep its state if asked, and
        release its plan once the work enqueued since has run."""
        if self.keep:
            with self.torch.cuda.stream(self.admin):  # not the default stream: no wait on the tick stream
                inst["req"].result = inst["f"].cpu().numpy()
        self._close_later([inst["plan"]])

    def discard(self, inst):
        """A request leaves before its end (failed, cancelled, stopped)."""
        self._close_later([inst["plan"]])

    def _close_later(self, objs):
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self.retired.append((ev, objs))

    def collect(self, force: bool = False):
        """Close retired batches and plans whose work has completed.  A batch
        keeps pointers to its plans, so batches close first, and a plan only
        once no live batch (current or retired) still holds it."""
        def ready(ev):
            if force:
                ev.synchronize()
                return True
            return ev.query()

        keep = []
        for ev, objs in self.retired:
            if all(isinstance(o, Batch) for o in objs) and ready(ev):
                for o in objs:
                    o.close()
            else:
                keep.append((ev, objs))
        held = {id(pl) for b in self.batches.values() for pl in b.plans}
        held |= {id(pl) for _, objs in keep for o in objs if isinstance(o, Batch) for pl in o.plans}
        self.retired = []
        for ev, objs in keep:
            if not any(isinstance(o, Batch) for o in objs) and not any(id(o) in held for o in objs) and ready(ev):
                for o in objs:
                    o.close()
            else:
                self.retired.append((ev, objs))

    def close(self):
        self.stream.synchronize()
        for b in self.batches.values():
            b.close()
        self.batches.clear()
        self.collect(force=True)  # retired batches, then the plans they held
        for p in self.anchors.values():
            p.close()
        self.anchors.clear()


# ---------------------------------------------------------------------------
class _Lane:
    """The active requests of one (d, N) cell: one batch, ticked as a unit."""
    __slots__ = ("key", "members", "dirty", "vtime")

    def __init__(self, key, vtime):
        self.key, self.members, self.dirty, self.vtime = key, [], True, vtime


class Server:
    """Continuous-batching server over an executor (GpuExecutor by default;
    make_input(req) -> (f0 ndarray, L)).

    Requests of one (d, N) cell share a lane (one batch, one graph); lanes
    take turns on the device by start-time fair queuing: each tick advances
    the lane's virtual time by its measured tick cost over its member count,
    and the lane with the least virtual time ticks next, so every active
    request gets about the same share of device time whatever its cell, and
    small requests are not held behind the ticks of large ones.

    max_service_s: refuse a request whose estimated service time (steps x
    device seconds per step of one member of its cell, measured on earlier
    ticks, else from step_cost(req) if given) exceeds this."""

    def __init__(self, make_input=None, budget_bytes: int = 0, dt: float = 0.01, keep_results: bool = False,
                 max_active: int = 256, precision: int = 0, depth: int = 2, executor=None,
                 max_service_s: float | None = None, step_cost=None):
        self.ex = executor if executor is not None else GpuExecutor(make_input, dt, precision, keep_results)
        self.dt = float(dt)
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.depth = max(1, int(depth))
        self.max_service_s = max_service_s
        self.step_cost = step_cost
        self.table_bytes = {}  # resident cell -> bytes of its tables
        self.cell_use = collections.Counter()  # active requests per cell
        self.member_s = {}  # cell -> measured device seconds per tick per member (last tick)
        self._cancel = set()

    def cancel(self, rid: int):
        """Cancel request rid: dropped if pending, removed from its lane at the
        next tick boundary if active."""
        self._cancel.add(rid)

    def nsteps(self, req) -> int:
        return max(1, int(math.ceil(req.t_end / self.dt - 1e-9)))

    def estimate_service(self, req):
        """Estimated device seconds to serve req, or None if nothing is known."""
        per = self.member_s.get((req.d, req.N))
        if per is None and self.step_cost is not None:
            per = self.step_cost(req)
        return None if per is None else per * self.nsteps(req)

    def _try_admit(self, req, used):
        own, tables = self.ex.footprint(req)
        key = (req.d, req.N)
        need = own + (tables if key not in self.table_bytes else 0)
        if used + need + sum(self.table_bytes.values()) > self.budget:
            # evict idle cells' tables until it fits
            for cell in list(self.table_bytes):
                if self.cell_use[cell] == 0 and cell != key:
                    self.ex.evict(cell)
                    del self.table_bytes[cell]
                    if used + need + sum(self.table_bytes.values()) <= self.budget:
                        break
            if used + need + sum(self.table_bytes.values()) > self.budget:
                return None, own + tables
        inst = self.ex.admit(req)
        if key not in self.table_bytes:
            self.table_bytes[key] = tables
        self.cell_use[key] += 1
        inst["bytes"] = own
        return inst, need

    def run(self, requests, max_wall: float | None = None, on_tick=None, metrics=None) -> dict:
        """Serve `requests` until all have left (or max_wall seconds); on_tick(server,
        now) is called at every tick boundary; metrics: a MetricsLog that gets
        one line per request that leaves and a summary line."""
        ex = self.ex
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        lanes = {}  # (d, N) -> _Lane
        inflight = collections.deque()  # (events, lane key, members, [instances that end with this tick])
        used = 0
        ticks = rebuilds = 0
        terms_done = busy = 0.0
        ex.begin()
        start = time.perf_counter()

        def retire(lane, inst, status, reason=""):
            # accounting and status; a finished request's state is read and
            # its plan released when its last tick has completed
            nonlocal used
            r = inst["req"]
            r.status, r.reason = status, reason
            used -= inst["bytes"]
            self.cell_use[lane.key] -= 1
            lane.members.remove(inst)
            lane.dirty = True
            if status != "done":
                ex.discard(inst)

        def land(entry):
            nonlocal busy
            ev, key, n, ending = entry
            ex.wait(ev)
            t_end = ex.time_of(ev)
            dur = ex.duration(ev)
            busy += dur
            self.member_s[key] = dur / n
            for inst in ending:
                inst["req"].done = t_end
                ex.finish(inst)

        while pending or inflight or any(ln.members for ln in lanes.values()):
            now = time.perf_counter() - start
            if max_wall is not None and now > max_wall:
                break
            if on_tick is not None:
                on_tick(self, now)
            # completed ticks: device time, per-member cost and completion times
            while inflight and (len(inflight) >= self.depth or ex.done(inflight[0][0])):
                land(inflight.popleft())
            ex.collect()
            # cancellations, then the health of the steps that have completed
            # (host-visible flags, no wait)
            for r in list(pending):
                if r.rid in self._cancel or (r.cancel_at is not None and now >= r.cancel_at):
                    pending.remove(r)
                    r.status = "cancelled"
            for lane in lanes.values():
                for inst in list(lane.members):
                    r = inst["req"]
                    if r.rid in self._cancel or (r.cancel_at is not None and now >= r.cancel_at):
                        retire(lane, inst, "cancelled")
                        continue
                    why = ex.health(inst)
                    if why:
                        retire(lane, inst, "failed", why)
            # admissions, first come first served
            nact = sum(len(ln.members) for ln in lanes.values())
            while pending and pending[0].arrival <= now and nact < self.max_active:
                req = pending[0]
                est = self.estimate_service(req)
                if self.max_service_s is not None and est is not None and est > self.max_service_s:
                    pending.popleft()
                    req.status, req.reason = "refused", f"estimated service {est:.3g} s > {self.max_service_s} s"
                    continue
                inst, need = self._try_admit(req, used)
                if inst is None:
                    if nact == 0 and not inflight:
                        pending.popleft()
                        req.status, req.reason = "refused", f"needs {need} bytes, budget {self.budget}"
                        continue
                    break
                key = (req.d, req.N)
                if key not in lanes:
                    live = [ln.vtime for ln in lanes.values() if ln.members]
                    lanes[key] = _Lane(key, min(live) if live else 0.0)
                req.admitted = now
                req.status = "active"
                lanes[key].members.append(inst)
                lanes[key].dirty = True
                used += inst["bytes"]
                nact += 1
                pending.popleft()
            # lanes left empty release their batch
            for key in [k for k, ln in lanes.items() if not ln.members]:
                ex.set_members(key, [])
                del lanes[key]
            if not lanes:
                if pending and not inflight:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - (time.perf_counter() - start))))
                continue
            lane = min(lanes.values(), key=lambda ln: ln.vtime)
            if lane.dirty:
                ex.set_members(lane.key, lane.members)
                rebuilds += 1
                lane.dirty = False
            try:
                ev = ex.step(lane.key)
            except BnqError as e:
                if e.status not in (BNQ_ENONFINITE, BNQ_EBOUND):
                    raise
                # a member's flags were set after the health poll: rebuild without it
                failed = 0
                for inst in list(lane.members):
                    why = ex.health(inst)
                    if why:
                        retire(lane, inst, "failed", why)
                        failed += 1
                if not failed:
                    raise
                continue
            ticks += 1
            n = len(lane.members)
            per = self.member_s.get(lane.key)
            if per is None and self.step_cost is not None:
                per = self.step_cost(lane.members[0]["req"])
            lane.vtime += per if per is not None else 0.0
            ending = []
            for inst in list(lane.members):
                r = inst["req"]
                r.steps += 1
                r.terms += inst["terms_step"]
                terms_done += inst["terms_step"]
                if r.steps >= inst["nsteps"]:
                    ending.append(inst)
                    retire(lane, inst, "done")
            inflight.append((ev, lane.key, n, ending))
        # drain
        while inflight:
            land(inflight.popleft())
        for lane in lanes.values():  # stopped by max_wall
            for inst in list(lane.members):
                retire(lane, inst, "active")
            ex.set_members(lane.key, [])
        ex.collect()
        elapsed = time.perf_counter() - start
        done = [r for r in requests if r.status == "done" and r.done is not None]
        lat = np.array([r.latency for r in done]) if done else np.array([np.nan])
        count = collections.Counter(r.status for r in requests)
        if metrics is not None:
            for r in requests:
                metrics.write("request", rid=r.rid, d=r.d, N=r.N, eps=r.eps, t_end=r.t_end, status=r.status,
                              reason=r.reason, arrival_s=r.arrival, admitted_s=r.admitted, done_s=r.done,
                              latency_s=r.latency if r.done is not None else None,
                              queue_s=(r.admitted - r.arrival) if r.admitted is not None else None,
                              steps=r.steps, terms=r.terms)
        stats = {"completed": len(done), "failed": count.get("failed", 0), "cancelled": count.get("cancelled", 0),
                 "refused": count.get("refused", 0), "unfinished": count.get("active", 0) + count.get("pending", 0),
                 "requests": len(requests), "elapsed_s": elapsed, "ticks": ticks, "rebuilds": rebuilds,
                 "terms": terms_done, "terms_per_s": terms_done / elapsed if elapsed > 0 else 0.0,
                 "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                 "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in done])) if done else float("nan"),
                 "busy_s": busy, "device_s_per_step_member": {f"{k[0]}d{k[1]}": v for k, v in self.member_s.items()},
                 "fail_reasons": dict(collections.Counter(r.reason for r in requests if r.status == "failed"))}
        if metrics is not None:
            metrics.write("serve_summary", **stats)
        return stats

    def close(self):
        self.ex.close()
