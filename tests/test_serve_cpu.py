"""Serving logic on the CPU, with a fake executor that stands in for the GPU:
admission by memory budget, refusal (by memory and by estimated service
time), eviction of idle tables, cancellation, failure isolation (a request
whose steps go non-finite is failed and its slot freed while the others
finish), recovery when a batch refuses to step, and fair turns between
lanes of different cost."""
import math
import time

import pytest

from paper_2110_13735_amd import BNQ_ENONFINITE, BnqError
from paper_2110_13735_amd.serve import Request, Server


class FakeExecutor:
    """Instant ticks; per-request plan bytes = 100 N, table bytes = 1000 N per
    (d, N) cell; fail_at[rid] = step after which the request's state is
    non-finite (seen by the health poll, or only when the batch steps if the
    rid is in `late`)."""

    def __init__(self, dt=0.01, fail_at=None, late=(), tick_s=0.0, cost=None):
        self.dt = dt
        self.tick_s = tick_s
        self.cost = cost or {}  # lane -> reported device seconds per member per tick
        self.order = []
        self.fail_at = fail_at or {}
        self.late = set(late)
        self.anchors = set()
        self.lanes = {}
        self.evicted, self.finished, self.discarded, self.batches = [], [], [], 0
        self.steps_taken = {}
        self.t0 = time.perf_counter()

    def begin(self):
        self.t0 = time.perf_counter()

    def footprint(self, req):
        return 100 * req.N, (0 if (req.d, req.N) in self.anchors else 1000 * req.N)

    def evict(self, key):
        self.anchors.remove(key)
        self.evicted.append(key)

    def admit(self, req):
        self.anchors.add((req.d, req.N))
        self.steps_taken[req.rid] = 0
        return {"req": req, "nsteps": max(1, int(math.ceil(req.t_end / self.dt - 1e-9))), "terms_step": 1.0,
                "flag": "", "seen": False}

    def health(self, inst):
        if inst["flag"] and inst["req"].rid in self.late and not inst["seen"]:
            inst["seen"] = True  # the flag becomes visible only after the next step attempt
            return ""
        return inst["flag"]

    def set_members(self, lane, insts):
        if insts:
            self.lanes[lane] = list(insts)
            self.batches += 1
        else:
            self.lanes.pop(lane, None)

    def step(self, lane):
        members = self.lanes[lane]
        self.order.append(lane)
        if any(i["flag"] for i in members):
            raise BnqError(BNQ_ENONFINITE, "a member's step wrote a non-finite value")
        t0 = time.perf_counter()
        for i in members:
            rid = i["req"].rid
            self.steps_taken[rid] += 1
            if self.fail_at.get(rid) == self.steps_taken[rid]:
                i["flag"] = "non-finite state"
        if self.tick_s:
            time.sleep(self.tick_s)
        return t0, t0 + self.cost.get(lane, 1e-3) * len(members)

    def done(self, ev):
        return True

    def wait(self, ev):
        pass

    def time_of(self, ev):
        return ev[1] - self.t0

    def duration(self, ev):
        return ev[1] - ev[0]

    def finish(self, inst):
        self.finished.append(inst["req"].rid)

    def discard(self, inst):
        self.discarded.append(inst["req"].rid)

    def collect(self, force=False):
        pass

    def close(self):
        pass


def _reqs(specs):
    return [Request(i, arr, 3, N, -1, t_end, seed=i) for i, (arr, N, t_end) in enumerate(specs)]


def test_all_requests_complete_with_their_steps():
    reqs = _reqs([(0.0, 8, 0.05), (0.0, 16, 0.03), (0.001, 8, 0.02)])
    ex = FakeExecutor()
    st = Server(budget_bytes=10 ** 6, executor=ex).run(reqs)
    assert st["completed"] == 3 and st["failed"] == 0
    for r in reqs:
        assert r.status == "done" and r.steps == math.ceil(r.t_end / 0.01 - 1e-9)
        assert ex.steps_taken[r.rid] == r.steps and r.latency >= 0.0
    assert sorted(ex.finished) == [0, 1, 2]


def test_refusal_of_a_request_that_cannot_fit_alone():
    # budget 20000: an N = 16 request needs 1600 + 16000, an N = 24 one 2400 + 24000
    reqs = _reqs([(0.0, 24, 0.02), (0.0, 16, 0.02)])
    st = Server(budget_bytes=20000, executor=FakeExecutor()).run(reqs)
    assert reqs[0].status == "refused" and "budget" in reqs[0].reason
    assert reqs[1].status == "done"
    assert st["refused"] == 1 and st["completed"] == 1


def test_idle_tables_are_evicted_for_another_cell():
    # room for one cell's tables at a time: the N = 8 cell is evicted once its
    # request is done and an N = 16 request needs the space
    reqs = _reqs([(0.0, 8, 0.02), (0.0, 16, 0.02)])
    ex = FakeExecutor()
    st = Server(budget_bytes=18000, executor=ex).run(reqs)
    assert st["completed"] == 2
    assert ex.evicted == [(3, 8)]
    assert reqs[1].admitted >= 0.0 and reqs[1].steps == 2


def test_cancellation_of_pending_and_active_requests():
    reqs = _reqs([(0.0, 8, 5.0), (0.0, 8, 0.02), (10.0, 8, 0.02)])
    reqs[0].cancel_at = 0.01  # active, long: removed at a tick boundary
    reqs[2].cancel_at = 0.0   # pending: never admitted
    ex = FakeExecutor(tick_s=0.002)  # 500 ticks of request 0 would take >= 1 s
    st = Server(budget_bytes=10 ** 6, executor=ex).run(reqs, max_wall=5.0)
    assert reqs[0].status == "cancelled" and 0 < reqs[0].steps < 500
    assert reqs[1].status == "done"
    assert reqs[2].status == "cancelled" and reqs[2].admitted is None
    assert 0 in ex.discarded and st["cancelled"] == 2


def test_cancel_call_from_the_tick_hook():
    reqs = _reqs([(0.0, 8, 5.0), (0.0, 16, 0.03)])
    calls = []

    def hook(server, now):
        calls.append(now)
        if len(calls) == 3:
            server.cancel(0)

    st = Server(budget_bytes=10 ** 6, executor=FakeExecutor()).run(reqs, on_tick=hook)
    assert reqs[0].status == "cancelled" and reqs[1].status == "done"
    assert st["completed"] == 1 and st["cancelled"] == 1


@pytest.mark.parametrize("late", [False, True])
def test_failed_request_is_isolated(late):
    # request 1 goes non-finite after its 2nd step; the others finish, its
    # slot is freed and the batch is rebuilt without it (late: the flag is
    # seen only when the batch refuses to step)
    reqs = _reqs([(0.0, 8, 0.06), (0.0, 8, 0.06), (0.0, 16, 0.04)])
    ex = FakeExecutor(fail_at={1: 2}, late=(1,) if late else ())
    st = Server(budget_bytes=10 ** 6, executor=ex).run(reqs)
    assert reqs[1].status == "failed" and reqs[1].reason == "non-finite state"
    assert ex.steps_taken[1] == 2
    assert reqs[0].status == "done" and reqs[0].steps == 6
    assert reqs[2].status == "done" and reqs[2].steps == 4
    assert st["failed"] == 1 and st["completed"] == 2 and 1 in ex.discarded


def test_lanes_share_device_time_fairly():
    # one N = 16 request whose ticks cost 10x those of the N = 8 lane: the
    # N = 8 requests tick about ten times per N = 16 tick, so they finish
    # long before the N = 16 request, whose steps are not starved either
    reqs = _reqs([(0.0, 16, 0.2), (0.0, 8, 0.3), (0.0, 8, 0.3)])
    ex = FakeExecutor(cost={(3, 8): 1e-3, (3, 16): 1e-2})
    st = Server(budget_bytes=10 ** 6, executor=ex).run(reqs)
    assert st["completed"] == 3
    # per-request fair shares: the N = 8 lane (2 members, 2e-3 s a tick) gets
    # 2/3 of the device time, the N = 16 lane (1e-2 s a tick) 1/3, so the N = 8
    # lane's 30 ticks interleave with about 3 N = 16 ticks (plus the first
    # ones, before any cost is measured)
    last_small = max(i for i, k in enumerate(ex.order) if k == (3, 8))
    assert ex.order.count((3, 8)) == 30 and ex.order.count((3, 16)) == 20
    assert 2 <= ex.order[:last_small].count((3, 16)) <= 6, ex.order
    assert st["device_s_per_step_member"]["3d16"] == pytest.approx(1e-2)


def test_refusal_by_estimated_service_time():
    # the N = 16 cell measures 0.1 s per step per member on its first
    # request: a later N = 16 request of 10 steps (1 s) is refused under a
    # 0.5 s limit, while N = 8 requests (cost from the hint) are served
    reqs = _reqs([(0.0, 16, 0.02), (0.05, 16, 0.1), (0.05, 8, 0.1)])
    ex = FakeExecutor(cost={(3, 16): 0.1, (3, 8): 1e-3}, tick_s=0.01)
    srv = Server(budget_bytes=10 ** 6, executor=ex, max_service_s=0.5, step_cost=lambda r: 1e-3)
    st = srv.run(reqs)
    assert reqs[0].status == "done"
    assert reqs[1].status == "refused" and "estimated service" in reqs[1].reason
    assert reqs[2].status == "done"
    assert st["refused"] == 1


def test_executor_closes_batches_before_their_plans():
    """A batch keeps pointers to its plans: the GPU executor's deferred close
    must release a retired batch before any plan it holds, and keep a plan that
    the lane's current batch still holds."""
    from paper_2110_13735_amd import Batch
    from paper_2110_13735_amd.serve import GpuExecutor

    log = []

    class Ev:
        def query(self):
            return True

        def synchronize(self):
            pass

    class P:
        def __init__(self, name):
            self.name = name

        def close(self):
            log.append(self.name)

    class B(Batch):
        def __init__(self, name, plans):
            self.name, self.plans = name, plans

        def close(self):
            log.append(self.name)

        def __del__(self):
            pass

    ex = object.__new__(GpuExecutor)
    p1, p2, p3 = P("p1"), P("p2"), P("p3")
    old, cur = B("old", [p1, p2, p3]), B("cur", [p2, p3])
    ex.batches = {(3, 8): cur}
    # retired in the order the server retires them: p1's plan, then the old batch
    ex.retired = [(Ev(), [p1]), (Ev(), [old]), (Ev(), [p3])]
    ex.collect()
    assert log == ["old", "p1"]  # p3 is still held by the current batch
    assert [objs[0] for _, objs in ex.retired] == [p3]
    ex.batches = {}
    ex.retired.append((Ev(), [cur]))
    ex.collect()
    assert log == ["old", "p1", "cur", "p3"]
