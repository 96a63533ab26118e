"""Serving loop: every request completes, and its final state is bitwise the
trajectory its own plan computes alone (whatever shared the batch); served
states are also checked against the oracle's RK4 trajectory directly."""
import math

import numpy as np
import pytest

import bnq_inputs as inp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")


def _input(req):
    return inp.mixed_instance(req.d, req.N, req.eps, req.seed)


def test_serving_results_equal_solo_runs():
    from paper_2110_13735_amd import serve
    reqs = serve.poisson_requests(14, rate=400.0, seed=3, cells=[((2, 8), 2), ((2, 16), 1), ((3, 8), 1)],
                                  eps_choices=(-1, 0, 1), t_end=(0.02, 0.08))
    srv = serve.Server(_input, budget_bytes=8 << 30, dt=0.01, keep_results=True)
    try:
        stats = srv.run(reqs, max_wall=120.0)
    finally:
        srv.close()
    assert stats["completed"] == len(reqs)
    assert stats["rebuilds"] >= 2 and stats["p50_latency_s"] <= stats["p99_latency_s"]
    for r in reqs[::3]:
        f0, L = _input(r)
        with bnq.Plan(bnq.Params(d=r.d, N=r.N, eps=r.eps, L=L)) as pl:
            f = torch.tensor(f0, device="cuda:0")
            for _ in range(int(math.ceil(r.t_end / 0.01 - 1e-9))):
                pl.step(f, 0.01)
            torch.cuda.synchronize()
            assert r.steps == int(math.ceil(r.t_end / 0.01 - 1e-9))
            assert np.array_equal(f.cpu().numpy(), r.result), f"request {r.rid} differs from its solo run"


def test_served_states_match_oracle():
    import oracle
    from paper_2110_13735_amd import serve
    reqs = serve.poisson_requests(6, rate=300.0, seed=5, cells=[((2, 8), 1), ((3, 6), 1)],
                                  eps_choices=(-1, 1), t_end=(0.02, 0.04))
    srv = serve.Server(_input, budget_bytes=8 << 30, dt=0.01, keep_results=True)
    try:
        stats = srv.run(reqs, max_wall=120.0)
    finally:
        srv.close()
    assert stats["completed"] == len(reqs)
    for r in reqs:
        f, L = _input(r)
        o = oracle.Oracle(r.d, r.N)
        for _ in range(r.steps):
            f = o.rk4_step(f, 0.01, r.eps, L)
        err = np.linalg.norm(r.result - f) / np.linalg.norm(f)
        assert err <= 1e-12, f"request {r.rid} (d={r.d}, N={r.N}, eps={r.eps}): relative error {err:.2e}"


def test_non_finite_request_fails_alone():
    """A request whose datum is non-finite is failed by the step health flags
    and its slot freed; the others complete with their solo results."""
    from paper_2110_13735_amd import serve
    reqs = serve.poisson_requests(5, rate=500.0, seed=7, cells=[((2, 8), 1)], t_end=(0.03, 0.05))

    def make(req):
        f, L = _input(req)
        if req.rid == 2:
            f = f.copy()
            f.reshape(-1)[5] = np.nan
        return f, L

    srv = serve.Server(make, budget_bytes=8 << 30, dt=0.01, keep_results=True)
    try:
        stats = srv.run(reqs, max_wall=120.0)
    finally:
        srv.close()
    assert reqs[2].status == "failed" and "non-finite" in reqs[2].reason
    assert stats["failed"] == 1 and stats["completed"] == len(reqs) - 1
    for r in reqs:
        if r.rid != 2:
            assert np.all(np.isfinite(r.result))
