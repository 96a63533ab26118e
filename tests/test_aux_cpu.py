"""Auxiliary subsystems on the CPU: checkpoint files, JSON-lines metrics
(including the serving loop's per-request lines, with the fake executor) and
the recorded workload configurations."""
import json
import math
import os

import numpy as np
import pytest

import bnq_inputs as inp
import paper_2110_13735_amd as bnq
from paper_2110_13735_amd import checkpoint, metrics
from paper_2110_13735_amd.serve import Server

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_checkpoint_roundtrip(tmp_path):
    p = bnq.Params(d=3, N=12, eps=-1, L=6.5, hbar=0.8, precision=bnq.FP32C, correction=bnq.CORR_MASS)
    f = np.random.Generator(np.random.PCG64(1)).random((12, 12, 12))
    path = str(tmp_path / "c.npz")
    checkpoint.save(path, p, f, t=0.125, step=25, rho_history=np.arange(3.0))
    c = checkpoint.load(path)
    assert c["params"] == p
    assert np.array_equal(c["f"], f) and c["f"].dtype == np.float64
    assert c["t"] == 0.125 and c["step"] == 25
    assert np.array_equal(c["extra"]["rho_history"], np.arange(3.0))
    with pytest.raises(ValueError):
        checkpoint.save(path, p, f.astype(np.float32), 0.0, 0)
    np.savez(str(tmp_path / "other.npz"), f=f)
    with pytest.raises(ValueError):
        checkpoint.load(str(tmp_path / "other.npz"))


def test_metrics_lines(tmp_path):
    path = str(tmp_path / "m.jsonl")
    with metrics.MetricsLog(path) as log:
        log.write("step", step=1, rho=np.float64(1.5), u=[0.0, 1.0], fmax=float("inf"))
        log.write("summary", n=np.int64(2))
    recs = metrics.read(path)
    assert [r["kind"] for r in recs] == ["step", "summary"]
    assert recs[0]["rho"] == 1.5 and recs[0]["fmax"] == "inf" and recs[1]["n"] == 2
    assert all("wall" in r for r in recs)


def test_serving_writes_one_line_per_request(tmp_path):
    from tests.test_serve_cpu import FakeExecutor, _reqs
    reqs = _reqs([(0.0, 8, 0.03), (0.0, 16, 0.02), (0.001, 8, 0.01)])
    path = str(tmp_path / "serve.jsonl")
    with metrics.MetricsLog(path) as log:
        st = Server(budget_bytes=10 ** 6, executor=FakeExecutor()).run(reqs, metrics=log)
    recs = metrics.read(path)
    req_lines = [r for r in recs if r["kind"] == "request"]
    assert sorted(r["rid"] for r in req_lines) == [0, 1, 2]
    assert all(r["status"] == "done" and r["latency_s"] >= 0 for r in req_lines)
    assert [r["steps"] for r in sorted(req_lines, key=lambda r: r["rid"])] == [3, 2, 1]
    summ = [r for r in recs if r["kind"] == "serve_summary"]
    assert len(summ) == 1 and summ[0]["completed"] == st["completed"] == 3


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C4", "C5"])
def test_configs_record_the_workloads(name):
    c = json.load(open(os.path.join(ROOT, "configs", f"{name}.json")))
    assert c["conventions"]["hbar"] == 1.0 and c["conventions"]["alpha"] == "-eps hbar^d"
    if name == "C1":
        f0, L = inp.two_gaussians_2d(N=c["N"], R_v=c["datum"]["R_v"])
        assert math.isclose(L, c["L"]) and c["eps"] == 1 and c["dt"] == 0.01
    if name == "C2":
        f0 = inp.fermion_mixture_3d(N=c["N"], L=c["L"], seed=c["seed"])
        assert f0.shape == (32, 32, 32) and float(f0.max()) < 1.0 and c["eps"] == -1 and c["dt"] == 0.001
    if name == "C3":
        assert c["N"] == [32, 48] and c["correction"] == "CORR_MASS"
    if name == "C4":
        assert c["instances"] == 512 and c["cells"]["N"] == [16, 24, 32]
    if name == "C5":
        assert c["rate_per_s"] == 200.0 and c["cells"]["weights"] == [4, 3, 2, 1]
