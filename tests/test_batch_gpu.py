"""Batched evaluation (bnq_batch_*): every instance of a batch must give
bitwise the result its own plan gives alone, eagerly and under HIP-graph
replay.  The solo path is itself checked against the oracle by
test_parity_gpu.py, so bitwise equality carries that parity over."""
import numpy as np
import pytest

import bnq_inputs as inp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")

# (d, N, eps, C_phi, hbar): two (d, N, C_phi) groups share tables, one differs
# only in C_phi (its own group), classical members skip the quantum terms.
MIX = [
    (2, 8, +1, 1.0, 1.0),
    (2, 16, -1, 1.0, 1.0),
    (2, 16, 0, 1.0, 1.0),
    (2, 16, +1, 1.0, 0.7),
    (3, 4, 0, 1.0, 1.0),
    (3, 6, -1, 1.0, 1.0),
    (3, 6, +1, 1.0, 0.8),
    (3, 6, -1, 2.0, 1.0),
]


def _instances(seed0=0):
    dev = torch.device("cuda:0")
    plans, fs = [], []
    for i, (d, N, eps, cphi, hbar) in enumerate(MIX):
        L = 6.0 if d == 2 else 5.0
        p = bnq.Params(d=d, N=N, eps=eps, L=L, C_phi=cphi, hbar=hbar)
        f = inp.gaussian_mixture(d, N, L, seed=seed0 + i)
        if eps == -1:
            f = np.minimum(f, 0.9)
        plans.append(bnq.Plan(p))
        fs.append(torch.tensor(f, device=dev))
    return plans, fs


def test_batch_collide_bitwise_equals_solo():
    plans, fs = _instances()
    solo = []
    for pl, f in zip(plans, fs):
        Q = torch.empty_like(f)
        Qh = torch.empty(f.shape, dtype=torch.complex128, device=f.device)
        pl.collide(f, Q, Qh)
        solo.append((Q, Qh))
    torch.cuda.synchronize()
    with bnq.Batch(plans, fs) as B:
        # five (d, N, C_phi) groups; the trilinear sums of all six quantum
        # members (three cells) share one launch per evaluation
        assert B.layout() == (5, 1)
        Qs = [torch.full_like(f, np.nan) for f in fs]
        Qhs = [torch.zeros(f.shape, dtype=torch.complex128, device=f.device) for f in fs]
        B.collide(Qs, Qhs)
        torch.cuda.synchronize()
        for i, ((Q, Qh), Qb, Qhb) in enumerate(zip(solo, Qs, Qhs)):
            assert torch.equal(Q, Qb), f"instance {i}: Q differs"
            assert torch.equal(Qh, Qhb), f"instance {i}: Qhat differs"


@pytest.mark.parametrize("scheme", [bnq.RK4, bnq.SSPRK2, bnq.EULER])
def test_batch_step_eager_bitwise_equals_solo(scheme):
    plans, fs = _instances(seed0=10)
    ref = [f.clone() for f in fs]
    dts = [0.01 * (1 + 0.1 * i) for i in range(len(plans))]
    for pl, f, dt in zip(plans, ref, dts):
        pl.step(f, dt, scheme)
    torch.cuda.synchronize()
    with bnq.Batch(plans, fs) as B:
        B.step(dts, scheme)
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(ref, fs)):
        assert torch.equal(a, b), f"instance {i} differs after one step"


def test_batch_graph_replays_bitwise():
    plans, fs = _instances(seed0=20)
    ref = [f.clone() for f in fs]
    dt = 0.01
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with bnq.Batch(plans, fs) as B:
        for rep in range(3):
            # eager solo reference step, with the program's own work between replays
            for pl, f in zip(plans, ref):
                pl.step(f, dt)
            torch.cuda.synchronize()
            B.step(dt, bnq.RK4, graph=True, stream=s)
            s.synchronize()
            for i, (a, b) in enumerate(zip(ref, fs)):
                assert torch.equal(a, b), f"replay {rep}, instance {i} differs"
            _ = (fs[0] * 2.0).sum().item()  # unrelated eager work on the default stream
        # a new dt recaptures
        for pl, f in zip(plans, ref):
            pl.step(f, 2 * dt)
        torch.cuda.synchronize()
        B.step(2 * dt, bnq.RK4, graph=True, stream=s)
        s.synchronize()
        for i, (a, b) in enumerate(zip(ref, fs)):
            assert torch.equal(a, b), f"after recapture, instance {i} differs"


def test_batch_invalid_uses_raise():
    plans, fs = _instances(seed0=30)
    with pytest.raises(bnq.BnqError):
        bnq.Batch([plans[0], plans[0]], [fs[0], fs[1]])
    with pytest.raises(bnq.BnqError):
        bnq.Batch([plans[0], plans[1]], [fs[0], fs[0]])
    with bnq.Batch(plans[:2], fs[:2]) as B:
        with pytest.raises(bnq.BnqError):
            B.step(0.01, bnq.RK4, graph=True, stream=0)  # default stream: no capture
        with pytest.raises(bnq.BnqError):
            B.collide([fs[0], torch.empty_like(fs[1])])  # output aliases a state


def test_dynamic_schedule_batch_matches_solo():
    # dynamic tickets change the summation order between runs: compare to 1e-12
    dev = torch.device("cuda:0")
    plans, fs = [], []
    for i, (d, N, eps) in enumerate([(3, 6, -1), (3, 6, 1), (3, 8, -1), (2, 16, 1)]):
        f = inp.gaussian_mixture(d, N, 5.0, seed=70 + i, fmax=0.9 if eps == -1 else None)
        plans.append(bnq.Plan(bnq.Params(d=d, N=N, eps=eps, L=5.0, schedule=bnq.SCHED_DYNAMIC)))
        fs.append(torch.tensor(f, device=dev))
    solo = []
    for pl, f in zip(plans, fs):
        Q = torch.empty_like(f)
        pl.collide(f, Q)
        solo.append(Q)
    torch.cuda.synchronize()
    with bnq.Batch(plans, fs) as B:
        assert B.layout()[1] == 1  # one shared queue launch over (3, 6), (3, 8) and (2, 16)
        Qs = [torch.empty_like(f) for f in fs]
        B.collide(Qs)
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(solo, Qs)):
        r = (torch.linalg.norm(a - b) / torch.linalg.norm(a)).item()
        assert r <= 1e-12, f"instance {i}: {r}"
    for pl in plans:
        pl.close()


def test_pair_sums_at_the_largest_n_batched_and_solo():
    # 2-D N = 64, the largest N: the spectrum plane staged by the pair sums is
    # 64 KiB.  A classical-only instance alone covers I_N; batched with an
    # instance that needs the W sums it runs in the E_g launch shape.  Both
    # must give the same modes bitwise, with exact mass conservation.
    dev = torch.device("cuda:0")
    d, N, L = 2, 64, 6.0
    f = torch.tensor(inp.gaussian_mixture(d, N, L, seed=91, kmin=2), device=dev)
    g = torch.tensor(inp.gaussian_mixture(d, N, L, seed=92, kmin=2), device=dev)
    pa = bnq.Plan(bnq.Params(d=d, N=N, eps=0, L=L))
    pb = bnq.Plan(bnq.Params(d=d, N=N, eps=1, L=L, terms=bnq.T_CLASSICAL | bnq.T_QMULT))
    Qa = torch.empty_like(f)
    Qha = torch.empty(f.shape, dtype=torch.complex128, device=dev)
    pa.collide(f, Qa, Qha)
    torch.cuda.synchronize()
    with bnq.Batch([pa, pb], [f, g]) as B:
        Qs = [torch.empty_like(f), torch.empty_like(g)]
        Qhs = [torch.empty(f.shape, dtype=torch.complex128, device=dev) for _ in range(2)]
        B.collide(Qs, Qhs)
        torch.cuda.synchronize()
    assert torch.equal(Qha, Qhs[0])
    qh = Qha.cpu().numpy()
    assert abs(qh[N // 2, N // 2]) <= 1e-12 * np.abs(qh).max()
    pa.close()
    pb.close()


def test_graph_replayed_batch_matches_oracle():
    """Each member of a graph-replayed batch, after two RK4 steps, against the
    oracle's own RK4 trajectory (no solo run in between)."""
    import oracle

    plans, fs = _instances(seed0=40)
    f0 = [f.cpu().numpy() for f in fs]
    dt = 0.01
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with bnq.Batch(plans, fs) as B:
        for _ in range(2):
            B.step(dt, bnq.RK4, graph=True, stream=s)
        s.synchronize()
    for i, ((d, N, eps, cphi, hbar), f) in enumerate(zip(MIX, f0)):
        L = 6.0 if d == 2 else 5.0
        o = oracle.Oracle(d, N, Cphi=cphi)
        for _ in range(2):
            f = o.rk4_step(f, dt, eps, L, hbar=hbar)
        got = fs[i].cpu().numpy()
        err = np.linalg.norm(got - f) / np.linalg.norm(f)
        assert err <= 1e-12, f"instance {i} {MIX[i]}: relative error {err:.2e}"
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_shared_launch_cut_into_chunks_is_bitwise_solo(prec):
    """Two 3-D N=32 quantum instances carry more than 2e13 trilinear terms, so
    the shared trilinear sum of this batch runs as several launches per
    evaluation, cut by item cost across instances of three sizes; under the
    static schedule every instance is still bitwise its solo evaluation."""
    dev = torch.device("cuda:0")
    P = bnq.FP32C if prec == "fp32c" else bnq.FP64
    specs = [(3, 32, -1), (3, 32, 1), (3, 24, -1), (2, 32, 1)]
    plans, fs = [], []
    for i, (d, N, eps) in enumerate(specs):
        f = inp.gaussian_mixture(d, N, 6.0, seed=110 + i, fmax=0.9 if eps == -1 else None)
        plans.append(bnq.Plan(bnq.Params(d=d, N=N, eps=eps, L=6.0, precision=P)))
        fs.append(torch.tensor(f, device=dev))
    solo = []
    for pl, f in zip(plans, fs):
        Qh = torch.empty(f.shape, dtype=torch.complex128, device=dev)
        pl.collide(f, torch.empty_like(f), Qh)
        solo.append(Qh)
    torch.cuda.synchronize()
    with bnq.Batch(plans, fs) as B:
        assert B.layout() == (3, 1)
        Qhs = [torch.zeros(f.shape, dtype=torch.complex128, device=dev) for f in fs]
        B.collide([torch.empty_like(f) for f in fs], Qhs)
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(solo, Qhs)):
        assert torch.equal(a, b), f"instance {i} differs from its solo evaluation"
    for pl in plans:
        pl.close()
