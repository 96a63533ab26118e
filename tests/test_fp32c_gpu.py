"""FP32c precision pattern: spectra, tables and short partial sums in FP32,
long sums in FP64.  Parity with the FP64 oracle to 1e-5 (the criteria of
tests/parity.py, as for FP64), at small sizes over several
tiles and ragged windows and at the full 3-D N = 32 shape."""
import numpy as np
import pytest

import bnq_inputs as inp
import oracle
from tests.parity import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")

TOL32 = 1e-5


def _rel(got, ref, scale=0.0):
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref), scale)


def _gpu(p, f):
    dev = torch.device("cuda:0")
    with bnq.Plan(p) as plan:
        ft = torch.tensor(f, device=dev)
        Q = torch.empty_like(ft)
        Qh = torch.empty(f.shape, dtype=torch.complex128, device=dev)
        plan.collide(ft, Q, Qh)
        torch.cuda.synchronize()
        return Q.cpu().numpy(), Qh.cpu().numpy()


@pytest.mark.parametrize("d,N", [(2, 8), (2, 16), (2, 30), (3, 4), (3, 6), (3, 10)])
@pytest.mark.parametrize("eps", [1, -1, 0])
def test_fp32c_collide_matches_oracle(d, N, eps):
    L = 5.0
    f = inp.gaussian_mixture(d, N, L, seed=7 * N + d + eps, fmax=0.9 if eps == -1 else None)
    Q, Qh = _gpu(bnq.Params(d=d, N=N, eps=eps, L=L, precision=bnq.FP32C), f)
    o = oracle.Oracle(d, N)
    Qo, Qho, m = o.collide(f, eps, L, full=True)
    check(Qh, Qho, m["gain"], tol=TOL32)
    check(Q, Qo, oracle.prefactor(d, L) * oracle.idft_real(m["gain"]), tol=TOL32)


def test_fp32c_is_not_fp64():
    # the FP32c path must really round: it differs from FP64 beyond FP64 noise
    d, N, eps, L = 3, 6, -1, 5.0
    f = inp.gaussian_mixture(d, N, L, seed=3, fmax=0.9)
    _, Qh64 = _gpu(bnq.Params(d=d, N=N, eps=eps, L=L), f)
    _, Qh32 = _gpu(bnq.Params(d=d, N=N, eps=eps, L=L, precision=bnq.FP32C), f)
    r = _rel(Qh32, Qh64)
    assert 1e-12 < r <= TOL32


def test_fp32c_full_size_3d32_sparse_spectrum():
    d, N, L, eps = 3, 32, 8.0, -1
    f, sm, co = inp.sparse_spectrum(d, N, seed=5, nmodes=8, amp=0.2)
    Q, Qh = _gpu(bnq.Params(d=d, N=N, eps=eps, L=L, precision=bnq.FP32C), f)
    Qc, T1, Xq = oracle.sparse_modes(d, N, sm, co, eps)
    alpha = oracle.alpha_of(eps, d)
    ref = oracle.sparse_dense(d, N, Qc) - alpha * (oracle.sparse_dense(d, N, T1) + oracle.sparse_dense(d, N, Xq))
    check(Qh, ref, tol=TOL32)
    check(Q, oracle.prefactor(d, L) * oracle.idft_real(ref), tol=TOL32)


def test_fp32c_and_fp64_instances_in_one_batch():
    dev = torch.device("cuda:0")
    specs = [(3, 6, -1, bnq.FP32C), (3, 6, -1, bnq.FP64), (2, 16, 1, bnq.FP32C), (3, 6, 1, bnq.FP32C)]
    plans, fs = [], []
    for i, (d, N, eps, prec) in enumerate(specs):
        f = inp.gaussian_mixture(d, N, 5.0, seed=50 + i, fmax=0.9 if eps == -1 else None)
        plans.append(bnq.Plan(bnq.Params(d=d, N=N, eps=eps, L=5.0, precision=prec)))
        fs.append(torch.tensor(f, device=dev))
    solo = []
    for pl, f in zip(plans, fs):
        Q = torch.empty_like(f)
        pl.collide(f, Q)
        solo.append(Q)
    torch.cuda.synchronize()
    with bnq.Batch(plans, fs) as B:
        # groups (3, 6) FP32c, (3, 6) FP64, (2, 16) FP32c; one shared
        # trilinear launch per precision
        assert B.layout() == (3, 2)
        Qs = [torch.empty_like(f) for f in fs]
        B.collide(Qs)
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(solo, Qs)):
        assert torch.equal(a, b), f"instance {i} differs from its solo evaluation"
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("schedule", ["static", "dynamic"])
def test_fp32c_mixed_cells_share_one_trilinear_launch(schedule):
    """Instances of five cells in FP32c, stepped as one graph-replayed batch
    whose trilinear sums run as one matrix-core launch per stage: bitwise
    the solo trajectories (static), within 1e-12 of them (dynamic tickets
    change the summation order), and within the FP32c bar of the oracle's
    RK4 step for the 2-D instances and the 3-D N = 6 one."""
    import oracle
    from tests.parity import check
    dev = torch.device("cuda:0")
    sched = bnq.SCHED_STATIC if schedule == "static" else bnq.SCHED_DYNAMIC
    specs = [(2, 8, 1), (2, 16, -1), (3, 6, -1), (3, 8, 1), (3, 8, -1), (2, 12, 0)]
    L, dt = 5.0, 0.002
    plans, fb, fsolo, f0s = [], [], [], []
    for i, (d, N, eps) in enumerate(specs):
        f = inp.gaussian_mixture(d, N, L, seed=90 + i, fmax=0.9 if eps == -1 else None)
        plans.append(bnq.Plan(bnq.Params(d=d, N=N, eps=eps, L=L, precision=bnq.FP32C, schedule=sched)))
        fb.append(torch.tensor(f, device=dev))
        fsolo.append(torch.tensor(f, device=dev))
        f0s.append(f)
    for pl, f in zip(plans, fsolo):
        pl.step(f, dt, bnq.RK4)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with bnq.Batch(plans, fb) as B:
        assert B.layout() == (5, 1)  # (3, 8) eps = +-1 are one group
        B.step(dt, bnq.RK4, graph=True, stream=s)
        s.synchronize()
    for i, (a, b) in enumerate(zip(fsolo, fb)):
        if sched == bnq.SCHED_STATIC:
            assert torch.equal(a, b), f"instance {i} differs from its solo step"
        else:
            r = (torch.linalg.norm(a - b) / torch.linalg.norm(a)).item()
            assert r <= 1e-12, f"instance {i}: {r}"
    for i, (d, N, eps) in enumerate(specs):
        if d == 3 and N > 6:
            continue  # the oracle's 3-D N = 8 RK4 step takes half a minute
        ref = oracle.Oracle(d, N).rk4_step(f0s[i], dt, eps, L)
        check(fb[i].cpu().numpy(), ref, tol=TOL32)
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("batched", [False, True])
def test_fp32c_mass_drift_with_mass_correction(batched):
    """FP32c RK4 with the mass correction keeps the discrete mass to 1e-12
    relative over several steps, solo and in a graph-replayed batch (the FP32c
    operator alone drifts at the 1e-8 level)."""
    dev = torch.device("cuda:0")
    cases = [(3, 16, -1, 8.0, 3), (2, 32, 1, 8.0, 4)]
    plans, fs, rho0 = [], [], []
    for d, N, eps, L, seed in cases:
        f = inp.gaussian_mixture(d, N, L, seed=seed, fmax=0.9 if eps == -1 else None)
        plans.append(bnq.Plan(bnq.Params(d=d, N=N, eps=eps, L=L, precision=bnq.FP32C, correction=bnq.CORR_MASS)))
        fs.append(torch.tensor(f, device=dev))
        rho0.append(float(np.sum(f)))
    dt, steps = 0.002, 6
    if batched:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with bnq.Batch(plans, fs) as B:
            for _ in range(steps):
                B.step(dt, bnq.RK4, graph=True, stream=s)
            s.synchronize()
    else:
        for pl, f in zip(plans, fs):
            for _ in range(steps):
                pl.step(f, dt, bnq.RK4)
        torch.cuda.synchronize()
    for (d, N, eps, L, seed), f, r0 in zip(cases, fs, rho0):
        fn = f.cpu().numpy()
        assert np.all(np.isfinite(fn))
        drift = abs(float(np.sum(fn)) - r0) / r0
        assert drift <= 1e-12, f"d={d} N={N} eps={eps}: mass drift {drift:.2e}"
    for pl in plans:
        pl.close()
