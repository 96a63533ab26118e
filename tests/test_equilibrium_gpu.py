"""Limit states on the GPU grid: bnq_equilibrium_fill and
bnq_equilibrium_distance against the oracle, the solved state as a near
zero of the operator, and relaxation towards it under RK4 steps."""
import math

import numpy as np
import pytest

import bnq_inputs as inp
import oracle
from oracle import equilibrium as oe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")

DEV = "cuda:0"

# (d, N, L, eps, rho, u, e): one case per kind of limit state
CASES = [
    (2, 30, 6.0, 0, 1.2, [0.3, -0.4], 0.8),            # classical Maxwellian
    (3, 12, 5.0, -1, 2.0, [0.2, 0.0, -0.3], 0.6),      # Fermi-Dirac
    (2, 24, 6.0, 1, 3.0, [0.0, 0.5], 0.5),             # Bose-Einstein
    (3, 10, 4.0, 1, 20.0, [0.0, 0.0, 0.0], 0.3),       # condensate (v = u is a node)
    (3, 10, 4.0, 1, 20.0, [0.05, -0.02, 1e-17], 0.3),  # condensate, u inside the origin's cell
]


def _saturated(d):
    A = 1.3
    vol = math.pi ** (d / 2) * A ** d / math.gamma(d / 2 + 1)
    return vol, d / (d + 2) * A ** 2 / 2


@pytest.mark.parametrize("case", range(len(CASES) + 1))
def test_fill_and_distance_match_oracle(case):
    if case < len(CASES):
        d, N, L, eps, rho, u, e = CASES[case]
    else:  # saturated Fermi-Dirac ball
        d, N, L, eps, u = 2, 32, 3.0, -1, [0.25, 0.0]
        rho, e = _saturated(d)
    st = bnq.equilibrium(d, eps, 1.0, rho, u, e)
    ref = oe.solve(d, eps, 1.0, rho, u, e)
    assert st.kind == ref["kind"]
    plan = bnq.Plan(bnq.Params(d=d, N=N, eps=eps, L=L))
    M = torch.empty((N,) * d, dtype=torch.float64, device=DEV)
    plan.equilibrium_fill(st, M)
    torch.cuda.synchronize()
    Mref, excl = oe.on_grid(d, N, L, ref)
    got = M.cpu().numpy()
    assert np.all(got[excl] == 0.0)
    assert np.max(np.abs(got - Mref)) <= 1e-12 * np.max(np.abs(Mref))
    rng = np.random.default_rng(case)
    f = Mref * (1.0 + 0.1 * rng.standard_normal(Mref.shape)) + np.where(excl, 0.7, 0.0)
    dist = plan.equilibrium_distance(torch.tensor(f, device=DEV), st)
    dref = oe.distance(f, L, ref)
    if st.kind == bnq.EQ_CONDENSATE:
        assert dref["n_excluded"] == 1
    for k in ("l1", "max_abs", "mass_of_state", "mass_excluded"):
        assert dist[k] == pytest.approx(dref[k], rel=1e-12, abs=1e-300), k
    assert dist["n_excluded"] == dref["n_excluded"]
    plan.close()


def test_unknown_state_is_refused():
    rho, e = _saturated(2)
    st = bnq.equilibrium(2, -1, 1.0, 1.2 * rho, [0.0, 0.0], e)
    assert st.kind == bnq.EQ_UNKNOWN
    plan = bnq.Plan(bnq.Params(d=2, N=8, eps=-1, L=3.0))
    M = torch.empty((8, 8), dtype=torch.float64, device=DEV)
    with pytest.raises(bnq.BnqError) as ex:
        plan.equilibrium_fill(st, M)
    assert ex.value.status == bnq.BNQ_EINVAL
    plan.close()


@pytest.mark.parametrize("eps", [-1, 1])
def test_relaxation_towards_the_solved_state(eps):
    # 2-D, two Gaussians of mass 3: the state solved from the datum's moments
    # is a near zero of the operator, and RK4 steps bring the datum to it
    N = 32
    f0, L = inp.two_gaussians_2d(N=N, R_v=4.0)
    f0 = 3.0 * f0
    p = bnq.Params(d=2, N=N, eps=eps, L=L)
    plan = bnq.Plan(p)
    f = torch.tensor(f0, device=DEV)
    m0 = plan.moments(f)
    st = bnq.equilibrium(2, eps, 1.0, m0["rho"], [m0["u0"], m0["u1"]], m0["e"])
    assert st.kind == bnq.EQ_QUANTUM
    M = torch.empty_like(f)
    plan.equilibrium_fill(st, M)
    QM, Qf = torch.empty_like(f), torch.empty_like(f)
    plan.collide(M, QM)
    plan.collide(f, Qf)
    torch.cuda.synchronize()
    ratio = (QM.abs().max() / Qf.abs().max()).item()
    print(f"eps={eps}: |Q(M)| / |Q(f0)| = {ratio:.2e}", flush=True)
    assert ratio < 1e-2
    d0 = plan.equilibrium_distance(f, st)["l1"]
    H0 = m0["H"]
    dist = []
    for k in range(40):
        plan.step(f, 0.05)
        if (k + 1) % 10 == 0:
            dist.append(plan.equilibrium_distance(f, st)["l1"])
    m1 = plan.moments(f)
    print(f"eps={eps}: L1 distance {d0:.3e} -> " + ", ".join(f"{x:.3e}" for x in dist)
          + f"; H {H0:.5f} -> {m1['H']:.5f}", flush=True)
    assert dist[0] < d0 / 10
    assert dist[-1] < d0 / 30
    assert m1["H"] < H0
    assert m1["rho"] == pytest.approx(m0["rho"], rel=1e-12)
    plan.close()
