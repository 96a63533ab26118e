"""Full-size parity on dense data: the GPU operator against the oracle's
Galerkin modes stored by tests/golden/make_dense_golden.py (series kernel
modes, pinned to the quadrature in tests/test_oracle.py):

  3-D N = 32, the C2 fermion datum, 34 output modes (n = 0, modes on the
      -N/2 faces, seeded modes): every trilinear row and both block-width
      templates of the FP64 kernel meet non-zero data;
  3-D N = 16, the same recipe, every output mode.

FP64 at 1e-12 and FP32c at 1e-5 (tests/parity.py criteria over the stored
modes), under the static and the dynamic schedule, the full operator and each
term alone."""
import os

import numpy as np
import pytest

import bnq_inputs as inp
import oracle
from tests.parity import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    z = np.load(os.path.join(GOLDEN, name), allow_pickle=False)
    N, L, seed, eps = int(z["N"]), float(z["L"]), int(z["seed"]), int(z["eps"])
    f = inp.fermion_mixture_3d(N=N, L=L, seed=seed)
    assert np.allclose(z["f_checksum"], [f.sum(), (f * f).sum()], rtol=1e-14, atol=0)
    return z, f, N, L, eps


def _gpu_qhat(p, f):
    dev = torch.device("cuda:0")
    with bnq.Plan(p) as plan:
        ft = torch.tensor(f, device=dev)
        Q = torch.empty_like(ft)
        Qh = torch.empty(f.shape, dtype=torch.complex128, device=dev)
        plan.collide(ft, Q, Qh)
        torch.cuda.synchronize()
        return Qh.cpu().numpy().reshape(-1)


def _expected(z, eps, mask):
    alpha = oracle.alpha_of(eps, 3)
    ref = np.zeros_like(z["Qc"])
    if mask & bnq.T_CLASSICAL:
        ref = ref + z["Qc"]
    if mask & bnq.T_QTRI:
        ref = ref - alpha * z["T1"]
    if mask & bnq.T_QMULT:
        ref = ref - alpha * z["Xq"]
    return ref


CASES = [(bnq.FP64, bnq.SCHED_STATIC, bnq.T_ALL), (bnq.FP64, bnq.SCHED_DYNAMIC, bnq.T_ALL),
         (bnq.FP32C, bnq.SCHED_STATIC, bnq.T_ALL), (bnq.FP32C, bnq.SCHED_DYNAMIC, bnq.T_ALL),
         (bnq.FP64, bnq.SCHED_STATIC, bnq.T_QTRI), (bnq.FP64, bnq.SCHED_STATIC, bnq.T_QMULT),
         (bnq.FP64, bnq.SCHED_STATIC, bnq.T_CLASSICAL), (bnq.FP32C, bnq.SCHED_STATIC, bnq.T_QTRI)]


@pytest.mark.parametrize("name", ["dense_3d16_all_modes.npz", "c2_3d32_sampled_modes.npz"])
@pytest.mark.parametrize("prec,sched,mask", CASES)
def test_dense_golden_modes(name, prec, sched, mask):
    if not os.path.exists(os.path.join(GOLDEN, name)):
        pytest.skip(f"{name} not generated")
    z, f, N, L, eps = _load(name)
    got = _gpu_qhat(bnq.Params(d=3, N=N, eps=eps, L=L, precision=prec, schedule=sched, terms=mask), f)[z["index"]]
    ref = _expected(z, eps, mask)
    gain = z["gain"] if mask & bnq.T_CLASSICAL else None
    check(got, ref, gain, tol=1e-12 if prec == bnq.FP64 else 1e-5)
