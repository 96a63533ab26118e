"""The allocation-free moments entry point (bnq_moments_noalloc) against
bnq_moments, through the C ABI: two calls in a row on one device, the second
on a smaller grid, each equal to the plan-based call."""
import numpy as np
import pytest

import bnq_inputs as inp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")


def _both(d, N, eps, L, hbar, f0):
    dev = torch.device("cuda:0")
    f = torch.tensor(f0, device=dev)
    out = torch.full((bnq.MOMENTS_LEN + 1,), -1.0, dtype=torch.float64, device=dev)
    p = bnq.Params(d=d, N=N, eps=eps, L=L, hbar=hbar)
    bnq.moments_noalloc(p, f, out)
    torch.cuda.synchronize()
    with bnq.Plan(p) as plan:
        m = plan.moments(f, check=False)
    got = out.cpu().numpy()
    ref = np.array([m[k] for k in bnq.MOMENT_NAMES])
    return got, ref


def test_noalloc_moments_equal_plan_moments_twice_smaller_second():
    cases = [(3, 32, -1, 8.0, 1.0), (2, 16, 1, 5.0, 1.3)]
    for d, N, eps, L, hbar in cases:
        f0 = inp.gaussian_mixture(d, N, L, seed=N + d, fmax=0.9 if eps == -1 else None)
        got, ref = _both(d, N, eps, L, hbar, f0)
        assert np.array_equal(got[:bnq.MOMENTS_LEN], ref), (got, ref)
        assert got[bnq.MOMENTS_LEN] == 0.0


def test_noalloc_moments_count_nonfinite_values():
    d, N, L = 2, 8, 4.0
    f0 = np.full((N, N), 0.25)
    f0[1, 2] = np.nan
    f0[5, 5] = np.inf
    got, ref = _both(d, N, 0, L, 1.0, f0)
    assert got[bnq.MOMENTS_LEN] == 2.0
    assert np.array_equal(got[:bnq.MOMENTS_LEN], ref)


def test_noalloc_rejects_bad_arguments():
    dev = torch.device("cuda:0")
    f = torch.zeros(8, 8, dtype=torch.float64, device=dev)
    with pytest.raises(bnq.BnqError):
        bnq.moments_noalloc(bnq.Params(d=2, N=7, L=4.0), f, f)
    with pytest.raises(bnq.BnqError):
        bnq.moments_noalloc(bnq.Params(d=2, N=8, L=4.0), f, None)
