"""Checkpoint and resume: a solve stopped, written to a checkpoint, and resumed
in a new plan from the file continues bitwise as the uninterrupted solve."""
import numpy as np
import pytest

import bnq_inputs as inp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")


@pytest.mark.parametrize("prec", [0, 1])
def test_resume_is_bitwise(tmp_path, prec):
    from paper_2110_13735_amd import checkpoint
    p = bnq.Params(d=3, N=12, eps=-1, L=6.0, precision=prec, correction=bnq.CORR_MASS)
    f0 = inp.gaussian_mixture(3, 12, 6.0, seed=9, fmax=0.9)
    dt = 0.01
    with bnq.Plan(p) as pl:
        f = torch.tensor(f0, device="cuda:0")
        for _ in range(4):
            pl.step(f, dt)
        torch.cuda.synchronize()
        straight = f.cpu().numpy()
    path = str(tmp_path / "state.npz")
    with bnq.Plan(p) as pl:
        f = torch.tensor(f0, device="cuda:0")
        for _ in range(2):
            pl.step(f, dt)
        torch.cuda.synchronize()
        checkpoint.save(path, p, f, t=2 * dt, step=2)
    c = checkpoint.load(path)
    assert c["params"] == p and c["step"] == 2
    with bnq.Plan(c["params"]) as pl:
        f = torch.tensor(c["f"], device="cuda:0")
        for _ in range(4 - c["step"]):
            pl.step(f, dt)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), straight)
