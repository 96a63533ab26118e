"""Persisted autotuning: bnq_plan_autotune's choice is recorded per device and
(d, N, precision), written to a JSON file and read back by another record
(bnq_tune_get / bnq_tune_set through the C ABI); a plan created after the
record starts with the recorded work distribution and computes bitwise what
the autotuned plan computes."""
import json

import numpy as np
import pytest

import bnq_inputs as inp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")


def _qhat(plan, f):
    Q = torch.empty_like(f)
    Qh = torch.empty(f.shape, dtype=torch.complex128, device=f.device)
    plan.collide(f, Q, Qh)
    torch.cuda.synchronize()
    return Qh.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_tuning_roundtrip_and_reuse(tmp_path, prec):
    d, N, L = 3, 12, 6.0
    f0 = inp.gaussian_mixture(d, N, L, seed=3, fmax=0.9)
    f = torch.tensor(f0, device="cuda:0")
    p = bnq.Params(d=d, N=N, eps=-1, L=L, precision=prec)
    with bnq.Plan(p) as pl:
        choice, ms = pl.autotune(f, reps=1)
        assert 0 <= choice < 4 and np.all(ms > 0)
        tuned = _qhat(pl, f)
    assert bnq.tune_get(d, N, prec) == choice
    path = str(tmp_path / "tuning.json")
    assert bnq.save_tuning(path, [(d, N, prec), (d, N + 2, prec)], ms={(d, N, prec): ms}) == 1
    rec = json.load(open(path))["entries"][0]
    assert (rec["d"], rec["N"], rec["precision"], rec["choice"]) == (d, N, prec, choice)
    bnq.tune_set(d, N, prec, None)
    assert bnq.tune_get(d, N, prec) is None
    assert bnq.load_tuning(path) == 1
    assert bnq.tune_get(d, N, prec) == choice
    with bnq.Plan(p) as pl:
        assert np.array_equal(_qhat(pl, f), tuned)
    with pytest.raises(bnq.BnqError):
        bnq.tune_set(d, N, prec, 4)
    bnq.tune_set(d, N, prec, None)
