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


def _oracle_qhat(d, N, f0, eps, L):
    import oracle
    _, Qh, m = oracle.Oracle(d, N).collide(f0, eps, L, full=True)
    return Qh, m["gain"]


@pytest.mark.parametrize("d,N,eps", [(3, 8, -1), (3, 8, 0), (2, 32, 1)])
def test_pair_split_parity(d, N, eps):
    """Every l-chunking of the pair sums meets the FP64 parity bar against the
    oracle; a recorded split is what a new plan starts with."""
    from tests.parity import check
    L = 6.0
    f0 = inp.gaussian_mixture(d, N, L, seed=5, fmax=0.9)
    ref, gain = _oracle_qhat(d, N, f0, eps, L)
    f = torch.tensor(f0, device="cuda:0")
    p = bnq.Params(d=d, N=N, eps=eps, L=L)
    try:
        for k in sorted({1, 2, 8, 16, 32} & set(range(1, min(N, 32) + 1)) | {3}):
            bnq.tune_pairs_set(d, N, 0, eps, k)
            assert bnq.tune_pairs_get(d, N, 0, eps) == k
            with bnq.Plan(p) as pl:
                print(f"split {k}")
                check(_qhat(pl, f), ref, gain, tol=1e-12)
    finally:
        bnq.tune_pairs_set(d, N, 0, eps, None)
    assert bnq.tune_pairs_get(d, N, 0, eps) is None
    with pytest.raises(bnq.BnqError):
        bnq.tune_pairs_set(d, N, 0, eps, min(N, 32) + 1)


@pytest.mark.parametrize("prec", [0, 1])
def test_pair_autotune_roundtrip(tmp_path, prec):
    d, N, L = 3, 16, 6.0
    f0 = inp.gaussian_mixture(d, N, L, seed=3, fmax=0.9)
    f = torch.tensor(f0, device="cuda:0")
    path = str(tmp_path / "tuning.json")
    try:
        for eps in (0, -1):
            p = bnq.Params(d=d, N=N, eps=eps, L=L, precision=prec)
            with bnq.Plan(p) as pl:
                split, ms = pl.autotune_pairs(f, reps=2)
                print(f"eps {eps} precision {prec}: split {split}, ms {ms}")
                assert split in (8, 16) and ms[0] > 0 and ms[1] > 0 and ms[2] == 0
                tuned = _qhat(pl, f)
            assert bnq.tune_pairs_get(d, N, prec, eps) == split
            bnq.save_tuning(path, [], pair_cells=[(d, N, prec, eps)], pair_ms={(d, N, prec, eps): ms})
            bnq.tune_pairs_set(d, N, prec, eps, None)
            assert bnq.load_tuning(path) >= 1
            assert bnq.tune_pairs_get(d, N, prec, eps) == split
            with bnq.Plan(p) as pl:
                assert np.array_equal(_qhat(pl, f), tuned)
        ent = json.load(open(path))["entries"]
        assert sorted((e["eps0"], e["precision"]) for e in ent) == [(0, prec), (1, prec)]
    finally:
        for eps in (0, -1):
            bnq.tune_pairs_set(d, N, prec, eps, None)


def test_batch_holds_its_plans():
    """A plan a batch holds (the batch copied its workspace pointers) cannot
    be destroyed or autotuned until the batch is gone."""
    d, N, L = 3, 8, 6.0
    f = torch.tensor(inp.gaussian_mixture(d, N, L, seed=1, fmax=0.9), device="cuda:0")
    pl = bnq.Plan(bnq.Params(d=d, N=N, eps=-1, L=L))
    b = bnq.Batch([pl], [f])
    with pytest.raises(bnq.BnqError):
        pl.close()
    with pytest.raises(bnq.BnqError):
        pl.autotune(f, reps=1)
    with pytest.raises(bnq.BnqError):
        pl.autotune_pairs(f, reps=1)
    b.close()
    pl.autotune_pairs(f, reps=1)
    pl.close()
    bnq.tune_pairs_set(d, N, 0, -1, None)
