"""3-D N = 48 on one GPU.

The FP32c kernel-mode tables fit (182 GB; the FP64 ones would take 364 GB of
the 288 GB of HBM), so an FP32c plan builds its FP32 tables directly (each
value formed in FP64, stored rounded to nearest).  An FP64 plan keeps the
168 GB of FP64 trilinear rows and forms its pair weights on the fly
(tests/test_n48_fp64_gpu.py); beside the FP32 set it is refused with ENOMEM
before anything is allocated.  The oracle cannot evaluate a dense
N = 48 operator in seconds; the operator is checked on a sparse spectrum,
whose exact Galerkin sums the oracle forms over the support, and the tables
on random index pairs against the oracle's own quadrature.
"""
import numpy as np
import pytest

import bnq_inputs as inp
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")

N = 48
TOL32 = 1e-5


@pytest.fixture(scope="module")
def plan48():
    plan = bnq.Plan(bnq.Params(d=3, N=N, eps=1, L=8.0, precision=bnq.FP32C))
    yield plan
    plan.close()


def _near32(got, ref):
    # an FP32 entry is the FP64 value (itself within 1e-12 of the oracle's)
    # rounded to nearest: within half an FP32 ulp, 2^-24 relative
    return np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) + 2e-12)


def test_fp32_tables_match_oracle_quadrature(plan48):
    rng = np.random.default_rng(48)
    n = 300
    a = rng.integers(-(N - 1), N, (n, 3)).astype(np.int32)
    b = rng.integers(-(N - 1), N, (n, 3)).astype(np.int32)
    a[:3] = 0
    b[2:5] = 0
    a[5] = b[6] = N - 1  # the far corner of the trilinear table
    assert _near32(plan48.lookup(0, a, b), oracle.beta_pairs(3, a, b))
    h = N // 2
    l = rng.integers(-h, h, (n, 3)).astype(np.int32)
    m = rng.integers(-h, h, (n, 3)).astype(np.int32)
    l[0] = m[0] = -h
    blm = oracle.beta_pairs(3, l, m)
    bmm = oracle.beta_pairs(3, m, m)
    bsl = oracle.beta_pairs(3, l + m, l)
    bls = oracle.beta_pairs(3, l, l + m)
    inI = np.all((l + m >= -h) & (l + m < h), axis=1)
    assert _near32(plan48.lookup(1, l, m), np.where(inI, blm - bmm, 0.0))
    assert _near32(plan48.lookup(2, l, m), blm - bsl - bls)


def test_fp32c_collide_sparse_spectrum_matches_oracle(plan48):
    # every kernel at 3-D N = 48 (all 19600 trilinear rows, the trilinear sum
    # cut into several launches), on a spectrum of 17 non-zero modes
    eps, L = 1, 8.0
    f, sm, co = inp.sparse_spectrum(3, N, seed=7, nmodes=8, amp=0.2)
    dev = torch.device("cuda:0")
    ft = torch.tensor(f, device=dev)
    Q = torch.empty_like(ft)
    Qh = torch.empty(f.shape, dtype=torch.complex128, device=dev)
    plan48.collide(ft, Q, Qh)
    torch.cuda.synchronize()
    Q, Qh = Q.cpu().numpy(), Qh.cpu().numpy()
    Qc, T1, Xq = oracle.sparse_modes(3, N, sm, co, eps)
    alpha = oracle.alpha_of(eps, 3)
    ref = oracle.sparse_dense(3, N, Qc) - alpha * (oracle.sparse_dense(3, N, T1) + oracle.sparse_dense(3, N, Xq))
    err = np.linalg.norm(Qh - ref) / np.linalg.norm(ref)
    print(f"3-D N=48 FP32c sparse spectrum: relative error {err:.2e}", flush=True)
    assert err <= TOL32
    Qref = oracle.prefactor(3, L) * oracle.idft_real(ref)
    assert np.linalg.norm(Q - Qref) / np.linalg.norm(Qref) <= TOL32
    # mass: the zero mode is a sum of terms that cancel pairwise
    h = N // 2
    assert abs(Qh[h, h, h]) <= TOL32 * np.abs(ref).max()


def test_fp64_plan_beside_the_fp32_tables_is_refused(plan48):
    # the FP64 trilinear rows (168 GB) do not fit beside the FP32 set (182 GB)
    with pytest.raises(bnq.BnqError) as e:
        bnq.Plan(bnq.Params(d=3, N=N, eps=1, L=8.0))
    assert e.value.status == bnq.BNQ_ENOMEM


def test_3d64_plan_refused_for_lack_of_memory():
    # 3-D N = 64: 45760 trilinear rows of 2.4e6 values, over 400 GB even in FP32
    for prec in (bnq.FP64, bnq.FP32C):
        with pytest.raises(bnq.BnqError) as e:
            bnq.Plan(bnq.Params(d=3, N=64, eps=1, L=8.0, precision=prec))
        assert e.value.status == bnq.BNQ_ENOMEM
