"""CPU checks of the C ABI: the library loads and exports every declared
entry point; parameter validation works without a GPU."""
import ctypes
import os
import re

import pytest

import paper_2110_13735_amd as bnq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bnq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bnq_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_entry_points():
    names = _declared()
    for n in ("bnq_plan", "bnq_collide", "bnq_step", "bnq_moments"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    lib = ctypes.CDLL(bnq.LIBPATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_status_strings_and_defaults():
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    L = bnq.lib()
    assert L.bnq_status_string(0) == b"ok"
    assert L.bnq_status_string(-1) == b"invalid argument"
    p = bnq._Params()
    L.bnq_params_default(ctypes.byref(p))
    assert (p.d, p.N, p.eps, p.terms) == (3, 16, 0, 7)
    assert p.hbar == 1.0 and p.L == 8.0


@pytest.mark.parametrize("kw", [dict(d=4), dict(N=7), dict(N=0), dict(N=66), dict(eps=2), dict(L=-1.0),
                                dict(precision=3), dict(terms=9), dict(correction=5)])
def test_invalid_params_rejected_on_host(kw):
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    p = bnq.Params(d=2, N=8, L=4.0)
    for k, v in kw.items():
        setattr(p, k, v)
    with pytest.raises(bnq.BnqError) as e:
        bnq.footprint(p)
    assert e.value.status in (bnq.BNQ_EINVAL, bnq.BNQ_ENOTSUP)


def test_footprint_sizes():
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    plan_b, tab_b = bnq.footprint(bnq.Params(d=3, N=32, L=8.0))
    # pair-weight tables 2 N^6 doubles plus the trilinear rows
    assert tab_b > 2 * 32 ** 6 * 8
    assert tab_b < 40e9
    assert plan_b > 0


def test_footprint_3d48_fp32_tables_fit_one_gpu():
    # 3-D N = 48: 19600 canonical trilinear rows of (2N-1)^2 (2N-1 + pad)
    # values plus two N^6 pair-weight tables.  Only the FP32 set fits the
    # 288 GB of one MI355X.
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    N = 48
    plan32, tab32 = bnq.footprint(bnq.Params(d=3, N=N, L=8.0, precision=bnq.FP32C))
    plan64, tab64 = bnq.footprint(bnq.Params(d=3, N=N, L=8.0))
    vals_lo = 19600 * (2 * N - 1) ** 3 + 2 * N ** 6
    vals_hi = 19600 * (2 * N - 1) ** 2 * (2 * N - 1 + 32) + 2 * N ** 6
    radial = tab64 - 2 * (tab64 - tab32)  # bytes shared by both precisions
    assert 0 < radial < 1e8
    assert 4 * vals_lo <= tab32 - radial <= 4 * vals_hi
    assert tab64 - radial == 2 * (tab32 - radial)
    assert tab32 + plan32 < 250e9 < 288e9 < tab64


def test_weights_on_the_fly_flag():
    # FP64 only; the 3-D N = 48 FP64 set without weight tables fits one GPU
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    with pytest.raises(bnq.BnqError) as e:
        bnq.footprint(bnq.Params(d=2, N=8, L=4.0, flags=8))  # no such flag
    assert e.value.status == bnq.BNQ_EINVAL
    with pytest.raises(bnq.BnqError) as e:
        bnq.footprint(bnq.Params(d=2, N=8, L=4.0, precision=bnq.FP32C, flags=bnq.FLAG_WEIGHTS_OTF))
    assert e.value.status == bnq.BNQ_ENOTSUP
    _, full = bnq.footprint(bnq.Params(d=3, N=48, L=8.0))
    _, rows = bnq.footprint(bnq.Params(d=3, N=48, L=8.0, flags=bnq.FLAG_WEIGHTS_OTF))
    assert full - rows == 2 * 48 ** 6 * 8
    assert rows < 180e9


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(bnq, "LIBPATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(bnq, "_lib", None)
    with pytest.raises(RuntimeError):
        bnq.lib()


def test_separated_route_flag():
    # FP64, d = 2 with N <= 32 or d = 3 with N <= 8; its workspace is counted in the plan bytes
    if not os.path.exists(bnq.LIBPATH):
        pytest.skip("libbnq.so not built")
    for kw in (dict(d=3, N=10, angles=2), dict(d=2, N=34), dict(d=2, N=8, precision=bnq.FP32C)):
        with pytest.raises(bnq.BnqError) as e:
            bnq.footprint(bnq.Params(L=4.0, flags=bnq.FLAG_T1_SEPARATED, **kw))
        assert e.value.status == bnq.BNQ_ENOTSUP
    with pytest.raises(bnq.BnqError) as e:  # 3-D needs an explicit angle count, at most 64
        bnq.footprint(bnq.Params(d=3, N=8, L=4.0, flags=bnq.FLAG_T1_SEPARATED))
    assert e.value.status == bnq.BNQ_EINVAL
    with pytest.raises(bnq.BnqError) as e:
        bnq.footprint(bnq.Params(d=3, N=8, L=4.0, flags=bnq.FLAG_T1_SEPARATED, angles=65))
    assert e.value.status == bnq.BNQ_EINVAL
    bnq.footprint(bnq.Params(d=3, N=8, L=4.0, flags=bnq.FLAG_T1_SEPARATED, angles=64))
    for bad in (dict(angles=5), dict(angles=-1, flags=bnq.FLAG_T1_SEPARATED),
                dict(angles=5000, flags=bnq.FLAG_T1_SEPARATED)):
        with pytest.raises(bnq.BnqError) as e:
            bnq.footprint(bnq.Params(d=2, N=8, L=4.0, **bad))
        assert e.value.status == bnq.BNQ_EINVAL
    base, _ = bnq.footprint(bnq.Params(d=2, N=32, L=4.0))
    sep, _ = bnq.footprint(bnq.Params(d=2, N=32, L=4.0, flags=bnq.FLAG_T1_SEPARATED, angles=100))
    # alpha rows, their transforms, the doubled-grid spectrum and >= 2048 partial arrays
    assert sep - base >= 8 * 2 * 100 * 63 ** 2 + 16 * (100 * 64 ** 2 + 64 ** 2 + 2048 * 32 ** 2)
