"""The relaxation experiment's runner on the GPU (short runs): below the
threshold the entropy does not increase and the state approaches the limit
the library solves; above it (the ball datum exceeds the Fermi bound of the
larger hbar) the step health flags stop the run."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bnq = pytest.importorskip("paper_2110_13735_amd")


def test_relaxation_below_threshold():
    from paper_2110_13735_amd import relaxation as R
    res = R.run("fd2-maxwellian", 0.5, 16, steps=40, every=10)
    assert res["status"] == "completed" and res["H_nonincreasing"]
    tr = res["track"]
    assert len(tr) == 5 and tr[-1]["l1"] < tr[0]["l1"]
    assert abs(tr[-1]["rho"] - tr[0]["rho"]) <= 1e-10 * tr[0]["rho"]


def test_relaxation_above_threshold_stops():
    from paper_2110_13735_amd import relaxation as R
    res = R.run("fd2-ball", 1.05, 16, steps=40, every=10)
    assert res["f0_max"] > res["bound"]
    assert res["status"] == "stopped" and res["stop_reason"] == "Fermi-Dirac bound reached"
    assert res["stop_step"] <= 10


def test_relaxation_without_the_bound_check_runs_on():
    from paper_2110_13735_amd import relaxation as R
    res = R.run("fd2-ball", 1.05, 16, steps=20, every=10, fermi_bound=False)
    assert res["f0_max"] > res["bound"]
    assert res["status"] == "completed" and len(res["track"]) == 3
    assert all(x["fmax"] > res["bound"] for x in res["track"])
