"""The relaxation experiment's host logic: the thresholds hbar* of the
Maxwellian data against the values the paper prints (tests/golden/
relaxation_thresholds.txt, section 'Relaxation towards equilibrium'), and the
initial data's moments."""
import math
import os

import numpy as np
import pytest

import bnq_inputs as inp
from paper_2110_13735_amd import relaxation as R

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "relaxation_thresholds.txt")


def _rows():
    out = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            case, d, N, L, q, val, digits = line.split()
            out.append((case, int(d), int(N), float(L), q, float(val), int(digits)))
    return out


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"{r[0]}-{r[4]}")
def test_printed_thresholds(row):
    case, d, N, L, q, val, digits = row
    dd, eps, kind, _, _, _ = R.CASES[case]
    assert dd == d
    f0 = inp.relaxation_datum(kind, d, N, L)
    m = R.discrete_moments(f0, d, N, L)
    hs = R.hbar_star(d, eps, m["rho"], m["e"])
    got = {"hbar_star": hs, "inv_hbar_star_d": hs ** -d, "f0_max": float(f0.max())}[q]
    # agreement to the printed significant digits (half a unit of the last one)
    tol = 0.5 * 10.0 ** (math.floor(math.log10(abs(val))) - digits + 1)
    assert abs(got - val) <= tol, (got, val)


def test_ball_data_have_the_stated_moments():
    # a fine grid: the indicator data carry mass 1 and internal energy 1, and
    # their maximum is hbar*^-d (the Fermi-Dirac saturation threshold)
    for d, N, L in ((2, 512, 8.0), (3, 128, 6.0)):
        f0 = inp.relaxation_datum("ball", d, N, L)
        m = R.discrete_moments(f0, d, N, L)
        assert abs(m["rho"] - 1.0) < 2e-2 and abs(m["e"] - 1.0) < 3e-2
        hs = R.hbar_star(d, -1, 1.0, 1.0)
        assert math.isclose(float(f0.max()), hs ** -d, rel_tol=1e-12)


def test_threshold_formulas():
    # Fermi-Dirac: hbar*^d = K_d (4 pi e / d)^(d/2) / rho; the limit at hbar* is
    # the saturated ball of height hbar*^-d whose mass is rho
    for d in (2, 3):
        rho, e = 1.7, 0.8
        hs = R.hbar_star(d, -1, rho, e)
        A = math.sqrt(2.0 * e * (d + 2) / d)  # the ball radius of the section's chi
        vol = math.pi * A * A if d == 2 else 4.0 * math.pi * A ** 3 / 3.0
        assert math.isclose(vol * hs ** -d, rho, rel_tol=1e-12)
    # Bose-Einstein 3-D: at hbar*, rho = (2 pi T)^(3/2) zeta(3/2) / hbar^3 with
    # T = 2 e zeta(3/2) / (3 zeta(5/2)) (critical density for the energy)
    rho, e = 2.3, 0.7
    hs = R.hbar_star(3, 1, rho, e)
    T = 2.0 * e * R.ZETA_32 / (3.0 * R.ZETA_52)
    assert math.isclose((2 * math.pi * T) ** 1.5 * R.ZETA_32 / hs ** 3, rho, rel_tol=1e-12)
    with pytest.raises(ValueError):
        R.hbar_star(2, 1, 1.0, 1.0)
