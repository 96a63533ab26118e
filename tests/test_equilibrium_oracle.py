"""Limit states (section 'Convergence towards a steady state'): the oracle
pinned to closed forms, and the library's host solver held to the oracle.

No GPU: the complete Fermi-Dirac / Bose-Einstein integrals and the fugacity
solve are host code in the library (bnq_fd_be_log, bnq_equilibrium_solve).
"""
import math
import os

import numpy as np
import pytest
from scipy.special import spence, zeta

from oracle import equilibrium as oe

import paper_2110_13735_amd as bnq

needs_lib = pytest.mark.skipif(not os.path.exists(bnq.LIBPATH), reason="libbnq.so not built")


def _li2(x):
    # dilogarithm Li_2(x) for x <= 1 (scipy's spence(z) = Li_2(1 - z))
    return spence(1.0 - x)


# ---------------------------------------------------------------- oracle pins
@pytest.mark.parametrize("z", [1e-4, 0.05, 0.5, 0.9, 0.999])
def test_integrals_of_order_one_and_two_are_logs_and_dilogs(z):
    assert oe.K(1, True, z) == pytest.approx(math.log1p(z), rel=1e-13)
    assert oe.K(1, False, z) == pytest.approx(-math.log1p(-z), rel=1e-13)
    assert oe.K(2, True, z) == pytest.approx(-_li2(-z), rel=1e-12)
    assert oe.K(2, False, z) == pytest.approx(_li2(z), rel=1e-13)


@pytest.mark.parametrize("nu", [1.5, 2.0, 2.5, 3.5])
def test_bose_integral_at_z_one_is_zeta(nu):
    assert oe.K(nu, False, 1.0) == pytest.approx(zeta(nu), rel=1e-13)


@pytest.mark.parametrize("nu", [1.0, 1.5, 2.0, 2.5])
def test_classical_limit_series(nu):
    # K_nu(z) = sum_k (-+1)^(k+1) z^k / k^nu: the first terms at small z
    z = 1e-3
    fd = z - z ** 2 / 2 ** nu + z ** 3 / 3 ** nu
    be = z + z ** 2 / 2 ** nu + z ** 3 / 3 ** nu
    assert oe.K(nu, True, z) == pytest.approx(fd, rel=1e-11)
    assert oe.K(nu, False, z) == pytest.approx(be, rel=1e-11)


@pytest.mark.parametrize("nu", [1.5, 2.5])
def test_degenerate_fermi_dirac_sommerfeld(nu):
    # F_nu(e^mu) = mu^nu / Gamma(nu + 1) [1 + nu (nu - 1) pi^2 / (6 mu^2) + O(mu^-4)]
    # (the remark on F_nu; its second coefficient is read as pi^2 / 6)
    mu = 500.0
    som = mu ** nu / math.gamma(nu + 1) * (1 + nu * (nu - 1) * math.pi ** 2 / (6 * mu ** 2))
    assert oe.K(nu, True, log_z=mu) == pytest.approx(som, rel=1e-9)


def _state_moments(d, eps, z_or_logz, T, fermi):
    nu = d / 2.0
    K0 = oe.K(nu, fermi, log_z=z_or_logz)
    K1 = oe.K(nu + 1, fermi, log_z=z_or_logz)
    rho = (2 * math.pi * T) ** nu * K0  # |alpha| = 1
    e = nu * T * K1 / K0
    return rho, e


@pytest.mark.parametrize("d,eps,logz,T", [(2, -1, -3.0, 0.7), (2, -1, 4.0, 0.3), (3, -1, 0.5, 1.2),
                                          (3, -1, 25.0, 0.2), (2, 1, -0.01, 0.9), (3, 1, -0.2, 0.4),
                                          (3, 1, -4.0, 2.0)])
def test_solve_recovers_fugacity_and_temperature(d, eps, logz, T):
    fermi = eps == -1
    rho, e = _state_moments(d, eps, logz, T, fermi)
    st = oe.solve(d, eps, 1.0, rho, [0.0] * d, e)
    assert st["kind"] == oe.QUANTUM
    assert st["log_z"] == pytest.approx(logz, rel=1e-10, abs=1e-12)
    assert st["T"] == pytest.approx(T, rel=1e-10)


def test_condensate_splits_mass_and_keeps_energy():
    # beyond I_eq the 3-D Bose-Einstein state is m0 at v = u plus the z = 1
    # distribution, which carries all the internal energy (the reading of
    # eq. Tcritical_bosons_3d that keeps the energy the section conserves)
    rho, e = 20.0, 0.3
    st = oe.solve(3, 1, 1.0, rho, [0.0] * 3, e)
    assert st["kind"] == oe.CONDENSATE and st["m0"] > 0
    T = st["T"]
    reg_mass = (2 * math.pi * T) ** 1.5 * zeta(1.5)
    reg_energy = (2 * math.pi * T) ** 1.5 * 1.5 * T * zeta(2.5)  # int |v|^2 / 2 of the z = 1 part
    assert reg_mass + st["m0"] == pytest.approx(rho, rel=1e-13)
    assert reg_energy == pytest.approx(rho * e, rel=1e-13)


def test_condensate_branch_meets_the_quantum_branch_at_criticality():
    # at the critical ratio the condensate has m0 = 0 and the temperature of
    # eq. Tcritical_bosons_3d; just below it the quantum Maxwellian has z -> 1
    # and the same temperature
    e = 0.4
    rho_c = (4 * math.pi * e / 3) ** 1.5 * zeta(1.5) ** 2.5 / zeta(2.5) ** 1.5
    at = oe.solve(3, 1, 1.0, rho_c * (1 + 1e-12), [0.0] * 3, e)
    below = oe.solve(3, 1, 1.0, rho_c * (1 - 1e-9), [0.0] * 3, e)
    assert at["kind"] == oe.CONDENSATE and below["kind"] == oe.QUANTUM
    assert abs(at["m0"]) < 1e-9 * rho_c
    assert at["T"] == pytest.approx(2 * e * zeta(1.5) / (3 * zeta(2.5)), rel=1e-11)
    assert below["T"] == pytest.approx(at["T"], rel=1e-5)
    assert below["log_z"] > -1e-4


@pytest.mark.parametrize("d", [2, 3])
def test_saturated_fermi_dirac_at_the_end_of_the_range(d):
    # the indicator of the ball of radius A at height 1/|alpha| has exactly
    # the largest admissible ratio: classified saturated, beyond it unknown
    A = 1.7
    vol = math.pi ** (d / 2) * A ** d / math.gamma(d / 2 + 1)
    rho = vol
    e = d / (d + 2) * A ** 2 / 2
    st = oe.solve(d, -1, 1.0, rho, [0.0] * d, e)
    assert st["kind"] == oe.SATURATED and st["A"] == pytest.approx(A, rel=1e-14)
    assert st["ratio"] == pytest.approx(oe.ieq_upper(d, True), rel=1e-14)
    assert oe.solve(d, -1, 1.0, 1.01 * rho, [0.0] * d, e)["kind"] == oe.UNKNOWN


@pytest.mark.parametrize("eps", [-1, 0, 1])
def test_state_on_a_fine_grid_has_the_requested_moments(eps):
    # discrete moments of the state (smooth, decayed at the box edge) match
    # rho, u, e to spectral accuracy
    d, N, L = 2, 96, 9.0
    rho, u, e = 1.3, [0.3, -0.2], 0.6
    st = oe.solve(d, eps, 1.0, rho, u, e)
    M, excl = oe.on_grid(d, N, L, st)
    assert not excl.any()
    dv = (2 * L / N) ** d
    ax = 2 * L * (np.arange(N) - N // 2) / N
    v = np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1)
    m = dv * M.sum()
    uu = dv * np.sum(v * M[..., None], axis=(0, 1)) / m
    ee = dv * np.sum(np.sum((v - uu) ** 2, axis=-1) * M) / (2 * m)
    assert m == pytest.approx(rho, rel=1e-10)
    assert uu == pytest.approx(u, abs=1e-10)
    assert ee == pytest.approx(e, rel=1e-9)


# ---------------------------------------------------------------- library vs oracle
@needs_lib
@pytest.mark.parametrize("nu", [1.0, 1.5, 2.0, 2.5, 3.5])
def test_library_integrals_match_oracle(nu):
    for lz in (-30.0, -2.0, -1e-6, 0.5, 8.0, 120.0, 3000.0):
        assert bnq.fd_be_log(nu, True, lz) == pytest.approx(math.log(oe.K(nu, True, log_z=lz)), rel=1e-13,
                                                            abs=1e-13)
    for delta in (1e-9, 1e-3, 0.2, 3.0, 40.0):
        assert bnq.fd_be_log(nu, False, delta) == pytest.approx(math.log(oe.K(nu, False, log_z=-delta)),
                                                                rel=1e-13, abs=1e-13)


@needs_lib
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("eps", [-1, 0, 1])
def test_library_solver_matches_oracle(d, eps):
    rng = np.random.default_rng(10 * d + eps)
    for _ in range(12):
        rho = float(np.exp(rng.uniform(-2.0, 3.5)))
        e = float(np.exp(rng.uniform(-2.0, 1.0)))
        u = rng.normal(size=d)
        hbar = float(rng.uniform(0.5, 2.0))
        ref = oe.solve(d, eps, hbar, rho, u, e)
        got = bnq.equilibrium(d, eps, hbar, rho, u, e).as_dict()
        assert got["kind"] == ref["kind"], (rho, e, hbar)
        assert got["u"][:d] == pytest.approx(list(u))
        for k in ("T", "m0", "A", "ratio"):
            assert got[k] == pytest.approx(ref[k], rel=1e-11, abs=1e-12), (k, rho, e, hbar)
        if ref["kind"] == oe.QUANTUM:
            assert got["log_z"] == pytest.approx(ref["log_z"], rel=1e-11, abs=1e-12)


@needs_lib
def test_library_solver_rejects_bad_input():
    for args in [(4, 1, 1.0, 1.0, [0, 0], 1.0), (2, 1, 1.0, -1.0, [0, 0], 1.0), (2, 1, 1.0, 1.0, [0, 0], 0.0),
                 (3, 2, 1.0, 1.0, [0, 0, 0], 1.0), (3, 1, 0.0, 1.0, [0, 0, 0], 1.0)]:
        with pytest.raises(bnq.BnqError) as e:
            bnq.equilibrium(*args)
        assert e.value.status == bnq.BNQ_EINVAL
