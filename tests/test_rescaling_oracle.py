"""The oracle of the velocity-rescaled scheme, pinned (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from oracle import equilibrium as oe
from oracle import rescaling as rs


def _gauss(d, N, sig, shift):
    xi = rs.xi_grid(d, N)
    r2 = np.sum((xi - np.asarray(shift)) ** 2, axis=-1)
    return np.exp(-r2 / (2 * sig ** 2)), xi


@pytest.mark.parametrize("d", [2, 3])
def test_drift_is_the_divergence_of_a_decayed_gaussian(d):
    # div((a xi - b) G) = G [d a - sum_i (a xi_i - b_i)(xi_i - c_i) / sig^2]
    # for G = exp(-|xi - c|^2 / 2 sig^2): ~1e-14 at the box edge, spectrum
    # ~1e-12 at the Nyquist wavenumber
    N, sig = 48 if d == 2 else 40, 0.38
    c = [0.2, -0.1, 0.05][:d]
    G, xi = _gauss(d, N, sig, c)
    a, b = 0.7, np.array([0.3, -0.2, 0.1][:d])
    exact = G * (d * a - np.sum((a * xi - b) * (xi - np.asarray(c)), axis=-1) / sig ** 2)
    got = rs.drift(G, a, b)
    assert np.max(np.abs(got - exact)) <= 1e-9 * np.max(np.abs(exact))


def test_drift_has_zero_mean():
    rng = np.random.default_rng(3)
    G = rng.random((12, 12, 12))
    assert abs(rs.drift(G, 1.3, np.array([0.4, -0.7, 0.2])).sum()) < 1e-12 * np.abs(G).sum()


@pytest.mark.parametrize("d,N,eps", [(2, 8, 1), (2, 8, -1), (3, 6, -1), (3, 6, 0)])
def test_rescaled_operator_is_the_plain_one_on_the_scaled_box(d, N, eps):
    # eq. rescaling_collision on the grid: with f = s^d G and the box of
    # half-width L / omega, c (L/(pi omega))^(d+gamma) Q_alpha(f) equals
    # s^d c s^-gamma Q_{alpha s^d}(G); two plain evaluations, no shared arithmetic
    rng = np.random.default_rng(N)
    o = oracle.Oracle(d, N)
    L, omega, hbar, c = 5.0, 1.7, 1.3, 0.8
    s = math.pi * omega / L
    G = 0.3 * rng.random((N,) * d)
    f = s ** d * G
    lhs = o.collide(f, eps, L / omega, hbar, c)[0]
    rhs = s ** d * rs.rescaled_operator(o, G, eps, L, omega, hbar, c)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))


@pytest.mark.parametrize("eps", [-1, 1, 0])
def test_rescaled_equilibrium_stays_put(eps):
    # G = the limit state written in xi (omega = sqrt(T), centred on u): one
    # Euler step keeps rho exactly, u, e and omega to the operator's
    # residual, and G to dt times it
    d, N, L, hbar = 2, 16, 4.0, 1.0
    rho, u, e = 1.0, np.array([0.2, -0.1]), 0.5
    lim = oe.solve(d, eps, hbar, rho, u, e)
    omega = math.sqrt(lim["T"]) if eps != 0 else math.sqrt(lim["T"] + float(u @ u) / d)
    s = math.pi * omega / L
    xi = rs.xi_grid(d, N)
    v = xi / s + u
    r2 = np.sum((v - u) ** 2, axis=-1)
    if eps == 0:
        f = rho * (2 * math.pi * lim["T"]) ** (-d / 2) * np.exp(-r2 / (2 * lim["T"]))
    else:
        al = -eps * hbar ** d
        f = 1.0 / abs(al) / (np.exp(r2 / (2 * lim["T"]) - lim["log_z"]) + math.copysign(1.0, al))
    G = f / s ** d
    m = rs.moments_of(G, L, omega, u)
    st = {"rho": m["rho"], "u": m["u"], "e": m["e"], "omega": omega}
    o = oracle.Oracle(d, N)
    G1, st1 = rs.euler_step(o, G, st, 0.01, eps, L, hbar)
    assert st1["rho"] == pytest.approx(st["rho"], rel=1e-13)
    assert st1["omega"] == pytest.approx(omega, rel=1e-3)
    assert np.max(np.abs(G1 - G)) <= 1e-3 * np.max(G)
