"""Oracle for the velocity-rescaled scheme of the space-homogeneous equation.

TEST INFRASTRUCTURE ONLY (like the rest of this package): only tests/, the
smoke check and the CPU-baseline leg of the benchmark may import it.

Sections 'A rescaling velocity model of the BNE' and 'Numerical scheme for
the velocity rescaled BNE' with lambda = 1, mu = 1: the distribution is held
as G on the fixed grid xi_j = 2 pi j / N (j in I_N) of [-pi, pi)^d, with

    f(v) = s^d G(xi),   xi = s (v - u),   s = pi omega / L,

so f lives on u + [-L/omega, L/omega)^d.  One forward Euler step (the
scheme's steps 1-5, in its order):

  2. K = c s^-gamma Q^R_{alpha s^d}(G) on the grid (the operator with the
     quantum parameter alpha s^d);
  3. (a) rho, rho u, rho e advanced by dt times the sums of K against
         1, L xi / (pi omega) + u, |L xi / (pi omega)|^2 / 2, weight
         Delta xi = (2 pi / N)^d;
     (b) T from the limit state of the new moments (oracle.equilibrium);
     (c) omega = sqrt(T) (alpha != 0) or sqrt(T + |u|^2 / d) (alpha = 0);
  4. the drift div_xi((a xi - b) G), a = (omega' - omega) / (dt omega),
     b = s (u' - u) / dt, by spectral differentiation (FFT);
  5. G' = G + dt (K - drift).

Pinned in tests/test_rescaling_oracle.py: the spectral drift against the
analytic divergence of a Gaussian, its zero mean, the homogeneity identity
of the rescaled operator (eq. rescaling_collision) between two plain oracle
evaluations, and a rescaled Maxwellian staying put under a step.
"""
from __future__ import annotations

import math

import numpy as np

from . import Oracle, gamma_of, modes
from . import equilibrium as oeq


def xi_axes(N: int) -> np.ndarray:
    return 2.0 * math.pi * modes(N) / N


def xi_grid(d: int, N: int) -> np.ndarray:
    ax = xi_axes(N)
    return np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1)


def drift(G: np.ndarray, a: float, b) -> np.ndarray:
    """div_xi((a xi - b) G) by spectral differentiation along each axis:
    Re IFFT(i k FFT(.)) with integer wavenumbers k in I_N (the Nyquist
    mode's derivative is imaginary and dropped by the real part)."""
    d, N = G.ndim, G.shape[0]
    xi = xi_grid(d, N)
    k = np.fft.fftfreq(N, 1.0 / N)
    out = np.zeros_like(G)
    for ax in range(d):
        H = (a * xi[..., ax] - b[ax]) * G
        Hk = np.fft.fft(H, axis=ax)
        shape = [1] * d
        shape[ax] = N
        out += np.real(np.fft.ifft(1j * k.reshape(shape) * Hk, axis=ax))
    return out


def rescaled_operator(o: Oracle, G: np.ndarray, eps: int, L: float, omega: float, hbar: float = 1.0,
                      c: float = 1.0) -> np.ndarray:
    """c s^-gamma Q^R_{alpha s^d}(G), s = pi omega / L: the plain operator on
    a box of half-width pi (prefactor 1) with hbar s in place of hbar."""
    s = math.pi * omega / L
    return o.collide(G, eps, math.pi, hbar * s, c * s ** (-gamma_of(o.d)))[0]


def moments_of(G: np.ndarray, L: float, omega: float, u_ref) -> dict:
    """rho, u, e of f = s^d G on u_ref + [-L/omega, L/omega)^d."""
    d, N = G.ndim, G.shape[0]
    dxi = (2.0 * math.pi / N) ** d
    w = L / (math.pi * omega) * xi_grid(d, N) + np.asarray(u_ref, dtype=np.float64)
    rho = dxi * G.sum()
    u = dxi * np.sum(w * G[..., None], axis=tuple(range(d))) / rho
    e = dxi * np.sum(np.sum((w - u) ** 2, axis=-1) * G) / (2.0 * rho)
    return {"rho": rho, "u": u, "e": e}


def euler_step(o: Oracle, G: np.ndarray, st: dict, dt: float, eps: int, L: float, hbar: float = 1.0,
               c: float = 1.0):
    """One forward Euler step of the rescaled scheme.  st holds rho, u (d
    components), e, omega; returns (G', st')."""
    d, N = G.ndim, G.shape[0]
    omega, rho, u, e = st["omega"], st["rho"], np.asarray(st["u"], dtype=np.float64), st["e"]
    s = math.pi * omega / L
    K = rescaled_operator(o, G, eps, L, omega, hbar, c)
    dxi = (2.0 * math.pi / N) ** d
    w = L / (math.pi * omega) * xi_grid(d, N)
    rho1 = rho + dt * dxi * K.sum()
    u1 = (rho * u + dt * dxi * np.sum((w + u) * K[..., None], axis=tuple(range(d)))) / rho1
    e1 = (rho * e + dt * 0.5 * dxi * np.sum(np.sum(w * w, axis=-1) * K)) / rho1
    lim = oeq.solve(d, eps, hbar, rho1, u1, e1)
    if lim["kind"] in (oeq.SATURATED, oeq.UNKNOWN):
        raise ValueError("no finite temperature for the new moments")
    T1 = lim["T"]
    omega1 = math.sqrt(T1) if eps != 0 else math.sqrt(T1 + float(u1 @ u1) / d)
    a = (omega1 - omega) / (dt * omega)
    b = s * (u1 - u) / dt
    G1 = G + dt * (K - drift(G, a, b))
    return G1, {"rho": rho1, "u": u1, "e": e1, "omega": omega1, "T": T1, "log_z": lim["log_z"],
                "kind": lim["kind"]}
