"""Seeded synthetic inputs for the homogeneous Boltzmann–Nordheim solver.

This module is shared by the CPU oracle and the GPU path.  It only builds
initial data on the velocity grid; it holds none of the collision operator's
arithmetic (no Fourier transforms, no kernel modes, no sums).

Velocity grid (section 'Numerical scheme for the velocity rescaled BNE', classical method with omega = 1):
    v_j = 2 L j / N,   j in I_N = {-N/2, ..., N/2 - 1}^d,   Delta v = (2L/N)^d.
Arrays are numpy float64 of shape (N,)*d in C order; storage index = j + N/2.

Initial data are sampled on the whole box [-L, L)^d, as the spectral-accuracy
tests of section 'Validation of spectral accuracy' require (their residuals decay to 1e-8 at 64^2, which a
cut inside the box would prevent).  Where a recipe asks for a compact support,
the datum is cut at |v| <= R_v = 2 L / (3 + sqrt 2), the velocity image of the
radius S fixed by R = S, pi = (3 + sqrt 2) S / 2 (section 'Validation of spectral accuracy').

Every generator takes an explicit seed and draws from numpy's PCG64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "support_radius", "velocity_axes", "velocity_grid", "cell_volume",
    "two_gaussians_2d", "fermion_mixture_3d", "boson_condensing_3d",
    "gaussian_mixture", "sparse_spectrum", "bkw_2d", "quantum_maxwellian",
]

SQRT2 = math.sqrt(2.0)


def support_radius(L: float) -> float:
    """R_v = 2L/(3+sqrt 2): velocity radius that maps onto the xi-radius S."""
    return 2.0 * L / (3.0 + SQRT2)


def velocity_axes(N: int, L: float) -> np.ndarray:
    """1-D velocity nodes 2 L j / N for j = -N/2 .. N/2-1."""
    j = np.arange(-N // 2, N // 2, dtype=np.float64)
    return 2.0 * L * j / N


def velocity_grid(d: int, N: int, L: float) -> np.ndarray:
    """Array of shape (N,)*d + (d,) with the velocity of every node."""
    ax = velocity_axes(N, L)
    mesh = np.meshgrid(*([ax] * d), indexing="ij")
    return np.stack(mesh, axis=-1)


def cell_volume(d: int, N: int, L: float) -> float:
    return (2.0 * L / N) ** d


def _truncate(f: np.ndarray, v: np.ndarray, L: float) -> np.ndarray:
    r2 = np.sum(v * v, axis=-1)
    out = np.where(r2 <= support_radius(L) ** 2, f, 0.0)
    return np.ascontiguousarray(out, dtype=np.float64)


def _normalise_mass(f: np.ndarray, d: int, N: int, L: float, mass: float) -> np.ndarray:
    m = cell_volume(d, N, L) * float(np.sum(f))
    return f * (mass / m)


def two_gaussians_2d(N: int = 32, R_v: float = 4.0, var: float = 0.5,
                     centre: float = 1.5, mass: float = 1.0):
    """2-D boson test datum: two isotropic Gaussians at (+-centre, 0) with the
    given per-component variance, cut at |v| <= R_v and scaled to discrete
    mass 1.  Returns (f0, L) with L = (3 + sqrt 2) R_v / 2."""
    L = (3.0 + SQRT2) * R_v / 2.0
    v = velocity_grid(2, N, L)
    g = np.zeros(v.shape[:-1])
    for s in (+1.0, -1.0):
        c = np.array([s * centre, 0.0])
        g += np.exp(-np.sum((v - c) ** 2, axis=-1) / (2.0 * var))
    f = _truncate(g, v, L)
    return _normalise_mass(f, 2, N, L, mass), L


def _uniform_ball(rng: np.random.Generator, d: int, radius: float) -> np.ndarray:
    while True:
        c = rng.uniform(-radius, radius, size=d)
        if float(c @ c) <= radius * radius:
            return c


def fermion_mixture_3d(N: int = 32, L: float = 8.0, seed: int = 0,
                       amp: float = 0.45, cap: float = 0.99, ncomp: int = 3, truncate: bool = False):
    """3-D fermion datum: amp * sum of ncomp Gaussians exp(-|v-c_i|^2/(2 s_i))
    with centres uniform in |v| <= 2 and s_i ~ U[0.3, 1], capped at `cap`
    (below the Fermi bound 1/|alpha| = 1 for hbar = 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cs = [_uniform_ball(rng, 3, 2.0) for _ in range(ncomp)]
    ss = [rng.uniform(0.3, 1.0) for _ in range(ncomp)]
    v = velocity_grid(3, N, L)
    g = np.zeros(v.shape[:-1])
    for c, s in zip(cs, ss):
        g += np.exp(-np.sum((v - c) ** 2, axis=-1) / (2.0 * s))
    f = np.minimum(amp * g, cap)
    return _truncate(f, v, L) if truncate else np.ascontiguousarray(f)


def boson_condensing_3d(N: int = 32, L: float = 3.0, T: float = 0.2, amp: float = 10.6):
    """3-D boson datum a * exp(-|v|^2 / T)."""
    v = velocity_grid(3, N, L)
    return np.ascontiguousarray(amp * np.exp(-np.sum(v * v, axis=-1) / T))


def gaussian_mixture(d: int, N: int, L: float, seed: int, kmin: int = 1, kmax: int = 4,
                     centre_radius: float = 1.5, var_lo: float = 0.2, var_hi: float = 1.0,
                     mass: float = 1.0, fmax: float | None = None, truncate: bool = False):
    """Mixture of K ~ U{kmin..kmax} isotropic Gaussians with Dirichlet(1)
    weights, centres uniform in |v| <= centre_radius, per-component variance
    U[var_lo, var_hi]; scaled to discrete mass `mass` (optionally cut at R_v
    first).  If fmax is given the datum is then scaled down so that
    max f < fmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = int(rng.integers(kmin, kmax + 1))
    w = rng.dirichlet(np.ones(K))
    v = velocity_grid(d, N, L)
    g = np.zeros(v.shape[:-1])
    for i in range(K):
        c = _uniform_ball(rng, d, centre_radius)
        s = rng.uniform(var_lo, var_hi)
        g += w[i] * np.exp(-np.sum((v - c) ** 2, axis=-1) / (2.0 * s)) / (2 * math.pi * s) ** (d / 2)
    g = _truncate(g, v, L) if truncate else g
    f = _normalise_mass(g, d, N, L, mass)
    if fmax is not None:
        m = float(f.max())
        if m >= fmax:
            f = f * (0.98 * fmax / m)
    return f


def mixed_instance(d: int, N: int, eps: int, seed: int):
    """One instance of the mixed batch/serving workloads: a mixture of
    K ~ U{1..4} isotropic Gaussians (Dirichlet(1) weights, centres uniform in
    |v| <= 1.5, variances U[0.2, 1], mass 1) on a box sized to the draw,
    L = (3 + sqrt 2)/2 (max|c| + 4 sqrt(max s)); fermion data (eps = -1) are
    scaled so that max f < 0.98.  Returns (f, L)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = int(rng.integers(1, 5))
    w = rng.dirichlet(np.ones(K))
    cs = [_uniform_ball(rng, d, 1.5) for _ in range(K)]
    ss = [float(rng.uniform(0.2, 1.0)) for _ in range(K)]
    L = (3.0 + math.sqrt(2.0)) / 2.0 * (max(float(np.linalg.norm(c)) for c in cs) + 4.0 * math.sqrt(max(ss)))
    v = velocity_grid(d, N, L)
    g = np.zeros(v.shape[:-1])
    for wi, c, s in zip(w, cs, ss):
        g += wi * np.exp(-np.sum((v - c) ** 2, axis=-1) / (2.0 * s)) / (2 * math.pi * s) ** (d / 2)
    f = _normalise_mass(g, d, N, L, 1.0)
    if eps == -1 and float(f.max()) >= 0.98:
        f = f * (0.97 / float(f.max()))
    return np.ascontiguousarray(f), L


def sparse_spectrum(d: int, N: int, seed: int, nmodes: int, amp: float = 1.0):
    """Real grid function with a sparse Fourier spectrum.

    Draws `nmodes` distinct wave vectors k in I_N with no component equal to
    -N/2 (so that -k is also in I_N) and k != 0, plus the mode 0, with complex
    amplitudes c_k; returns (f, modes, coeffs) where
        f_j = sum_k c_k e^{2 pi i k.j/N} + conj,   (mode 0 real, counted once)
    so that the exact discrete spectrum is c_k at k and conj(c_k) at -k.
    `modes` is an (M, d) int array and `coeffs` the matching complex amplitudes
    (both k and -k listed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = N // 2
    chosen = {}
    while len(chosen) < nmodes:
        k = tuple(int(x) for x in rng.integers(-h + 1, h, size=d))
        if all(x == 0 for x in k):
            continue
        mk = tuple(-x for x in k)
        if k in chosen or mk in chosen:
            continue
        chosen[k] = complex(rng.normal(), rng.normal()) * amp
    modes = [tuple([0] * d)]
    coeffs = [complex(rng.normal() * amp, 0.0)]
    for k, c in chosen.items():
        modes.append(k)
        coeffs.append(c)
        modes.append(tuple(-x for x in k))
        coeffs.append(c.conjugate())
    modes = np.array(modes, dtype=np.int64)
    coeffs = np.array(coeffs, dtype=np.complex128)
    j = np.arange(-h, h)
    grids = np.meshgrid(*([j] * d), indexing="ij")
    f = np.zeros((N,) * d, dtype=np.complex128)
    for k, c in zip(modes, coeffs):
        phase = sum(int(k[i]) * grids[i] for i in range(d))
        f += c * np.exp(2j * math.pi * phase / N)
    return np.ascontiguousarray(f.real), modes, coeffs


def bkw_2d(N: int, L: float, t: float, lam: float, truncate: bool = False):
    """Bobylev / Krook–Wu self-similar solution of the classical 2-D Maxwell
    molecule equation (mass 1, temperature 1):
        f = exp(-v^2/(2K)) / (2 pi K^2) * (2K - 1 + (1 - K) v^2 / (2K)),
        K = 1 - exp(-lam t) / 2.
    The rate `lam` depends on the collision kernel and is supplied by the
    caller."""
    K = 1.0 - 0.5 * math.exp(-lam * t)
    v = velocity_grid(2, N, L)
    r2 = np.sum(v * v, axis=-1)
    f = np.exp(-r2 / (2 * K)) / (2 * math.pi * K * K) * (2 * K - 1 + (1 - K) * r2 / (2 * K))
    return _truncate(f, v, L) if truncate else np.ascontiguousarray(f)


def quantum_maxwellian(d: int, N: int, L: float, z: float, T: float, alpha: float,
                       u=None, truncate: bool = False):
    """Quantum Maxwellian of section 'Convergence towards a steady state':
        M_q(v) = (1/|alpha|) / ( z^{-1} exp(|v-u|^2 / (2T)) + sgn(alpha) ),
    alpha = +hbar^d (Fermi–Dirac) or -hbar^d (Bose–Einstein, needs 0 < z < 1).
    Returned on the grid (optionally cut at R_v)."""
    v = velocity_grid(d, N, L)
    w = v if u is None else v - np.asarray(u, dtype=np.float64)
    r2 = np.sum(w * w, axis=-1)
    f = (1.0 / abs(alpha)) / (np.exp(r2 / (2 * T)) / z + math.copysign(1.0, alpha))
    if truncate:
        return _truncate(f, v, L)
    return np.ascontiguousarray(f)


def relaxation_datum(kind: str, d: int, N: int, L: float, rho: float = 1.0, e: float = 1.0, sigma: float = 1.0):
    """Initial data of 'Relaxation towards equilibrium' (mean velocity 0):
      'ball'      the indicator datum, rho / |B(0, A)| on the ball of radius
                  A = 2 sqrt(e) (2-D, eq. fermions_2d_init_indicator) or
                  A = sqrt(10 e / 3) (3-D, eq. fermions_3d_init_cmax), so that
                  its internal energy (half the second moment per particle) is e;
      'maxwellian' rho / (2 pi sigma)^(d/2) exp(-|v|^2 / (2 sigma)) (eqs.
                  fermions_2d_init_cmax, fermions_3d_init_ball).
    The paper gives rho = sigma = 1 for the Maxwellian and leaves rho, e of the
    ball unstated; rho = e = 1 here."""
    v = velocity_grid(d, N, L)
    r2 = np.sum(v * v, axis=-1)
    if kind == "ball":
        A = 2.0 * math.sqrt(e) if d == 2 else math.sqrt(10.0 * e / 3.0)
        vol = math.pi * A * A if d == 2 else 4.0 * math.pi * A ** 3 / 3.0
        f = np.where(r2 <= A * A, rho / vol, 0.0)
    elif kind == "maxwellian":
        f = rho / (2.0 * math.pi * sigma) ** (d / 2.0) * np.exp(-r2 / (2.0 * sigma))
    else:
        raise ValueError(f"unknown relaxation datum {kind!r}")
    return np.ascontiguousarray(f, dtype=np.float64)
