"""Brute-force evaluation of the truncated collision operator in physical space.

Used only to pin the oracle's Galerkin sums.  It evaluates, for the
trigonometric interpolant G_N(xi) = sum_{k in I_N} G_k e^{i k.xi},

    Q^R(G)(xi) = int_{B(0,R)^2} Btilde(x,y) delta(x.y) [ ... ] dx dy

(the truncated operator of section 'Truncation and periodization of the BNE operator' with the Filbet–Hu–Jin indicator) by
plain quadrature over x, y, on an oversampled xi grid, then takes the Fourier
modes n in I_N of the result.  Q^R(G_N) is a trigonometric polynomial with
frequencies in {-3N/2, ..., 3N/2 - 3}^d, so a grid of 3N points per axis
recovers its modes in I_N exactly (no aliasing).

The delta(x.y) constraint is resolved in polar coordinates:
  d = 2, Btilde = 2 C_phi:
     int dtheta in [0, 2pi) int_0^R drho int_{-R}^{R} drho'   F(rho e_t, rho' e_{t+pi/2})
  d = 3, Btilde = 4 C_phi:
     int_{S^2} de int_0^pi dpsi int_0^R rho drho int_{-R}^{R} |rho'| drho'
         F(rho e, rho' (cos psi u1 + sin psi u2)),   (u1, u2) a basis of e-perp.
The bracket is returned split into its classical gain part
    G(xi+x) G(xi+y),
its classical part
    G(xi+x) G(xi+y) - G(xi) G(xi+x+y)
and its cubic part
    G(xi+x)G(xi+y)G(xi+x+y) + G(xi)G(xi+x)G(xi+y)
      - G(xi)G(xi+x+y)G(xi+x) - G(xi)G(xi+x+y)G(xi+y),
so that Q^R = classical - alpha * cubic.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.legendre import leggauss


def _grid_phases(N: int, M: int, d: int):
    k = np.arange(-(N // 2), N // 2)
    xi = 2 * math.pi * np.arange(-(M // 2), M // 2) / M
    E = np.exp(1j * np.outer(k, xi))  # (N, M)
    return k, xi, E


def _eval_shifted(Ghat: np.ndarray, shifts: np.ndarray, k: np.ndarray, E: np.ndarray) -> np.ndarray:
    """G_N(xi + w) on the M^d grid for each shift w (S, d) -> (S, M, ..., M)."""
    d = Ghat.ndim
    S = shifts.shape[0]
    ph = [np.exp(1j * shifts[:, i:i + 1] * k[None, :]) for i in range(d)]  # (S, N) each
    if d == 2:
        A = Ghat[None] * ph[0][:, :, None] * ph[1][:, None, :]
        return np.einsum("ax,sab,by->sxy", E, A, E, optimize=True)
    A = Ghat[None] * ph[0][:, :, None, None] * ph[1][:, None, :, None] * ph[2][:, None, None, :]
    T = np.einsum("ax,sabc->sxbc", E, A, optimize=True)
    T = np.einsum("by,sxbc->sxyc", E, T, optimize=True)
    return np.einsum("cz,sxyc->sxyz", E, T, optimize=True)


def _modes_of(Q: np.ndarray, N: int, M: int) -> np.ndarray:
    d = Q.ndim
    j = np.arange(-(M // 2), M // 2)
    k = np.arange(-(N // 2), N // 2)
    F = np.exp(-2j * math.pi * np.outer(k, j) / M) / M
    out = Q
    for ax in range(d):
        out = np.moveaxis(np.tensordot(F, out, axes=([1], [ax])), 0, ax)
    return out


def bruteforce_modes(Ghat: np.ndarray, R: float, Cphi: float = 1.0, nodes=None, gain: bool = False):
    """Return (classical modes, cubic modes) on I_N from physical-space
    quadrature (and the classical gain modes when gain=True).  `nodes`
    overrides the default node counts."""
    d, N = Ghat.ndim, Ghat.shape[0]
    M = 3 * N
    k, xi, E = _grid_phases(N, M, d)
    G0 = _eval_shifted(Ghat, np.zeros((1, d)), k, E)[0]
    Qc = np.zeros((M,) * d, dtype=np.complex128)
    Qq = np.zeros((M,) * d, dtype=np.complex128)
    Qg = np.zeros((M,) * d, dtype=np.complex128)

    def accumulate(X, Y, w):
        """X: (A, d) first shifts, Y: (B, d) second shifts, w: (A, B) weights."""
        nonlocal Qc, Qq, Qg
        GX = _eval_shifted(Ghat, X, k, E)
        GY = _eval_shifted(Ghat, Y, k, E)
        XY = (X[:, None, :] + Y[None, :, :]).reshape(-1, d)
        GXY = _eval_shifted(Ghat, XY, k, E).reshape((X.shape[0], Y.shape[0]) + (M,) * d)
        ww = w.reshape(w.shape + (1,) * d)
        gx = GX[:, None]
        gy = GY[None, :]
        Qg += np.sum(ww * (gx * gy), axis=(0, 1))
        Qc += np.sum(ww * (gx * gy - G0 * GXY), axis=(0, 1))
        Qq += np.sum(ww * (gx * gy * GXY + G0 * gx * gy - G0 * GXY * gx - G0 * GXY * gy), axis=(0, 1))

    if d == 2:
        nth, nr = nodes if nodes else (64, 24)
        t, w = leggauss(nr)
        rho, wr = R * (t + 1) / 2, w * R / 2
        rhop = np.concatenate([-rho[::-1], rho])
        wrp = np.concatenate([wr[::-1], wr])
        for i in range(nth):
            th = 2 * math.pi * i / nth
            e = np.array([math.cos(th), math.sin(th)])
            ep = np.array([-math.sin(th), math.cos(th)])
            accumulate(rho[:, None] * e[None], rhop[:, None] * ep[None],
                       2 * Cphi * (2 * math.pi / nth) * wr[:, None] * wrp[None, :])
    else:
        nt, nph, nps, nr = nodes if nodes else (12, 20, 14, 10)
        tt, wt = leggauss(nt)
        t, w = leggauss(nr)
        rho, wr = R * (t + 1) / 2, w * R / 2
        rhop = np.concatenate([-rho[::-1], rho])
        wrp = np.concatenate([wr[::-1], wr]) * np.abs(rhop)
        for a in range(nt):
            ct = tt[a]
            st = math.sqrt(1 - ct * ct)
            for b in range(nph):
                ph = 2 * math.pi * b / nph
                e = np.array([st * math.cos(ph), st * math.sin(ph), ct])
                u1 = np.array([math.cos(ph) * ct, math.sin(ph) * ct, -st])
                u2 = np.cross(e, u1)
                wsph = wt[a] * (2 * math.pi / nph)
                for c in range(nps):
                    ps = math.pi * c / nps
                    ep = math.cos(ps) * u1 + math.sin(ps) * u2
                    accumulate(rho[:, None] * e[None], rhop[:, None] * ep[None],
                               4 * Cphi * wsph * (math.pi / nps) * (wr * rho)[:, None] * wrp[None, :])
    if gain:
        return _modes_of(Qc, N, M), _modes_of(Qq, N, M), _modes_of(Qg, N, M)
    return _modes_of(Qc, N, M), _modes_of(Qq, N, M)
