"""Separated kernel modes and the transform evaluation of the trilinear term.

TEST INFRASTRUCTURE ONLY: imported by tests/ alone; the product library never
imports, links or calls it.

Mouton & Rey, arXiv 2110.13735:

* section 'Fast computation of the collision modes', eq. betadD: the kernel
  modes written as a rank-P sum  beta_P(k, l) = C sum_p alpha_p(k) alpha'_p(l);
  - 2-D (eq. alphap, Maxwell molecules, Btilde = 2 C_phi): P = M angles
    theta_p = p pi / M, C = pi / M,
        alpha_p(k)  = 2 C_phi phi2(k . e_p),   alpha'_p(l) = phi2(l . e_p^perp),
        phi2(s) = 2 R sinc(R s),  e_p = (cos theta_p, sin theta_p),
        e_p^perp = (-sin theta_p, cos theta_p);
  - 3-D (eq. alphapprime, hard spheres, Btilde = 4 C_phi): P = M1 M2 directions
    e_pq = (sin t_p cos f_q, sin t_p sin f_q, cos t_p), t_p = p pi / M1,
    f_q = q pi / M2, C = pi^2 / (M1 M2),
        alpha_{q + M2 p}(k)  = 4 C_phi sin t_p phi3(k . e_pq),
        alpha'_{q + M2 p}(l) = psi(|l - (l . e_pq) e_pq|),
        phi3(s) = int_{-R}^{R} |r| e^{i r s} dr,
    with psi taken as the great-circle integral of phi3 without a sine factor,
    psi(s) = int_0^pi phi3(s cos t) dt = 2 pi R J_1(R s) / s (the reading the
    direct oracle uses; the closed form printed for hard spheres,
    2 R^2 sinc^2(R s / 2), carries the sine factor).
* appendix 'Fast evaluation of the collision kernel': with that form,
      T1_n = sum_{a,b} beta_P(a, b) G_{n-a} G_{n-b} G_{a+b-n}
           = C sum_p sum_j G_j e^{2 pi i n.j} (g_pj * G)_n (g'_pj * G)_n,
  the modulated modes (g_pj)_k = alpha_p(k) e^{-2 pi i k.j}, each convolution
  done as the transform of a product in physical space.  Reading: the
  physical grid is the doubled grid I_M, M = 2N, on which the spectrum is
  extended by zeros (so G_j below is sum_k G_k e^{2 pi i k.j/M}); on it every
  index sum that occurs stays clear of the period, and the result is the
  linear Galerkin sum.  On the N grid itself the printed identity wraps
  k + l - n modulo N.

Pins (tests/test_separated_oracle.py): the transform route against the direct
trilinear sum of liboracle run on the beta_P table (2-D and 3-D); beta_P
against the converged kernel modes (spectrally in 2-D, at the rectangle
rule's second-order rate in 3-D); a constant datum.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import R_DEFAULT, modes


def phi2(R: float, s):
    """int_{-R}^{R} e^{i r s} dr = 2 R sinc(R s)."""
    return 2.0 * R * np.sinc(R * np.asarray(s, dtype=np.float64) / math.pi)


def phi3(R: float, s):
    """int_{-R}^{R} |r| e^{i r s} dr = R^2 (2 sinc(R s) - sinc^2(R s / 2))."""
    x = R * np.asarray(s, dtype=np.float64)
    return R * R * (2.0 * np.sinc(x / math.pi) - np.sinc(x / (2.0 * math.pi)) ** 2)


def psi3(R: float, s):
    """int_0^pi phi3(s cos t) dt = 2 pi R J_1(R s) / s (pi R^2 at s = 0)."""
    x = R * np.asarray(s, dtype=np.float64)
    safe = np.where(x == 0.0, 1.0, x)
    return np.where(x == 0.0, math.pi * R * R, 2.0 * math.pi * R * R * special.j1(safe) / safe)


def box(d: int, lo: int, hi: int) -> np.ndarray:
    """Integer vectors of {lo..hi-1}^d in C order, shape (n, d)."""
    ax = np.arange(lo, hi)
    return np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1).reshape(-1, d)


def alphas(d: int, vecs, M, Cphi: float = 1.0, R: float = R_DEFAULT):
    """(C, alpha, alpha') with alpha[p, i] = alpha_p(vecs[i]); M is the angle
    count in 2-D, the pair (M1, M2) in 3-D (eqs. alphap, alphapprime)."""
    v = np.asarray(vecs, dtype=np.float64).reshape(-1, d)
    if d == 2:
        th = math.pi * np.arange(M) / M
        e = np.stack([np.cos(th), np.sin(th)], axis=1)
        ep = np.stack([-np.sin(th), np.cos(th)], axis=1)
        A = 2.0 * Cphi * phi2(R, e @ v.T)
        Ap = phi2(R, ep @ v.T)
        return math.pi / M, A, Ap
    M1, M2 = M
    t = math.pi * np.arange(M1) / M1
    f = math.pi * np.arange(M2) / M2
    tt, ff = np.meshgrid(t, f, indexing="ij")  # direction index q + M2 p
    e = np.stack([np.sin(tt) * np.cos(ff), np.sin(tt) * np.sin(ff), np.cos(tt)], axis=-1).reshape(-1, 3)
    proj = e @ v.T
    A = 4.0 * Cphi * np.sin(tt).reshape(-1, 1) * phi3(R, proj)
    perp = np.sqrt(np.maximum(np.sum(v * v, axis=1)[None, :] - proj * proj, 0.0))
    Ap = psi3(R, perp)
    return math.pi ** 2 / (M1 * M2), A, Ap


def beta_separated(d: int, a, b, M, Cphi: float = 1.0, R: float = R_DEFAULT) -> np.ndarray:
    """beta_P(a_i, b_i) of eq. betadD for vector pairs (arrays of shape (n, d))."""
    a = np.asarray(a).reshape(-1, d)
    b = np.asarray(b).reshape(-1, d)
    C, A, _ = alphas(d, a, M, Cphi, R)
    _, _, Bp = alphas(d, b, M, Cphi, R)
    return C * np.sum(A * Bp, axis=0)


def beta_separated_table(d: int, N: int, M, Cphi: float = 1.0, R: float = R_DEFAULT) -> np.ndarray:
    """beta_P(a, b) for a, b in X = {-N..N-1}^d, in the [a][b] layout of the
    direct oracle's tables."""
    X = box(d, -N, N)
    C, A, Ap = alphas(d, X, M, Cphi, R)
    return C * (A.T @ Ap)


def t1_transform(d: int, N: int, Ghat: np.ndarray, M, Cphi: float = 1.0, R: float = R_DEFAULT) -> np.ndarray:
    """T1_n, n in I_N, by the appendix's route on the doubled grid (array
    indexed like Ghat, modes + N/2)."""
    Mg = 2 * N
    sh = (Mg,) * d
    axes = tuple(range(1, d + 1))
    # spectrum on the doubled grid (zero outside I_N), storage index k mod Mg
    Gpad = np.zeros(sh, dtype=np.complex128)
    k = modes(N) % Mg
    Gpad[np.ix_(*([k] * d))] = Ghat
    # physical values G_j = sum_k G_k e^{2 pi i k.j/Mg}
    Gphys = np.fft.ifftn(Gpad) * Mg ** d
    # alpha_p on one period of the doubled grid; a component -N never meets
    # a mode of I_N, so it is left out and the transforms below are real
    vec = box(d, -N, N)
    C, A, Ap = alphas(d, vec, M, Cphi, R)
    keep = np.all(vec > -N, axis=1)
    A[:, ~keep] = 0.0
    Ap[:, ~keep] = 0.0
    flat = np.ravel_multi_index(tuple((vec % Mg).T), sh)
    # shifts j and the output modes n
    J = box(d, 0, Mg)
    Xg = box(d, 0, Mg)
    shift = np.ravel_multi_index(tuple(((Xg[None, :, :] - J[:, None, :]) % Mg).transpose(2, 0, 1)), sh)
    nsel = np.ix_(*([k] * d))
    nvec = box(d, -(N // 2), N // 2)
    phase = np.exp(2j * math.pi * (J @ nvec.T) / Mg)  # e^{2 pi i n.j/Mg}, (|J|, N^d)
    T1 = np.zeros(N ** d, dtype=np.complex128)
    for p in range(A.shape[0]):
        ga = np.zeros(Mg ** d, dtype=np.complex128)
        gb = np.zeros(Mg ** d, dtype=np.complex128)
        ga[flat] = A[p]
        gb[flat] = Ap[p]
        # g_p(x) = sum_a alpha_p(a) e^{2 pi i a.x/Mg}
        ga = (np.fft.ifftn(ga.reshape(sh)) * Mg ** d).ravel()
        gb = (np.fft.ifftn(gb.reshape(sh)) * Mg ** d).ravel()
        # for every j: (g_pj * G)_n = Mg^-d sum_x g_p(x - j) G(x) e^{-2 pi i n.x/Mg}
        Ha = (ga[shift] * Gphys.ravel()[None, :]).reshape((-1,) + sh)
        Hb = (gb[shift] * Gphys.ravel()[None, :]).reshape((-1,) + sh)
        ca = (np.fft.fftn(Ha, axes=axes) / Mg ** d)[(slice(None),) + nsel].reshape(len(J), -1)
        cb = (np.fft.fftn(Hb, axes=axes) / Mg ** d)[(slice(None),) + nsel].reshape(len(J), -1)
        # the third factor: G_{a+b-n} = Mg^-d sum_j G(j) e^{-2 pi i (a+b-n).j/Mg}
        T1 += np.sum(Gphys.ravel()[:, None] * phase * ca * cb, axis=0)
    return (C / Mg ** d * T1).reshape(Ghat.shape)


def angles_2d(N: int, R: float = R_DEFAULT) -> int:
    """An angle count at which the 2-D rectangle rule reproduces the kernel
    modes of every pair a, b in X to rounding: the integrand's angular
    spectrum is that of e^{i x cos(.)} with x <= R (|a| + |b|) <= 2 sqrt(2) R N,
    negligible beyond order x + 10 x^(1/3) + 20, and the rule on the
    half-period integrates orders below 2M exactly."""
    x = 2.0 * math.sqrt(2.0) * R * N
    return int(math.ceil((x + 10.0 * x ** (1.0 / 3.0) + 20.0) / 2.0)) + 4
