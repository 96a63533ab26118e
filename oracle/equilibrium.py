"""Oracle for the limit states of the space-homogeneous equation.

TEST INFRASTRUCTURE ONLY (like the rest of this package): only tests/, the
smoke check and the CPU-baseline leg of the benchmark may import it.

Section 'Convergence towards a steady state', written out plainly:

* classical (alpha = 0): M_c = rho (2 pi T)^(-d/2) exp(-|v-u|^2 / 2T),
  T = 2e/d;
* quantum (alpha != 0): M_q = (1/|alpha|) / (z^-1 exp(|v-u|^2/2T) + sgn alpha)
  with, by eqs. mom0_qmaxwell and mom2_qmaxwell,
      rho = (2 pi T)^(d/2) K_{d/2}(z) / |alpha|,
      e   = (d T / 2) K_{d/2+1}(z) / K_{d/2}(z),
  K_nu the complete Fermi-Dirac (alpha > 0) or Bose-Einstein (alpha < 0)
  integral; eliminating T gives eq. eq_fugacity,
      |alpha| rho (nu / (2 pi e))^nu = K_nu(z)^(nu+1) / K_(nu+1)(z)^nu,
  nu = d/2, solvable iff the left side lies in I_eq (eq. def_Ieq);
* outside I_eq: the 3-D Bose-Einstein condensate (z = 1, m0 from eq.
  m0critical_bosons_3d; T such that the z = 1 part carries the internal
  energy rho e: eq. Tcritical_bosons_3d as printed conserves it only at the
  critical ratio, so it is read this way), the saturated Fermi-Dirac
  state chi (eq. def_chi) when the equality critical_FD holds, and no
  identified state otherwise.

Here K_nu comes from adaptive quadrature (scipy.integrate.quad) of its
definition and the fugacity from scipy.optimize.brentq: library primitives,
independent of the library's own quadrature and root finder.  Pinned in
tests/test_equilibrium_oracle.py against closed forms (K_1, K_2 by
logarithms and dilogarithms, K_nu(1) = zeta(nu) for Bose-Einstein, the
Sommerfeld expansion of degenerate Fermi-Dirac, the classical limit) and
against states built from a chosen (z, T).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

MAXWELL, QUANTUM, CONDENSATE, SATURATED, UNKNOWN = 0, 1, 2, 3, 4


def K(nu: float, fermi: bool, z: float | None = None, log_z: float | None = None) -> float:
    """Complete Fermi-Dirac / Bose-Einstein integral
    K_nu(z) = Gamma(nu)^-1 int_0^inf x^(nu-1) / (z^-1 e^x + sgn) dx
    (sgn = +1 Fermi-Dirac, -1 Bose-Einstein, which needs z <= 1)."""
    lz = math.log(z) if log_z is None else log_z
    opts = dict(epsabs=0.0, epsrel=5e-14, limit=500)
    if fermi:
        top = max(lz, 0.0) + 60.0
        pts = [lz] if 0.0 < lz < top else None
        val, _ = integrate.quad(lambda x: x ** (nu - 1.0) / (math.exp(x - lz) + 1.0), 0.0, top, points=pts, **opts)
    elif nu > 1.0:
        # x^(nu-1) / (e^(x - ln z) - 1) = x^(nu-2) * [x / expm1(x - ln z)], the
        # algebraic factor taken by the quadrature's own weight
        val, _ = integrate.quad(lambda x: x / math.expm1(x - lz) if x > 0 else (1.0 if lz == 0 else 0.0),
                                0.0, 60.0, weight="alg", wvar=(nu - 2.0, 0.0), **opts)
    else:  # nu = 1 needs z < 1
        val, _ = integrate.quad(lambda x: 1.0 / math.expm1(x - lz), 0.0, 60.0, **opts)
    return val / math.gamma(nu)


def ieq_upper(d: int, fermi: bool) -> float:
    """Upper end of I_eq (eq. def_Ieq)."""
    nu = d / 2.0
    if fermi:
        return (nu + 1.0) ** nu / math.gamma(nu + 1.0)
    if d == 2:
        return math.inf
    return K(1.5, False, 1.0) ** 2.5 / K(2.5, False, 1.0) ** 1.5


def solve(d: int, eps: int, hbar: float, rho: float, u, e: float) -> dict:
    """Limit state for (rho, u, e), following the paper's classification."""
    alpha = -eps * hbar ** d
    nu = d / 2.0
    out = {"kind": None, "alpha": alpha, "rho": rho, "u": list(u)[:d], "e": e,
           "z": 0.0, "log_z": 0.0, "T": 0.0, "m0": 0.0, "A": 0.0, "ratio": 0.0}
    if alpha == 0:
        out.update(kind=MAXWELL, T=2.0 * e / d)
        return out
    fermi = alpha > 0
    ratio = abs(alpha) * rho * (d / (4.0 * math.pi * e)) ** nu
    out["ratio"] = ratio
    up = ieq_upper(d, fermi)
    if fermi:
        out["A"] = math.sqrt(2.0 * e * (d + 2.0) / d)
        if abs(ratio / up - 1.0) <= 1e-9:
            out["kind"] = SATURATED
            return out
        if ratio > up:
            out["kind"] = UNKNOWN
            return out

        def g(mu):
            return (nu + 1) * math.log(K(nu, True, log_z=mu)) - nu * math.log(K(nu + 1, True, log_z=mu)) \
                - math.log(ratio)
        lo, hi = math.log(ratio) - 5.0, 5.0
        while g(hi) < 0:
            hi *= 2.0
        while g(lo) > 0:
            lo -= 5.0
        mu = optimize.brentq(g, lo, hi, xtol=1e-14, rtol=1e-15, maxiter=500)
        T = e * K(nu, True, log_z=mu) / (nu * K(nu + 1, True, log_z=mu))
        out.update(kind=QUANTUM, log_z=mu, z=math.exp(mu) if mu < 700 else math.inf, T=T)
        return out
    if ratio >= up:
        # reading: the z = 1 part carries the whole internal energy rho e,
        #   rho e = (2 pi T)^(3/2) (3/2) T zeta(5/2) / |alpha|;
        # eq. Tcritical_bosons_3d gives the same T only at the critical ratio
        z32, z52 = K(1.5, False, 1.0), K(2.5, False, 1.0)
        T = (abs(alpha) * rho * e / ((2.0 * math.pi) ** 1.5 * 1.5 * z52)) ** 0.4
        out.update(kind=CONDENSATE, z=1.0, log_z=0.0, T=T,
                   m0=rho - (2.0 * math.pi * T) ** 1.5 * z32 / abs(alpha))
        return out

    def gb(w):  # w = ln(-ln z)
        lz = -math.exp(w)
        return (nu + 1) * math.log(K(nu, False, log_z=lz)) - nu * math.log(K(nu + 1, False, log_z=lz)) \
            - math.log(ratio)
    lo, hi = -3.0, math.log(max(-math.log(ratio), 0.0) + 8.0)
    while gb(lo) < 0:
        lo -= 4.0
    while gb(hi) > 0:
        hi += 1.0
    w = optimize.brentq(gb, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    lz = -math.exp(w)
    T = e * K(nu, False, log_z=lz) / (nu * K(nu + 1, False, log_z=lz))
    out.update(kind=QUANTUM, log_z=lz, z=math.exp(lz), T=T)
    return out


def on_grid(d: int, N: int, L: float, st: dict):
    """The state at the nodes v_j = 2 L j / N (j in I_N, axis order of the
    grid arrays) and a mask of the nodes where it is not a finite function: for
    a condensate the node of the grid cell holding u (|v - u|_inf < L / N),
    where its mass m0 sits."""
    ax = 2.0 * L * (np.arange(N) - N // 2) / N
    v = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1)
    w = v - np.asarray(st["u"], dtype=np.float64)
    r2 = np.sum(w ** 2, axis=-1)
    k = st["kind"]
    # a condensate's mass sits at v = u: the node of the grid cell holding u
    excl = (np.max(np.abs(w), axis=-1) < L / N) if k == CONDENSATE else np.zeros(r2.shape, dtype=bool)
    if k == MAXWELL:
        M = st["rho"] * (2 * math.pi * st["T"]) ** (-d / 2.0) * np.exp(-r2 / (2 * st["T"]))
    elif k == SATURATED:
        vol = math.pi ** (d / 2.0) * st["A"] ** d / math.gamma(d / 2.0 + 1.0)
        M = np.where(r2 <= st["A"] ** 2, st["rho"] / vol, 0.0)
    elif k in (QUANTUM, CONDENSATE):
        a = r2 / (2 * st["T"]) - (0.0 if k == CONDENSATE else st["log_z"])
        if st["alpha"] > 0:
            den = np.exp(a) + 1.0
        else:
            den = np.expm1(a)
            excl = excl | ~(den > 0)
        with np.errstate(divide="ignore"):
            M = np.where(excl, 0.0, 1.0 / abs(st["alpha"]) / np.where(excl, 1.0, den))
    else:
        raise ValueError("no limit state identified")
    return M, excl


def distance(f: np.ndarray, L: float, st: dict) -> dict:
    """Delta v sum |f - M| and max |f - M| over the nodes where M is finite,
    the mass of M there, and the count and mass of f at the other nodes."""
    d, N = f.ndim, f.shape[0]
    dv = (2.0 * L / N) ** d
    M, excl = on_grid(d, N, L, st)
    diff = np.abs(f - M)[~excl]
    return {"l1": dv * diff.sum(), "max_abs": float(diff.max()) if diff.size else 0.0,
            "mass_of_state": dv * M[~excl].sum(), "n_excluded": int(excl.sum()),
            "mass_excluded": dv * f[excl].sum()}
