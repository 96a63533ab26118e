"""Relaxation towards equilibrium (section 'Relaxation towards equilibrium':
2-D and 3-D Fermi-Dirac, 3-D Bose-Einstein) with hbar = r hbar*.

For an initial datum f0 the threshold hbar* follows from its discrete mass
rho and internal energy e (half the second moment per particle):
  - Fermi-Dirac: the hbar at which the limit state is the saturated ball,
    hbar*^d = K_d (4 pi e / d)^(d/2) / rho with K_2 = 2, K_3 = (5/3) sqrt(10/pi)
    (the criterion m_0 = 0 of the section's Fermi-Dirac case; the printed
    thresholds 3.5449 and 3.60452 of the Maxwellian data are this value);
  - Bose-Einstein (3-D): the critical hbar of condensation,
    hbar* = rho^(-1/3) (4 pi e / 3)^(1/2) zeta(3/2)^(5/6) / zeta(5/2)^(1/2).
Below the threshold the solution relaxes to the quantum Maxwellian of the
same moments; at and above it to the saturated or condensed limit, which the
grid cannot hold (the paper's runs blow up there).

run() advances f0 with SSP-RK2 (the paper's integrator) at hbar = r hbar*
and records, every `every` steps, the entropy H, max f, and the l1 and
pointwise distances to the limit state solved by the library; it stops at
the first step whose health flags report a non-finite state or a
Fermi-Dirac value at or above 1/hbar^d.  All arithmetic is libbnq's.

Usage: python -m paper_2110_13735_amd.relaxation --case fd2-ball --r 0.5 0.9 0.99 1.01 --N 64 --out file.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

K_FD = {2: 2.0, 3: (5.0 / 3.0) * math.sqrt(10.0 / math.pi)}
ZETA_32 = 2.612375348685488343348567567924071
ZETA_52 = 1.341487257250917179756769702826091

# the section's cases: (d, eps, datum, L, dt, t_end)
CASES = {
    "fd2-ball": (2, -1, "ball", 8.0, 0.025, 30.0),
    "fd2-maxwellian": (2, -1, "maxwellian", 8.0, 0.025, 30.0),
    "fd3-ball": (3, -1, "ball", 6.0, 0.025, 10.0),
    "fd3-maxwellian": (3, -1, "maxwellian", 6.0, 0.025, 10.0),
    "be3-ball": (3, 1, "ball", 6.0, 0.025, 10.0),
    "be3-maxwellian": (3, 1, "maxwellian", 6.0, 0.025, 10.0),
}


def hbar_star(d: int, eps: int, rho: float, e: float) -> float:
    """The threshold hbar* for mass rho and internal energy e (module docstring)."""
    if eps == -1:
        return (K_FD[d] * (4.0 * math.pi * e / d) ** (d / 2.0) / rho) ** (1.0 / d)
    if eps == 1 and d == 3:
        return rho ** (-1.0 / 3.0) * math.sqrt(4.0 * math.pi * e / 3.0) * ZETA_32 ** (5.0 / 6.0) / math.sqrt(ZETA_52)
    raise ValueError("hbar* is defined for Fermi-Dirac data (2-D, 3-D) and 3-D Bose-Einstein data")


def discrete_moments(f, d: int, N: int, L: float) -> dict:
    """rho, u and e of grid data (host arithmetic on the datum, for hbar*)."""
    import numpy as np
    from bnq_inputs import cell_volume, velocity_grid

    v = velocity_grid(d, N, L)
    w = cell_volume(d, N, L)
    rho = w * float(f.sum())
    u = [w * float((f * v[..., i]).sum()) / rho for i in range(d)]
    c = v - np.asarray(u)
    e = 0.5 * w * float((f * np.sum(c * c, axis=-1)).sum()) / rho
    return {"rho": rho, "u": u, "e": e}


def run(case: str, r: float, N: int, steps: int | None = None, every: int = 20, precision: int = 0,
        dt: float | None = None, fermi_bound: bool = True, log=None) -> dict:
    """One run at hbar = r hbar*; fermi_bound=False lets Fermi-Dirac values at
    or above 1/hbar^d pass the step health flags (BNQ_FLAG_NO_FERMI_BOUND), as
    the section's runs with data above that bound require; max f is recorded."""
    import numpy as np
    import torch

    import bnq_inputs as inp

    from . import (BNQ_EBOUND, BNQ_ENONFINITE, EQ_UNKNOWN, FLAG_NO_FERMI_BOUND, HEALTH_NONFINITE, SSPRK2, BnqError,
                   Params, Plan, equilibrium)

    d, eps, kind, L, dt0, t_end = CASES[case]
    dt = dt0 if dt is None else dt
    nsteps = int(round(t_end / dt)) if steps is None else steps
    f0 = inp.relaxation_datum(kind, d, N, L)
    m0 = discrete_moments(f0, d, N, L)
    hs = hbar_star(d, eps, m0["rho"], m0["e"])
    hbar = r * hs
    p = Params(d=d, N=N, eps=eps, L=L, hbar=hbar, precision=precision,
               flags=0 if fermi_bound else FLAG_NO_FERMI_BOUND)
    out = {"case": case, "d": d, "eps": eps, "datum": kind, "N": N, "L": L, "dt": dt, "r": r, "fermi_bound": fermi_bound,
           "hbar_star": hs, "hbar": hbar, "f0_max": float(f0.max()), "bound": 1.0 / hbar ** d if eps == -1 else None,
           "moments0": m0, "track": [], "status": "running"}
    with Plan(p) as plan:
        try:
            lim = equilibrium(d, eps, hbar, m0["rho"], m0["u"], m0["e"])
            out["limit_state"] = lim.as_dict()
            if lim.kind == EQ_UNKNOWN:  # past the saturated Fermi-Dirac state no limit exists
                lim = None
        except BnqError as err:
            lim = None
            out["limit_state"] = {"error": str(err)}
        f = torch.tensor(f0, device="cuda:0")

        def record(k):
            mk = plan.moments(f, check=False)
            dk = plan.equilibrium_distance(f, lim) if lim is not None else {"l1": float("nan"), "max_abs": float("nan")}
            rec = {"step": k, "t": k * dt, "H": mk["H"], "fmax": mk["fmax"], "rho": mk["rho"], "e": mk["e"],
                   "l1": dk["l1"], "max_abs": dk["max_abs"]}
            out["track"].append(rec)
            if log is not None:
                print(f"[relax {case} r={r}] step {k} t={k * dt:.3f} H={mk['H']:.6f} l1={dk['l1']:.3e} "
                      f"fmax={mk['fmax']:.4f}", file=log, flush=True)

        record(0)
        t0 = time.perf_counter()

        def stop(k, fl):
            out["status"] = "stopped"
            out["stop_step"] = k
            out["stop_reason"] = "non-finite state" if fl & HEALTH_NONFINITE else "Fermi-Dirac bound reached"

        for k in range(1, nsteps + 1):
            try:
                plan.step(f, dt, SSPRK2)
            except BnqError as err:  # a completed step's flags refuse the next one
                if err.status not in (BNQ_ENONFINITE, BNQ_EBOUND):
                    raise
                stop(k - 1, plan.health(wait=True))
                break
            if k % every == 0 or k == nsteps:
                fl = plan.health(wait=True)
                if fl:
                    stop(k, fl)
                    break
                record(k)
        torch.cuda.synchronize()
        out["elapsed_s"] = time.perf_counter() - t0
        if out["status"] == "running":
            out["status"] = "completed"
        H = [x["H"] for x in out["track"] if math.isfinite(x["H"])]
        out["H_nonincreasing"] = bool(all(b <= a + 1e-12 * max(1.0, abs(a)) for a, b in zip(H, H[1:])))
        out["final"] = out["track"][-1]
        # the v_y = 0 (2-D) or (., 0, 0) (3-D) profile of the last recorded state
        fh = f.cpu().numpy()
        h = N // 2
        out["profile"] = (fh[:, h] if d == 2 else fh[:, h, h]).tolist()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--case", choices=sorted(CASES), required=True)
    ap.add_argument("--r", type=float, nargs="+", required=True)
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--steps", type=int, default=None, help="default: the case's t_end / dt")
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--dt", type=float, default=None)
    ap.add_argument("--fp32c", action="store_true")
    ap.add_argument("--no-bound-check", action="store_true",
                    help="let Fermi-Dirac values at or above 1/hbar^d pass the step health flags")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    N = a.N or (64 if CASES[a.case][0] == 2 else 32)
    res = [run(a.case, r, N, a.steps, a.every, 1 if a.fp32c else 0, a.dt, not a.no_bound_check, log=sys.stderr)
           for r in a.r]
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    else:
        print(text)


if __name__ == "__main__":
    main()
