"""Spectral-accuracy experiment of section 'Validation of spectral accuracy'.

For the quantum Maxwellian f0 (hbar = 3, rho = 1, temperature sigma, mean
velocity u0 in {0, u_b}, u_b = 8 / (3 sqrt 2 + 2) (1, ..., 1)):

  1. f0 on the grid, its discrete moments rho_h, u_h, e_h;
  2. the limit state with rho = rho_h, u = u0 and the temperature and
     fugacity solved from (rho_h, e_h) (bnq_equilibrium_solve);
  3. that state on the grid, and the residual max_j |Q(f_h^inf)_j|, the
     operator's value (c (L/pi)^(d+gamma) times the Galerkin sums) in f's
     units.

'without rescaling': the fixed box [-L, L)^d.  'with rescaling': the box of
the rescaled scheme, u0 + [-L/omega, L/omega)^d with omega = sqrt(T) of the
discrete limit state (the moments of step 1 taken on the box of omega =
sqrt(sigma)); the operator is translation invariant, so the box is centred
on 0 and the state on 0 as well.

Usage: python -m paper_2110_13735_amd.spectral_accuracy [--dims 2 3] [--out file.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

HBAR = 3.0
U_B = 8.0 / (3.0 * math.sqrt(2.0) + 2.0)


def fugacity(d: int, eps: int, rho: float, T: float) -> float:
    """ln z with rho = (2 pi T)^(d/2) K_{d/2}(z) / |alpha| (eq. mom0_qmaxwell),
    by bisection on the library's ln K."""
    from . import fd_be_log

    alpha = HBAR ** d
    target = math.log(alpha * rho) - 0.5 * d * math.log(2 * math.pi * T)
    nu = 0.5 * d
    if eps == -1:  # Fermi-Dirac: ln K increases with mu = ln z
        lo, hi = -50.0, 50.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if fd_be_log(nu, True, mid) < target else (lo, mid)
        return 0.5 * (lo + hi)
    lo, hi = 1e-300, 50.0  # Bose-Einstein: ln K decreases with delta = -ln z
    for _ in range(400):
        mid = math.sqrt(lo * hi) if hi / lo > 4 else 0.5 * (lo + hi)
        lo, hi = (lo, mid) if fd_be_log(nu, False, mid) < target else (mid, hi)
    return -0.5 * (lo + hi)


def residual(d: int, N: int, L: float, eps: int, sigma: float, ub: bool, rescaled: bool) -> dict:
    import torch

    from . import EQ_QUANTUM, Params, Plan, equilibrium

    dev = torch.device("cuda:0")
    u0 = np.full(d, U_B if ub else 0.0)
    lz0 = fugacity(d, eps, 1.0, sigma)
    # step 1: f0 on the box (centred on u0 when rescaled), discrete moments
    half = L / math.sqrt(sigma) if rescaled else L
    ax = 2.0 * half * (np.arange(N) - N // 2) / N
    v = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1) + (u0 if rescaled else 0.0)
    r2 = np.sum((v - u0) ** 2, axis=-1)
    sgn = 1.0 if eps == -1 else -1.0
    f0 = (1.0 / HBAR ** d) / (np.exp(r2 / (2 * sigma) - lz0) + sgn)
    p = Params(d=d, N=N, eps=eps, L=half, hbar=HBAR)
    with Plan(p) as plan:
        m = plan.moments(torch.tensor(f0, device=dev))
    us = [m["u0"], m["u1"], m["u2"]][:d]
    # step 2: the limit state (u = u0; T, z from rho_h, e_h)
    st = equilibrium(d, eps, HBAR, m["rho"], us, m["e"])
    if st.kind != EQ_QUANTUM:
        return {"residual": None, "kind": st.kind}
    half_inf = L / math.sqrt(st.T) if rescaled else L
    # step 3: the state on the grid (centred on u0 in the fixed box)
    ax = 2.0 * half_inf * (np.arange(N) - N // 2) / N
    v = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1)
    w = v if rescaled else v - u0
    finf = (1.0 / HBAR ** d) / (np.exp(np.sum(w * w, axis=-1) / (2 * st.T) - st.log_z) + sgn)
    p = Params(d=d, N=N, eps=eps, L=half_inf, hbar=HBAR)
    with Plan(p) as plan:
        ft = torch.tensor(finf, device=dev)
        Q = torch.empty_like(ft)
        plan.collide(ft, Q)
        torch.cuda.synchronize()
        res = float(Q.abs().max())
    return {"residual": res, "z0": math.exp(lz0), "T_h": st.T, "z_h": math.exp(st.log_z)}


CASES = {
    2: {"species": (-1, 1), "sigma": (0.5, 1.0), "L": (4.0, 6.0, 8.0, 10.0), "N": (16, 32, 64)},
    3: {"species": (-1,), "sigma": (0.5, 1.0), "L": (4.0, 6.0, 8.0, 10.0), "N": (16, 32)},
}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs="+", default=[2, 3])
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch

    from . import Params, Plan

    torch.cuda.set_device(0)  # the plans use torch's device and streams

    rows = []
    anchors = []  # one live plan per (d, N) keeps its tables resident across the cases
    for d in args.dims:
        c = CASES[d]
        for eps in c["species"]:
            for sigma in c["sigma"]:
                for L in c["L"]:
                    for N in c["N"]:
                        if (d, N) not in [a[0] for a in anchors]:
                            anchors.append(((d, N), Plan(Params(d=d, N=N, eps=eps, L=L, hbar=HBAR))))
                        row = {"d": d, "statistics": "FD" if eps == -1 else "BE", "sigma": sigma, "L": L, "N": N}
                        for ub in (False, True):
                            for resc in (True, False):
                                r = residual(d, N, L, eps, sigma, ub, resc)
                                key = ("ub" if ub else "u0") + ("_with" if resc else "_without")
                                row[key] = r["residual"]
                                row["z0"] = r.get("z0")
                        rows.append(row)
                        print(json.dumps(row), file=sys.stderr, flush=True)
    for _, pl in anchors:
        pl.close()
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rows, fh, indent=1)
    return rows


if __name__ == "__main__":
    main()
