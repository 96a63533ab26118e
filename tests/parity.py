"""Parity criteria shared by the GPU tests (the HIP path against the oracle)."""
import numpy as np


def check(got, ref, gain=None, tol=1e-12, cancel=10.0):
    """Parity of `got` with the oracle's `ref` (both arrays over the same
    modes or nodes); `gain` is the oracle's classical gain term on the same
    modes or nodes (the scale of the cancellation near equilibrium).
      (i)   norm:         |got - ref|_2   <= tol max(|ref|_2, |gain|_2)
      (ii)  element-wise: max |got - ref| <= tol max(max |ref|, max |gain|)
      (iii) relative:     |got - ref|_2 / |ref|_2 <= tol, whenever the gain
            is at most `cancel` times the result (no strong cancellation)."""
    dlt = np.asarray(got) - np.asarray(ref)
    g = np.zeros(1) if gain is None else np.asarray(gain)
    nref, ngain = np.linalg.norm(ref), np.linalg.norm(g)
    err = np.linalg.norm(dlt) / max(nref, ngain, 1e-300)
    emax = np.max(np.abs(dlt)) / max(np.max(np.abs(ref)), np.max(np.abs(g)), 1e-300)
    rel = np.linalg.norm(dlt) / max(nref, 1e-300)
    print(f"parity: norm {err:.2e}, element-wise {emax:.2e}, relative {rel:.2e} (gain/result "
          f"{ngain / max(nref, 1e-300):.2e})")
    assert err <= tol, f"error {err:.3e} > {tol:.1e} (|ref| {nref:.3e}, |gain| {ngain:.3e})"
    assert emax <= tol, f"element-wise error {emax:.3e} > {tol:.1e}"
    if ngain <= cancel * nref:
        assert rel <= tol, f"relative error {rel:.3e} > {tol:.1e} (gain/result {ngain / nref:.2e})"
