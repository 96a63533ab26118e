"""Writes the oracle's Galerkin modes on dense data at full size, for the GPU
parity tests (tests/test_golden_dense_gpu.py).  Calls only oracle/ and the
seeded input recipes; the kernel modes come from the oracle's Funk-Hecke
series (pinned to its quadrature in tests/test_oracle.py).

  c2_3d32_sampled_modes.npz  the C2 datum (3-D fermions, N = 32, L = 8, three
      Gaussians, seed 0): Qc, the classical gain, T1 and X at 34 output modes:
      n = 0, six modes on the -N/2 faces (one, two and three components at
      -N/2) and 27 seeded modes;
  dense_3d16_all_modes.npz   the same recipe at N = 16: every output mode.

Run from the repository root:  python tests/golden/make_dense_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import bnq_inputs as inp  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
EPS, L, SEED = -1, 8.0, 0


def c2_modes(N=32, nrand=27, seed=32):
    h = N // 2
    fixed = [(0, 0, 0), (-h, 0, 0), (0, -h, 5), (3, 7, -h), (-h, -h, 2), (-h, 4, -h), (-h, -h, -h)]
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [tuple(int(v) for v in rng.integers(-h, h, 3)) for _ in range(nrand)]
    modes = fixed + [p for p in pts if p not in fixed]
    idx = np.array([((a + h) * N + (b + h)) * N + (c + h) for a, b, c in modes], dtype=np.int64)
    return np.array(modes, dtype=np.int64), idx


def write(name, N, select, modes):
    f = inp.fermion_mixture_3d(N=N, L=L, seed=SEED)
    t0 = time.time()
    s = oracle.series_modes(f, EPS, select)
    print(f"{name}: N={N}, {select.size} modes, {time.time() - t0:.1f} s", flush=True)
    flat = {k: s[k].reshape(-1)[select] for k in ("Qc", "gain", "T1", "Xq")}
    np.savez(os.path.join(HERE, name), N=N, L=L, seed=SEED, eps=EPS, modes=modes, index=select,
             f_checksum=np.array([f.sum(), (f * f).sum()]), **flat)


if __name__ == "__main__":
    which = sys.argv[1:] or ["16", "32"]
    if "16" in which:
        N = 16
        h = N // 2
        grid = np.stack(np.meshgrid(*([np.arange(-h, h)] * 3), indexing="ij"), axis=-1).reshape(-1, 3)
        write("dense_3d16_all_modes.npz", N, np.arange(N ** 3, dtype=np.int64), grid)
    if "32" in which:
        modes, idx = c2_modes()
        write("c2_3d32_sampled_modes.npz", 32, idx, modes)
