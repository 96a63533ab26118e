"""Checkpoint and resume of a solve: the state f (FP64, the plan's layout),
the time t, the step count and the parameters of the plan, in one .npz file
of plain arrays (no pickled objects).  The kernels are deterministic under the
static schedule, so a solve resumed from a checkpoint continues bitwise as the
uninterrupted one."""
from __future__ import annotations

import os

import numpy as np

from . import Params

_FIELDS = ("d", "N", "eps", "precision", "terms", "correction", "schedule", "flags", "angles", "hbar", "L",
           "C_phi", "c")


def save(path: str, p: Params, f, t: float, step: int, **extra) -> None:
    """Write the checkpoint (atomically: a temporary file, then a rename).
    f: a device tensor or an ndarray; extra: further arrays to keep."""
    arr = f.detach().cpu().numpy() if hasattr(f, "detach") else np.asarray(f)
    if arr.dtype != np.float64:
        raise ValueError("the state must be FP64")
    fields = {k: np.asarray(getattr(p, k)) for k in _FIELDS if hasattr(p, k)}
    tmp = path + ".tmp.npz"
    np.savez(tmp, f=arr, t=np.float64(t), step=np.int64(step), format=np.array("bnq-checkpoint-1"),
             **{"p_" + k: v for k, v in fields.items()}, **{"x_" + k: np.asarray(v) for k, v in extra.items()})
    os.replace(tmp, path)


def load(path: str) -> dict:
    """Read a checkpoint: {'params': Params, 'f': ndarray, 't', 'step', 'extra': {...}}."""
    with np.load(path, allow_pickle=False) as z:
        if "format" not in z.files or str(z["format"]) != "bnq-checkpoint-1":
            raise ValueError(f"{path}: not a bnq checkpoint")
        kw = {}
        for k in _FIELDS:
            if "p_" + k in z.files:
                v = z["p_" + k]
                kw[k] = float(v) if v.dtype.kind == "f" else int(v)
        return {"params": Params(**kw), "f": np.array(z["f"]), "t": float(z["t"]), "step": int(z["step"]),
                "extra": {k[2:]: np.array(z[k]) for k in z.files if k.startswith("x_")}}
