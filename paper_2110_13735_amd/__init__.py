"""Python binding of libbnq (include/bnq.h): argument marshalling only.

Every computation runs in the HIP kernels of libbnq.so, which must have been
built in-tree (paper_2110_13735_amd/build_lib.py); importing this package
without the library raises, there is no fallback.  Device arrays are passed as
torch tensors (their data_ptr) or raw integer addresses; streams default to
torch's current HIP stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbnq.so")
# Trilinear work distributions measured by bnq_plan_autotune on an MI355X for
# the batch cells (d in {2, 3}, N in {16, 24, 32}, FP64 and FP32c); not loaded
# by default (a tuned choice may change the last bits of a result): pass it to
# load_tuning.
TUNING_MI355X = os.path.join(HERE, "tuning_mi355x.json")

BNQ_OK, BNQ_EINVAL, BNQ_ENOMEM, BNQ_EHIP, BNQ_ENOTSUP, BNQ_ENONFINITE, BNQ_EBOUND = 0, -1, -2, -3, -4, -5, -6
T_CLASSICAL, T_QMULT, T_QTRI, T_ALL = 1, 2, 4, 7
FP64, FP32C = 0, 1
FLAG_WEIGHTS_OTF = 1
FLAG_T1_SEPARATED = 2
FLAG_NO_FERMI_BOUND = 4
SCHED_STATIC, SCHED_DYNAMIC = 0, 1
CORR_NONE, CORR_MASS, CORR_MOMENTS = 0, 1, 2
RK4, EULER, SSPRK2 = 0, 1, 2
MOMENTS_LEN = 10
HEALTH_NONFINITE, HEALTH_BOUND = 1, 2
NKERNELS = 8
KERNEL_FAMILIES = ("dft", "pairs", "outer", "trilinear", "reduce", "combine", "step", "moments")
MOMENT_NAMES = ("rho", "u0", "u1", "u2", "Ec", "e", "H", "fmax", "fmin", "n_excluded")


class BnqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bnq status {status}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int32), ("eps", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("terms", ctypes.c_int32), ("correction", ctypes.c_int32),
                ("hbar", ctypes.c_double), ("C_phi", ctypes.c_double), ("c", ctypes.c_double),
                ("L", ctypes.c_double), ("schedule", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("angles", ctypes.c_int32)]


@dataclass
class Params:
    d: int = 3
    N: int = 16
    eps: int = 0
    L: float = 8.0
    hbar: float = 1.0
    C_phi: float = 1.0
    c: float = 1.0
    terms: int = T_ALL
    correction: int = CORR_NONE
    precision: int = FP64
    schedule: int = 0  # SCHED_STATIC
    flags: int = 0  # FLAG_*
    angles: int = 0  # FLAG_T1_SEPARATED: 2-D angle count P (0 = enough for FP64); 3-D polar count M1 (required)

    def _c(self) -> _Params:
        return _Params(self.d, self.N, self.eps, self.precision, self.terms, self.correction,
                       self.hbar, self.C_phi, self.c, self.L, self.schedule, self.flags, self.angles)


EQ_MAXWELL, EQ_QUANTUM, EQ_CONDENSATE, EQ_SATURATED, EQ_UNKNOWN = 0, 1, 2, 3, 4
EQDIST_NAMES = ("l1", "max_abs", "mass_of_state", "n_excluded", "mass_excluded")


class Equilibrium(ctypes.Structure):
    """bnq_equilibrium: a limit state (kind EQ_*) and its parameters."""
    _fields_ = [("kind", ctypes.c_int32), ("d", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("rho", ctypes.c_double), ("u", ctypes.c_double * 3), ("e", ctypes.c_double),
                ("z", ctypes.c_double), ("log_z", ctypes.c_double), ("T", ctypes.c_double),
                ("m0", ctypes.c_double), ("A", ctypes.c_double), ("ratio", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: (list(getattr(self, k)) if k == "u" else getattr(self, k)) for k, _ in self._fields_}


class RescaledState(ctypes.Structure):
    """bnq_rescaled_state: moments and velocity scale of the rescaled scheme."""
    _fields_ = [("rho", ctypes.c_double), ("u", ctypes.c_double * 3), ("e", ctypes.c_double),
                ("omega", ctypes.c_double), ("T", ctypes.c_double), ("log_z", ctypes.c_double),
                ("kind", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: (list(getattr(self, k)) if k == "u" else getattr(self, k)) for k, _ in self._fields_}


def equilibrium(d: int, eps: int, hbar: float, rho: float, u, e: float) -> Equilibrium:
    """Limit state for mass rho, mean velocity u (d components) and internal
    energy e (bnq_equilibrium_solve)."""
    uu = np.zeros(3)
    uv = np.asarray(u, dtype=np.float64).ravel()[:3]
    uu[:uv.size] = uv
    out = Equilibrium()
    _check(lib().bnq_equilibrium_solve(int(d), int(eps), float(hbar), float(rho), uu.ctypes.data, float(e),
                                       ctypes.byref(out)))
    return out


def fd_be_log(nu: float, fermi: bool, p: float) -> float:
    """ln of the complete Fermi-Dirac (p = ln z) or Bose-Einstein (p = -ln z)
    integral K_nu (bnq_fd_be_log)."""
    out = ctypes.c_double()
    _check(lib().bnq_fd_be_log(float(nu), 1 if fermi else 0, float(p), ctypes.byref(out)))
    return out.value


_lib = None


def lib():
    """Load libbnq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with paper_2110_13735_amd/build_lib.py")
        L = ctypes.CDLL(LIBPATH)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER(_Params)
        L.bnq_params_default.argtypes = [P]
        L.bnq_params_default.restype = None
        L.bnq_plan.argtypes = [P, vp, ctypes.POINTER(vp)]
        L.bnq_plan_destroy.argtypes = [vp]
        L.bnq_plan_footprint.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.bnq_collide.argtypes = [vp, vp, vp, vp, vp]
        L.bnq_step.argtypes = [vp, vp, f64, i32, vp]
        L.bnq_moments.argtypes = [vp, vp, vp, vp]
        L.bnq_health.argtypes = [vp, i32, i32, vp, vp]
        L.bnq_moments_noalloc.argtypes = [P, vp, vp, vp]
        L.bnq_table_lookup.argtypes = [vp, i32, i64, vp, vp, vp]
        L.bnq_plan_counts.argtypes = [vp, vp]
        L.bnq_plan_set_timing.argtypes = [vp, i32]
        L.bnq_plan_timing.argtypes = [vp, vp, vp]
        L.bnq_plan_autotune.argtypes = [vp, vp, i32, vp, vp, vp]
        L.bnq_tune_get.argtypes = [i32, i32, i32, ctypes.POINTER(i32)]
        L.bnq_tune_set.argtypes = [i32, i32, i32, i32]
        L.bnq_plan_autotune_pairs.argtypes = [vp, vp, i32, vp, vp, vp]
        L.bnq_tune_pairs_get.argtypes = [i32, i32, i32, i32, ctypes.POINTER(i32)]
        L.bnq_tune_pairs_set.argtypes = [i32, i32, i32, i32, i32]
        L.bnq_batch_create.argtypes = [i32, vp, vp, ctypes.POINTER(vp)]
        L.bnq_batch_destroy.argtypes = [vp]
        L.bnq_batch_layout.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.bnq_batch_collide.argtypes = [vp, vp, vp, vp]
        L.bnq_batch_step.argtypes = [vp, vp, i32, i32, vp]
        EQ = ctypes.POINTER(Equilibrium)
        L.bnq_equilibrium_solve.argtypes = [i32, i32, f64, f64, vp, f64, EQ]
        L.bnq_fd_be_log.argtypes = [f64, i32, f64, ctypes.POINTER(f64)]
        L.bnq_equilibrium_fill.argtypes = [vp, EQ, vp, vp]
        L.bnq_equilibrium_distance.argtypes = [vp, vp, EQ, vp, vp]
        RS = ctypes.POINTER(RescaledState)
        L.bnq_rescaled_init.argtypes = [vp, vp, f64, vp, RS, vp]
        L.bnq_step_rescaled.argtypes = [vp, vp, RS, f64, vp]
        for fn in ("bnq_plan", "bnq_plan_destroy", "bnq_plan_footprint", "bnq_collide", "bnq_step",
                   "bnq_moments", "bnq_health", "bnq_moments_noalloc", "bnq_table_lookup", "bnq_plan_counts", "bnq_plan_set_timing",
                   "bnq_plan_timing", "bnq_plan_autotune", "bnq_tune_get", "bnq_tune_set", "bnq_plan_autotune_pairs",
                   "bnq_tune_pairs_get", "bnq_tune_pairs_set", "bnq_batch_create", "bnq_batch_destroy", "bnq_batch_layout", "bnq_batch_collide",
                   "bnq_batch_step", "bnq_equilibrium_solve", "bnq_fd_be_log", "bnq_equilibrium_fill",
                   "bnq_equilibrium_distance", "bnq_rescaled_init", "bnq_step_rescaled"):
            getattr(L, fn).restype = ctypes.c_int
        L.bnq_status_string.argtypes = [ctypes.c_int]
        L.bnq_status_string.restype = ctypes.c_char_p
        L.bnq_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st: int, allow=()):
    if st != BNQ_OK and st not in allow:
        raise BnqError(st, lib().bnq_last_error().decode(errors="replace"))
    return st


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def footprint(p: Params):
    """(plan workspace bytes, shared table bytes still to allocate)."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    cp = p._c()
    _check(lib().bnq_plan_footprint(ctypes.byref(cp), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class Plan:
    """A libbnq plan (bnq_plan / bnq_plan_destroy)."""

    def __init__(self, p: Params, stream=None):
        self.params = p
        self._h = ctypes.c_void_p()
        cp = p._c()
        _check(lib().bnq_plan(ctypes.byref(cp), _stream(stream), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(lib().bnq_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def collide(self, f, Q, Qhat=None, stream=None):
        _check(lib().bnq_collide(self._h, _ptr(f), _ptr(Q), _ptr(Qhat), _stream(stream)))

    def step(self, f, dt: float, scheme: int = RK4, stream=None):
        _check(lib().bnq_step(self._h, _ptr(f), float(dt), int(scheme), _stream(stream)))

    def moments(self, f, stream=None, check: bool = True) -> dict:
        out = np.zeros(MOMENTS_LEN)
        st = lib().bnq_moments(self._h, _ptr(f), out.ctypes.data, _stream(stream))
        if check:
            _check(st)
        res = dict(zip(MOMENT_NAMES, out.tolist()))
        res["status"] = st
        return res

    def health(self, wait: bool = True, clear: bool = False, stream=None) -> int:
        """BNQ_HEALTH_* bits recorded by completed steps (bnq_health); never
        raises for set flags."""
        fl = ctypes.c_int32(0)
        _check(lib().bnq_health(self._h, 1 if wait else 0, 1 if clear else 0, ctypes.byref(fl), _stream(stream)),
               allow=(BNQ_ENONFINITE, BNQ_EBOUND))
        return fl.value

    def equilibrium_fill(self, eq: Equilibrium, out, stream=None):
        _check(lib().bnq_equilibrium_fill(self._h, ctypes.byref(eq), _ptr(out), _stream(stream)))

    def equilibrium_distance(self, f, eq: Equilibrium, stream=None) -> dict:
        out = np.zeros(len(EQDIST_NAMES))
        _check(lib().bnq_equilibrium_distance(self._h, _ptr(f), ctypes.byref(eq), out.ctypes.data,
                                              _stream(stream)))
        return dict(zip(EQDIST_NAMES, out.tolist()))

    def rescaled_init(self, G, omega: float, u_ref, stream=None) -> RescaledState:
        uu = np.zeros(3)
        uv = np.asarray(u_ref, dtype=np.float64).ravel()[:3]
        uu[:uv.size] = uv
        st = RescaledState()
        _check(lib().bnq_rescaled_init(self._h, _ptr(G), float(omega), uu.ctypes.data, ctypes.byref(st),
                                       _stream(stream)))
        return st

    def step_rescaled(self, G, st: RescaledState, dt: float, stream=None) -> RescaledState:
        _check(lib().bnq_step_rescaled(self._h, _ptr(G), ctypes.byref(st), float(dt), _stream(stream)))
        return st

    def lookup(self, table: int, a, b) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.int32).reshape(-1, 3)
        b = np.ascontiguousarray(b, dtype=np.int32).reshape(-1, 3)
        out = np.zeros(a.shape[0])
        _check(lib().bnq_table_lookup(self._h, int(table), a.shape[0], a.ctypes.data, b.ctypes.data,
                                      out.ctypes.data))
        return out

    def counts(self) -> dict:
        c = np.zeros(4)
        _check(lib().bnq_plan_counts(self._h, c.ctypes.data))
        return {"classical": c[0], "w_pairs": c[1], "outer": c[2], "trilinear": c[3]}

    def autotune(self, f, reps: int = 2, stream=None):
        """Pick the fastest trilinear work distribution on input f; returns
        (chosen index, mean ms per evaluation of each candidate)."""
        ms = np.zeros(4)
        ch = ctypes.c_int32(-1)
        _check(lib().bnq_plan_autotune(self._h, _ptr(f), int(reps), ms.ctypes.data, ctypes.byref(ch),
                                       _stream(stream)))
        return ch.value, ms

    def autotune_pairs(self, f, reps: int = 3, stream=None):
        """Pick the fastest l-chunking of the pair sums (8, 16 or 32 slices) on
        input f; returns (slices kept, mean ms of each candidate, 0 = not run)."""
        ms = np.zeros(3)
        sp = ctypes.c_int32(0)
        _check(lib().bnq_plan_autotune_pairs(self._h, _ptr(f), int(reps), ms.ctypes.data, ctypes.byref(sp),
                                             _stream(stream)))
        return sp.value, ms

    def set_timing(self, enable: bool):
        _check(lib().bnq_plan_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> dict:
        ms = np.zeros(NKERNELS)
        n = np.zeros(NKERNELS, dtype=np.int64)
        _check(lib().bnq_plan_timing(self._h, ms.ctypes.data, n.ctypes.data))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_FAMILIES)}


def tune_get(d: int, N: int, precision: int):
    """bnq_tune_get: the recorded trilinear work distribution (0 .. 3) for
    (d, N, precision) on the current device, or None."""
    ch = ctypes.c_int32(-1)
    _check(lib().bnq_tune_get(int(d), int(N), int(precision), ctypes.byref(ch)))
    return None if ch.value < 0 else ch.value


def tune_set(d: int, N: int, precision: int, choice):
    """bnq_tune_set: record a choice (None removes the record)."""
    _check(lib().bnq_tune_set(int(d), int(N), int(precision), -1 if choice is None else int(choice)))


def tune_pairs_get(d: int, N: int, precision: int, eps: int):
    """bnq_tune_pairs_get: the recorded pair-sum slices for (d, N, precision,
    eps == 0) on the current device, or None."""
    sp = ctypes.c_int32(0)
    _check(lib().bnq_tune_pairs_get(int(d), int(N), int(precision), int(eps), ctypes.byref(sp)))
    return sp.value or None


def tune_pairs_set(d: int, N: int, precision: int, eps: int, split):
    """bnq_tune_pairs_set: record a pair-sum split (None removes the record)."""
    _check(lib().bnq_tune_pairs_set(int(d), int(N), int(precision), int(eps), 0 if split is None else int(split)))


def save_tuning(path: str, cells, ms=None, device: str = "", pair_cells=(), pair_ms=None):
    """Write the recorded choices to a JSON file, merged into what the file
    already holds (the entries of other cells stay):
      cells [(d, N, precision)]: the trilinear work distribution ('choice');
      pair_cells [(d, N, precision, eps)]: the pair-sum split ('pair_split',
      keyed by eps == 0 as 'eps0');
    ms / pair_ms: optional {cell: candidate times in ms} kept beside them."""
    import json
    data = {"format": "bnq-tuning-1", "device": device, "entries": []}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)

    def key(e):
        return (e["d"], e["N"], e["precision"], "pairs" if "pair_split" in e else "trilinear", e.get("eps0", -1))
    ent = {key(e): e for e in data.get("entries", [])}
    for d, N, prec in cells:
        ch = tune_get(d, N, prec)
        if ch is None:
            continue
        e = {"d": int(d), "N": int(N), "precision": int(prec), "choice": int(ch)}
        if ms and (d, N, prec) in ms:
            e["ms"] = [float(x) for x in ms[(d, N, prec)]]
        ent[key(e)] = e
    for d, N, prec, eps in pair_cells:
        sp = tune_pairs_get(d, N, prec, eps)
        if sp is None:
            continue
        e = {"d": int(d), "N": int(N), "precision": int(prec), "eps0": int(eps == 0), "pair_split": int(sp)}
        if pair_ms and (d, N, prec, eps) in pair_ms:
            e["ms"] = [float(x) for x in pair_ms[(d, N, prec, eps)]]
        ent[key(e)] = e
    data["entries"] = [ent[k] for k in sorted(ent)]
    if device:
        data["device"] = device
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1)
    os.replace(tmp, path)
    return len(data["entries"])


def load_tuning(path: str) -> int:
    """Record every choice of a file written by save_tuning for the current
    device (plans created afterwards start with them); returns the count."""
    import json
    with open(path) as fh:
        data = json.load(fh)
    if data.get("format") != "bnq-tuning-1":
        raise ValueError(f"{path}: not a bnq tuning file")
    for e in data["entries"]:
        if "pair_split" in e:
            tune_pairs_set(e["d"], e["N"], e["precision"], 0 if e["eps0"] else 1, e["pair_split"])
        else:
            tune_set(e["d"], e["N"], e["precision"], e["choice"])
    return len(data["entries"])


class Batch:
    """A libbnq batch (bnq_batch_create / bnq_batch_destroy): plans[i] with
    state tensor f[i], evaluated together.  Keeps references to both."""

    def __init__(self, plans, f):
        if len(plans) != len(f) or not plans:
            raise ValueError("need as many state tensors as plans (at least one)")
        self.plans = list(plans)
        self.f = list(f)
        n = len(plans)
        ph = (ctypes.c_void_p * n)(*[pl._h.value for pl in plans])
        fp = (ctypes.c_void_p * n)(*[_ptr(x) for x in f])
        self._h = ctypes.c_void_p()
        _check(lib().bnq_batch_create(n, ph, fp, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(lib().bnq_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def layout(self):
        """(groups, shared trilinear launches per stage)."""
        g, t = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().bnq_batch_layout(self._h, ctypes.byref(g), ctypes.byref(t)))
        return g.value, t.value

    def collide(self, Q, Qhat=None, stream=None):
        n = len(self.plans)
        qp = (ctypes.c_void_p * n)(*[_ptr(x) for x in Q])
        hp = None if Qhat is None else (ctypes.c_void_p * n)(*[_ptr(x) for x in Qhat])
        _check(lib().bnq_batch_collide(self._h, qp, hp, _stream(stream)))

    def step(self, dt, scheme: int = RK4, graph: bool = False, stream=None):
        n = len(self.plans)
        dts = np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).copy()
        _check(lib().bnq_batch_step(self._h, dts.ctypes.data, int(scheme), 1 if graph else 0, _stream(stream)))


def moments_noalloc(p: Params, f, out, stream=None):
    """bnq_moments_noalloc: moments of device array f into the device array
    out (MOMENTS_LEN + 1 FP64 values, the last the non-finite count),
    asynchronously, with no allocation."""
    cp = p._c()
    _check(lib().bnq_moments_noalloc(ctypes.byref(cp), _ptr(f), _ptr(out), _stream(stream)))


def terms_per_eval(p: Params, counts: dict) -> float:
    """Collision terms of one evaluation with the selected terms (plain
    Galerkin counts: classical pairs, W pairs, outer pairs, trilinear)."""
    t = p.terms if p.eps != 0 else (p.terms & T_CLASSICAL)
    n = 0.0
    if t & T_CLASSICAL:
        n += counts["classical"]
    if t & T_QMULT:
        n += counts["w_pairs"] + counts["outer"]
    if t & T_QTRI:
        n += counts["trilinear"]
    return n
