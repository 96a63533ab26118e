"""CPU oracle for the spectral-Galerkin Boltzmann–Nordheim collision operator.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library and its
Python binding never import, link or call it, and the two share no code.

What it computes (Mouton & Rey, arXiv 2110.13735), plainly and in FP64:

* Fourier modes of the grid data (section 'Numerical scheme for the velocity rescaled BNE', step 2(a), with the d-dimensional
  normalisation N^-d):   G_k = N^-d sum_{j in I_N} f_j e^{-2 pi i k.j/N}.
* Kernel modes beta(k,l) by quadrature of their definition (Lemma of section
  'Fast spectral approximation of the BNE operator', polar forms of section 'Expansion of the kernel modes'); see bnq_oracle.c.
* The Galerkin sums of that Lemma for F = G = H, assembled as in the
  decomposition of section 'The Carleman representation':
      Qhat_n = Qc_n - alpha Qq_n,  alpha = -eps hbar^d  (eps = +1 boson,
      -1 fermion, 0 classical; the paper's alpha is +hbar^d for Fermi–Dirac).
* The classical method of section 'Application to the space homogeneous BNE' (lambda = 0, omega = 1, mu = (L/pi)^d):
      d f_j/dt = c (L/pi)^(d+gamma) Q_j,
      Q_j = Re sum_{n in I_N} Qhat_n e^{2 pi i n.j/N},
  with gamma = 0 (2-D Maxwell molecules) or 1 (3-D hard spheres), advanced by
  the classical fourth-order Runge–Kutta scheme.
* Discrete moments and entropy of section 'Numerical results' (diagnostics list).

R = S = 2 pi/(3 + sqrt 2) (section 'Validation of spectral accuracy').  Functions with no independent pin
are marked "parity unpinned" in their docstrings.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")
R_DEFAULT = 2.0 * math.pi / (3.0 + math.sqrt(2.0))

_lib = None


def build(force: bool = False) -> str:
    """Compile bnq_oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    src = os.path.join(HERE, "bnq_oracle.c")
    if force or not os.path.exists(LIBPATH) or os.path.getmtime(LIBPATH) < os.path.getmtime(src):
        tmp = LIBPATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIBPATH)
    return LIBPATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIBPATH)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.or_beta_pairs.argtypes = [i32, f64, f64, i64, vp, vp, vp, f64]
        L.or_beta_pairs.restype = None
        L.or_xsize.argtypes = [i32, i32]
        L.or_xsize.restype = i64
        L.or_beta_table.argtypes = [i32, i32, f64, f64, vp]
        L.or_beta_table.restype = i32
        L.or_sums_direct.argtypes = [i32, i32, vp, vp, i32, i64, vp, vp, vp, vp, vp]
        L.or_sums_direct.restype = None
        L.or_factored.argtypes = [i32, i32, vp, vp, vp, vp]
        L.or_factored.restype = None
        L.or_num_threads.restype = i32
        L.or_beta3_inv.argtypes = [f64, f64, f64, f64, f64, i32, i32]
        L.or_beta3_inv.restype = f64
        L.or_beta2_vec.argtypes = [f64, f64, f64, f64, f64, f64, i32]
        L.or_beta2_vec.restype = f64
        L.or_beta3_series_pairs.argtypes = [i64, vp, vp, vp, vp, i32, vp, f64]
        L.or_beta3_series_pairs.restype = None
        L.or_series_modes.argtypes = [i32, vp, vp, i32, vp, f64, i32, i64, vp, vp, vp, vp, vp, vp]
        L.or_series_modes.restype = None
        L.or_w_series.argtypes = [i32, vp, vp, i32, vp, f64, vp]
        L.or_w_series.restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


# --------------------------------------------------------------------------
# geometry
def gamma_of(d: int) -> int:
    """VHS exponent: 2-D Maxwell molecules (gamma = 0), 3-D hard spheres (1)."""
    return 0 if d == 2 else 1


def prefactor(d: int, L: float, c: float = 1.0) -> float:
    """c (L/pi)^(d+gamma): classical method of section 'Application to the space homogeneous BNE'."""
    return c * (L / math.pi) ** (d + gamma_of(d))


def alpha_of(eps: int, d: int, hbar: float = 1.0) -> float:
    """alpha = -eps hbar^d (paper: +hbar^d Fermi–Dirac, -hbar^d Bose–Einstein)."""
    return -float(eps) * hbar ** d


def modes(N: int) -> np.ndarray:
    return np.arange(-(N // 2), N // 2)


def _as3(G: np.ndarray, d: int) -> np.ndarray:
    return G.reshape((1,) + G.shape) if d == 2 else G


# --------------------------------------------------------------------------
# discrete Fourier transform (plain definition, one axis at a time)
def _dft_matrix(N: int, sign: int) -> np.ndarray:
    j = modes(N)
    kj = np.mod(np.outer(j, j), N).astype(np.float64)
    return np.exp(sign * 2j * math.pi * kj / N)


def dft(f: np.ndarray) -> np.ndarray:
    """G_k = N^-d sum_{j in I_N} f_j e^{-2 pi i k.j/N}; array indexed k + N/2."""
    d, N = f.ndim, f.shape[0]
    F = _dft_matrix(N, -1)
    out = f.astype(np.complex128)
    for ax in range(d):
        out = np.moveaxis(np.tensordot(F, out, axes=([1], [ax])), 0, ax)
    return out / N ** d


def idft_real(Qh: np.ndarray) -> np.ndarray:
    """Q_j = Re sum_{n in I_N} Qhat_n e^{2 pi i n.j/N}."""
    d, N = Qh.ndim, Qh.shape[0]
    F = _dft_matrix(N, +1)
    out = Qh.astype(np.complex128)
    for ax in range(d):
        out = np.moveaxis(np.tensordot(F, out, axes=([1], [ax])), 0, ax)
    return np.ascontiguousarray(out.real)


# --------------------------------------------------------------------------
# kernel modes
def beta_pairs(d: int, a, b, Cphi: float = 1.0, R: float = R_DEFAULT, scale: float = 1.0) -> np.ndarray:
    """beta(a_i, b_i) for integer vectors (arrays of shape (n, d))."""
    a = np.asarray(a, dtype=np.int64).reshape(-1, d)
    b = np.asarray(b, dtype=np.int64).reshape(-1, d)
    n = a.shape[0]
    A = np.zeros((n, 3), dtype=np.int32)
    B = np.zeros((n, 3), dtype=np.int32)
    A[:, 3 - d:] = a
    B[:, 3 - d:] = b
    out = np.zeros(n)
    lib().or_beta_pairs(d, R, Cphi, n, A.ctypes.data, B.ctypes.data, out.ctypes.data, scale)
    return out


def beta_table(d: int, N: int, Cphi: float = 1.0, R: float = R_DEFAULT) -> np.ndarray:
    """Dense beta(a, b) for a, b in X = {-N..N-1}^d, shape (|X|, |X|)."""
    X = int(lib().or_xsize(d, N))
    out = np.empty((X, X))
    lib().or_beta_table(d, N, R, Cphi, out.ctypes.data)
    return out


def xindex(d: int, N: int, a) -> np.ndarray:
    """Linear index of vectors a (shape (n, d)) in X = {-N..N-1}^d."""
    a = np.asarray(a, dtype=np.int64).reshape(-1, d) + N
    idx = np.zeros(a.shape[0], dtype=np.int64)
    for i in range(d):
        idx = idx * (2 * N) + a[:, i]
    return idx


# --------------------------------------------------------------------------
# Galerkin sums
def galerkin_sums(d: int, N: int, Ghat: np.ndarray, table: np.ndarray, want=("c", "q", "t1"),
                  select=None) -> dict:
    """Direct sums of the Fourier-modes Lemma for every n in I_N (or the
    linear indices in `select`).  Returns complex arrays shaped like Ghat
    (entries not selected are zero): 'c' = Qc, 'q' = Qq (all four quantum
    terms), 't1' = the Q_{1,q} term alone, 'g' = the classical gain term
    Q_{1,c} = sum beta(l,m) G_l G_m (used as the cancellation scale)."""
    G = np.ascontiguousarray(_as3(Ghat, d), dtype=np.complex128)
    out = {k: np.zeros(Ghat.size, dtype=np.complex128) for k in want}
    flag = (1 if "c" in want else 0) | (2 if "q" in want else 0) | (4 if "t1" in want else 0) | \
        (8 if "g" in want else 0)
    dummy = np.zeros(2)
    ptr = lambda k: out[k].ctypes.data if k in out else dummy.ctypes.data
    if select is None:
        nsel, sel = -1, np.zeros(1, dtype=np.int64)
    else:
        sel = np.ascontiguousarray(select, dtype=np.int64)
        nsel = sel.size
    lib().or_sums_direct(d, N, G.ctypes.data, table.ctypes.data, flag, nsel, sel.ctypes.data,
                         ptr("c"), ptr("q"), ptr("t1"), ptr("g"))
    return {k: v.reshape(Ghat.shape) for k, v in out.items()}


def factored_sums(d: int, N: int, Ghat: np.ndarray, table: np.ndarray):
    """(W over X, X_n over I_N): the pair sum with weight
    beta(l,m) - beta(l+m,l) - beta(l,l+m) and its convolution with G."""
    G = np.ascontiguousarray(_as3(Ghat, d), dtype=np.complex128)
    Xs = table.shape[0]
    W = np.zeros(Xs, dtype=np.complex128)
    Xo = np.zeros(Ghat.size, dtype=np.complex128)
    lib().or_factored(d, N, G.ctypes.data, table.ctypes.data, W.ctypes.data, Xo.ctypes.data)
    return W.reshape((2 * N,) * d), Xo.reshape(Ghat.shape)


# --------------------------------------------------------------------------
# the operator
class Oracle:
    """Plain evaluation of Q for one (d, N, C_phi); caches its beta table."""

    def __init__(self, d: int, N: int, Cphi: float = 1.0, R: float = R_DEFAULT):
        self.d, self.N, self.Cphi, self.R = d, N, Cphi, R
        self._table = None

    @property
    def table(self) -> np.ndarray:
        if self._table is None:
            self._table = beta_table(self.d, self.N, self.Cphi, self.R)
        return self._table

    def modes(self, f: np.ndarray, eps: int, hbar: float = 1.0, terms=("c", "x", "t1"), select=None):
        """Galerkin modes: dict with 'Ghat', 'Qc', 'T1', 'Xq' (= Qq - T1),
        'Qhat' = Qc - alpha (T1 + Xq) restricted to `terms`, and 'gain' (the
        classical gain term, a scale for judging cancellation)."""
        d, N = self.d, self.N
        G = dft(f)
        want = ["c", "g"]
        if eps != 0 and ("x" in terms or "t1" in terms):
            want += ["q", "t1"]
        s = galerkin_sums(d, N, G, self.table, want=tuple(want), select=select)
        alpha = alpha_of(eps, d, hbar)
        Qc = s["c"]
        T1 = s.get("t1", np.zeros_like(G))
        Xq = s["q"] - T1 if "q" in s else np.zeros_like(G)
        Qh = np.zeros_like(G)
        if "c" in terms:
            Qh = Qh + Qc
        if "t1" in terms:
            Qh = Qh - alpha * T1
        if "x" in terms:
            Qh = Qh - alpha * Xq
        return {"Ghat": G, "Qc": Qc, "T1": T1, "Xq": Xq, "Qhat": Qh, "gain": s["g"]}

    def collide(self, f: np.ndarray, eps: int, L: float, hbar: float = 1.0, c: float = 1.0,
                terms=("c", "x", "t1"), full: bool = False):
        """Q on the grid, already multiplied by c (L/pi)^(d+gamma), and Qhat
        (with full=True also the dict of modes)."""
        m = self.modes(f, eps, hbar, terms)
        Q = prefactor(self.d, L, c) * idft_real(m["Qhat"])
        if full:
            return Q, m["Qhat"], m
        return Q, m["Qhat"]

    def rhs(self, f, eps, L, hbar=1.0, c=1.0):
        return self.collide(f, eps, L, hbar, c)[0]

    def rk4_step(self, f: np.ndarray, dt: float, eps: int, L: float, hbar: float = 1.0, c: float = 1.0):
        """Classical RK4 for d f/dt = c (L/pi)^(d+gamma) Q(f)."""
        k1 = self.rhs(f, eps, L, hbar, c)
        k2 = self.rhs(f + 0.5 * dt * k1, eps, L, hbar, c)
        k3 = self.rhs(f + 0.5 * dt * k2, eps, L, hbar, c)
        k4 = self.rhs(f + dt * k3, eps, L, hbar, c)
        return f + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


# --------------------------------------------------------------------------
# 3-D kernel modes by their Funk–Hecke series (bnq_oracle.c, beta3_series):
# for full-size checks, where a quadrature per kernel mode is too slow
class RadialSeries:
    """Radial integrals J_n(s) = int_0^R r j_n(r s) dr at s = sqrt(q), q = 0 ..
    qmax, even n only (J[q, m] = J_{2m}), by Gauss-Legendre over spherical
    Bessel values (scipy), and the number of even orders kept per q: the
    series is cut where J_n(s) has fallen below rounding, n > R s +
    12 (R s)^(1/3) + 24 (doubling the cut changes nothing, tests)."""

    def __init__(self, qmax: int, R: float = R_DEFAULT, nodes: int = 200, extra: float = 1.0):
        from scipy.special import spherical_jn
        x, w = np.polynomial.legendre.leggauss(nodes)
        r = 0.5 * R * (x + 1.0)
        wr = 0.5 * R * w * r
        kap = np.sqrt(np.arange(qmax + 1, dtype=np.float64))
        ncut = np.ceil(extra * (R * kap + 12.0 * np.cbrt(R * kap) + 24.0)).astype(np.int64)
        self.mcut = np.ascontiguousarray(ncut // 2 + 1, dtype=np.int32)
        self.nm = int(self.mcut.max())
        orders = 2 * np.arange(self.nm)
        J = np.zeros((qmax + 1, self.nm))
        for q in range(qmax + 1):
            m = int(self.mcut[q])
            J[q, :m] = spherical_jn(orders[:m, None], r[None, :] * kap[q]) @ wr
        self.J = np.ascontiguousarray(J)
        self.qmax, self.R = qmax, R


def beta3_series_pairs(a, b, rs: RadialSeries, Cphi: float = 1.0) -> np.ndarray:
    """beta(a_i, b_i) for 3-D integer vectors (n x 3) by the series."""
    A = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 3))
    B = np.ascontiguousarray(np.asarray(b, dtype=np.int32).reshape(-1, 3))
    if max(np.max(np.sum(A.astype(np.int64) ** 2, axis=1)), np.max(np.sum(B.astype(np.int64) ** 2, axis=1))) > rs.qmax:
        raise ValueError("vector beyond the radial table")
    out = np.zeros(A.shape[0])
    lib().or_beta3_series_pairs(A.shape[0], A.ctypes.data, B.ctypes.data, out.ctypes.data, rs.J.ctypes.data, rs.nm,
                                rs.mcut.ctypes.data, Cphi)
    return out


def series_modes(f: np.ndarray, eps: int, select, hbar: float = 1.0, Cphi: float = 1.0, rs: RadialSeries = None):
    """3-D Galerkin modes at the output modes `select` (linear indices in I_N)
    with series kernel modes: dict of complex arrays over I_N (zero where not
    selected) 'Qc', 'gain', 'T1', 'Xq' and 'Qhat' = Qc - alpha (T1 + Xq), the
    quantum parts only when eps != 0.  W is summed over all of E first."""
    N = f.shape[0]
    if f.ndim != 3:
        raise ValueError("3-D data only")
    if rs is None:
        rs = RadialSeries(3 * N * N)
    G = np.ascontiguousarray(dft(f), dtype=np.complex128)
    sel = np.ascontiguousarray(select, dtype=np.int64)
    out = {k: np.zeros(G.size, dtype=np.complex128) for k in ("Qc", "gain", "T1", "Xq")}
    W = np.zeros((2 * N) ** 3, dtype=np.complex128)
    want = 1
    if eps != 0:
        lib().or_w_series(N, G.ctypes.data, rs.J.ctypes.data, rs.nm, rs.mcut.ctypes.data, Cphi, W.ctypes.data)
        want |= 2 | 4
    lib().or_series_modes(N, G.ctypes.data, rs.J.ctypes.data, rs.nm, rs.mcut.ctypes.data, Cphi, want, sel.size,
                          sel.ctypes.data, W.ctypes.data, out["Qc"].ctypes.data, out["gain"].ctypes.data,
                          out["T1"].ctypes.data, out["Xq"].ctypes.data)
    res = {k: v.reshape(G.shape) for k, v in out.items()}
    alpha = alpha_of(eps, 3, hbar)
    res["Qhat"] = res["Qc"] - alpha * (res["T1"] + res["Xq"])
    res["Ghat"] = G
    return res


# --------------------------------------------------------------------------
# sparse spectrum: exact sums over the support only
def sparse_modes(d: int, N: int, smodes: np.ndarray, coeffs: np.ndarray, eps: int, hbar: float = 1.0,
                 Cphi: float = 1.0, R: float = R_DEFAULT):
    """Galerkin sums for a spectrum supported on `smodes` (K x d) with values
    `coeffs`; every other mode is zero, so the sums reduce to the support.
    Returns (Qc, T1, Xq) as dicts {mode tuple: complex}."""
    h = N // 2
    K = len(smodes)
    sm = [tuple(int(x) for x in m) for m in smodes]
    val = {m: complex(c) for m, c in zip(sm, coeffs)}
    inI = lambda m: all(-h <= x < h for x in m)
    add = lambda u, v: tuple(x + y for x, y in zip(u, v))
    pairs, keyidx = [], {}

    def need(a, b):
        k = (a, b)
        if k not in keyidx:
            keyidx[k] = len(pairs)
            pairs.append(k)
        return keyidx[k]

    cl, tri = [], []
    for l in sm:
        for m in sm:
            n = add(l, m)
            if inI(n):
                cl.append((n, l, m, need(l, m), need(m, m)))
    if eps != 0:
        for k in sm:
            for l in sm:
                for m in sm:
                    n = add(add(k, l), m)
                    if inI(n):
                        tri.append((n, k, l, m, need(add(k, m), add(l, m)), need(l, m),
                                    need(add(l, m), l), need(l, add(l, m))))
    a = np.array([p[0] for p in pairs], dtype=np.int64).reshape(-1, d)
    b = np.array([p[1] for p in pairs], dtype=np.int64).reshape(-1, d)
    beta = beta_pairs(d, a, b, Cphi, R) if len(pairs) else np.zeros(0)
    Qc, T1, Xq = {}, {}, {}
    for n, l, m, i1, i2 in cl:
        Qc[n] = Qc.get(n, 0) + (beta[i1] - beta[i2]) * val[l] * val[m]
    for n, k, l, m, i1, i2, i3, i4 in tri:
        p = val[k] * val[l] * val[m]
        T1[n] = T1.get(n, 0) + beta[i1] * p
        Xq[n] = Xq.get(n, 0) + (beta[i2] - beta[i3] - beta[i4]) * p
    return Qc, T1, Xq


def sparse_dense(d: int, N: int, table: dict) -> np.ndarray:
    out = np.zeros((N,) * d, dtype=np.complex128)
    for m, v in table.items():
        out[tuple(x + N // 2 for x in m)] = v
    return out


# --------------------------------------------------------------------------
# moments and entropy (section 'Numerical results', diagnostics), classical method
def moments(f: np.ndarray, L: float, eps: int, hbar: float = 1.0) -> dict:
    """rho, u, E_c, e, entropy and extrema.  The entropy is
    Delta v sum [f ln f + (1 - alpha f)/alpha ln(1 - alpha f)] (alpha != 0) or
    Delta v sum f ln f (alpha = 0), summed over nodes with f > 0 and
    1 - alpha f > 0; `n_excluded` counts the other nodes."""
    d, N = f.ndim, f.shape[0]
    dv = (2.0 * L / N) ** d
    ax = 2.0 * L * modes(N) / N
    v = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1)
    rho = dv * f.sum()
    mom = dv * np.sum(v * f[..., None], axis=tuple(range(d)))
    u = mom / rho
    Ec = dv * np.sum(np.sum(v * v, axis=-1) * f)
    e = dv * np.sum(np.sum((v - u) ** 2, axis=-1) * f) / (2.0 * rho)
    alpha = alpha_of(eps, d, hbar)
    ok = f > 0
    if alpha != 0.0:
        ok &= (1.0 - alpha * f) > 0
    fo = f[ok]
    if alpha == 0.0:
        H = dv * np.sum(fo * np.log(fo))
    else:
        H = dv * np.sum(fo * np.log(fo) + (1.0 - alpha * fo) / alpha * np.log(1.0 - alpha * fo))
    return {"rho": rho, "u": u, "Ec": Ec, "e": e, "H": H, "fmax": float(f.max()),
            "fmin": float(f.min()), "n_excluded": int((~ok).sum())}


def project_moments(Q: np.ndarray, d: int, N: int, L: float) -> np.ndarray:
    """Conservation correction (not part of the paper's scheme): the grid
    function closest to Q in the discrete L2 norm whose discrete mass,
    momentum and kinetic energy vanish, i.e. Q minus its orthogonal projection
    onto span{1, v_1..v_d, |v|^2} over the velocity nodes v_j = 2 L j / N.
    Written as the definition: C Q' = 0 with Q' = Q - C^T (C C^T)^-1 C Q."""
    axes = [(2.0 * L / N) * np.arange(-N // 2, N // 2)] * d
    v = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d)
    C = np.concatenate([np.ones((1, v.shape[0])), v.T, np.sum(v * v, axis=1)[None, :]], axis=0)
    q = Q.reshape(-1)
    lam = np.linalg.solve(C @ C.T, C @ q)
    return (q - C.T @ lam).reshape(Q.shape)
