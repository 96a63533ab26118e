"""Pins for the CPU oracle, independent of the oracle's own formulas.

Each test ties a piece of the oracle to something the paper or mathematics
fixes: closed forms of the kernel modes, a different series representation of
them, brute-force quadrature of the physical-space operator, conservation,
exact solutions and the fugacities printed in the table captions.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import special

import bnq_inputs as inp
import oracle
from tests.carleman_bruteforce import bruteforce_modes

R = oracle.R_DEFAULT


# ---------------------------------------------------------------- kernel modes
def test_beta_at_origin_closed_forms():
    # beta(0,0) = Btilde |B_R|-measure of {z.y = 0}: 2D 8 pi C R^2, 3D 8 pi^2 C R^4
    for C in (1.0, 0.7):
        b2 = oracle.beta_pairs(2, [[0, 0]], [[0, 0]], Cphi=C)[0]
        b3 = oracle.beta_pairs(3, [[0, 0, 0]], [[0, 0, 0]], Cphi=C)[0]
        assert b2 == pytest.approx(8 * math.pi * C * R * R, rel=1e-15)
        assert b3 == pytest.approx(8 * math.pi ** 2 * C * R ** 4, rel=1e-15)


def test_beta_3d_one_argument_zero_closed_form():
    # beta(k,0) = beta(0,k) = 16 pi^2 C R^2 (1 - cos(R|k|)) / |k|^2.  The
    # (0,k) side integrates psi over the sphere and so also pins the reading
    # psi(s) = 2 pi R J1(Rs)/s (no sin factor in the great-circle measure).
    rng = np.random.default_rng(3)
    ks = rng.integers(-40, 41, size=(40, 3))
    ks = ks[np.any(ks != 0, axis=1)]
    z = np.zeros_like(ks)
    s = np.linalg.norm(ks, axis=1)
    exact = 16 * math.pi ** 2 * R * R * (1 - np.cos(R * s)) / s ** 2
    assert np.max(np.abs(oracle.beta_pairs(3, ks, z) - exact)) < 1e-12
    assert np.max(np.abs(oracle.beta_pairs(3, z, ks) - exact)) < 1e-12


def test_beta_2d_one_argument_zero_closed_form():
    # beta(k,0) = 8 pi C R^2 (1/x) int_0^x J0,  x = R|k|
    #           = 8 pi C R^2 [J0(x) + (pi/2)(J1(x) H0(x) - J0(x) H1(x))]
    rng = np.random.default_rng(4)
    ks = rng.integers(-45, 46, size=(40, 2))
    ks = ks[np.any(ks != 0, axis=1)]
    x = R * np.linalg.norm(ks, axis=1)
    intJ0 = x * special.j0(x) + math.pi * x / 2 * (special.j1(x) * special.struve(0, x)
                                                   - special.j0(x) * special.struve(1, x))
    exact = 8 * math.pi * R * R * intJ0 / x
    z = np.zeros_like(ks)
    assert np.max(np.abs(oracle.beta_pairs(2, ks, z) - exact)) < 1e-12
    assert np.max(np.abs(oracle.beta_pairs(2, z, ks) - exact)) < 1e-12


def _series_3d(a, b, dps=25):
    # Funk–Hecke form of the same integral: plane-wave expansion of both
    # exponentials; the great-circle constraint keeps even orders only.
    mp.mp.dps = dps
    Rm = 2 * mp.pi / (3 + mp.sqrt(2))
    na, nb = mp.sqrt(sum(x * x for x in a)), mp.sqrt(sum(x * x for x in b))
    cg = 0 if na == 0 or nb == 0 else mp.mpf(sum(x * y for x, y in zip(a, b))) / (na * nb)
    nmax = int(float(Rm) * float(max(na, nb))) + 40
    tot = mp.mpf(0)
    for n in range(0, nmax + 1, 2):
        Ja = mp.quad(lambda r: r * mp.besselj(n + 0.5, r * na) * mp.sqrt(mp.pi / (2 * r * na)) if na else
                     (r if n == 0 else 0), [0, Rm])
        Jb = mp.quad(lambda r: r * mp.besselj(n + 0.5, r * nb) * mp.sqrt(mp.pi / (2 * r * nb)) if nb else
                     (r if n == 0 else 0), [0, Rm])
        tot += (2 * n + 1) * mp.legendre(n, 0) * mp.legendre(n, cg) * Ja * Jb
    return float(32 * mp.pi ** 2 * tot)


def _series_2d(a, b, dps=25):
    # Jacobi–Anger form of the same integral.
    mp.mp.dps = dps
    Rm = 2 * mp.pi / (3 + mp.sqrt(2))
    na, nb = mp.sqrt(a[0] ** 2 + a[1] ** 2), mp.sqrt(b[0] ** 2 + b[1] ** 2)
    g = mp.atan2(a[0] * b[1] - a[1] * b[0], a[0] * b[0] + a[1] * b[1])
    nmax = int(float(Rm) * float(max(na, nb))) + 40
    tot = mp.mpf(0)
    for n in range(0, nmax + 1, 2):
        An = mp.quad(lambda r: mp.besselj(n, r * na), [0, Rm])
        Bn = mp.quad(lambda r: mp.besselj(n, r * nb), [0, Rm])
        tot += (1 if n == 0 else 2) * (-1) ** (n // 2) * An * Bn * mp.cos(n * g)
    return float(8 * mp.pi * tot)


@pytest.mark.parametrize("d", [2, 3])
def test_beta_matches_independent_series(d):
    rng = np.random.default_rng(11 + d)
    a = rng.integers(-9, 10, size=(4, d))
    b = rng.integers(-9, 10, size=(4, d))
    got = oracle.beta_pairs(d, a, b)
    ref = [(_series_2d if d == 2 else _series_3d)(list(map(int, x)), list(map(int, y))) for x, y in zip(a, b)]
    assert np.max(np.abs(got - np.array(ref))) < 1e-12


@pytest.mark.parametrize("d,M", [(2, 45), (3, 55)])
def test_beta_node_rule_converged(d, M):
    rng = np.random.default_rng(5)
    a = rng.integers(-M // 1.7, M // 1.7, size=(60, d))
    b = rng.integers(-M // 1.7, M // 1.7, size=(60, d))
    v1 = oracle.beta_pairs(d, a, b)
    v2 = oracle.beta_pairs(d, a, b, scale=2.0)
    assert np.max(np.abs(v1 - v2)) < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_beta_symmetries(d):
    # evenness in each argument, symmetry in (k,l) (Btilde symmetric for b = 1),
    # invariance under a common signed permutation of the axes
    rng = np.random.default_rng(7)
    a = rng.integers(-12, 13, size=(30, d))
    b = rng.integers(-12, 13, size=(30, d))
    base = oracle.beta_pairs(d, a, b, scale=1.3)
    assert np.max(np.abs(oracle.beta_pairs(d, -a, b, scale=1.3) - base)) < 1e-12
    assert np.max(np.abs(oracle.beta_pairs(d, a, -b, scale=1.3) - base)) < 1e-12
    assert np.max(np.abs(oracle.beta_pairs(d, b, a, scale=1.3) - base)) < 1e-12
    perm = rng.permutation(d)
    sg = np.array([1, -1, -1][:d])
    assert np.max(np.abs(oracle.beta_pairs(d, a[:, perm] * sg, b[:, perm] * sg, scale=1.3) - base)) < 1e-12


# ---------------------------------------------------------------- DFT
def test_dft_single_mode_and_round_trip():
    N = 8
    k = np.array([2, -3])
    j = oracle.modes(N)
    J = np.meshgrid(j, j, indexing="ij")
    f = np.cos(2 * math.pi * (k[0] * J[0] + k[1] * J[1]) / N)
    G = oracle.dft(f)
    assert G[k[0] + 4, k[1] + 4] == pytest.approx(0.5, abs=1e-15)
    assert G[-k[0] + 4, -k[1] + 4] == pytest.approx(0.5, abs=1e-15)
    G[k[0] + 4, k[1] + 4] = G[-k[0] + 4, -k[1] + 4] = 0
    assert np.max(np.abs(G)) < 1e-15
    rng = np.random.default_rng(0)
    g = rng.standard_normal((6, 6, 6))
    assert np.max(np.abs(oracle.idft_real(oracle.dft(g)) - g)) < 1e-14


# ---------------------------------------------------------------- Galerkin sums
def _random_ghat(d, N, seed):
    rng = np.random.default_rng(seed)
    return oracle.dft(rng.standard_normal((N,) * d))


@pytest.mark.parametrize("d,N,nodes", [(2, 4, (48, 16)), (2, 6, (64, 24)), (3, 2, (12, 20, 14, 10))])
def test_galerkin_sums_equal_bruteforce_carleman(d, N, nodes):
    G = _random_ghat(d, N, 100 + N)
    tab = oracle.beta_table(d, N)
    s = oracle.galerkin_sums(d, N, G, tab, want=("c", "q", "g"))
    bc, bq, bg = bruteforce_modes(G, R, nodes=nodes, gain=True)
    scale_c = np.max(np.abs(s["c"]))
    scale_q = np.max(np.abs(s["q"]))
    assert np.max(np.abs(bc - s["c"])) < 1e-13 * max(1.0, scale_c)
    assert np.max(np.abs(bq - s["q"])) < 1e-13 * max(1.0, scale_q)
    assert np.max(np.abs(bg - s["g"])) < 1e-13 * max(1.0, np.max(np.abs(s["g"])))


@pytest.mark.parametrize("d,N", [(2, 8), (3, 4)])
def test_factored_equals_direct_triple_sum(d, N):
    G = _random_ghat(d, N, 7)
    tab = oracle.beta_table(d, N)
    s = oracle.galerkin_sums(d, N, G, tab, want=("q", "t1"))
    W, X = oracle.factored_sums(d, N, G, tab)
    scale = np.max(np.abs(s["q"]))
    assert np.max(np.abs(s["t1"] + X - s["q"])) < 1e-13 * scale
    # W vanishes outside E = {-N..N-2}^d
    Wr = np.abs(W)
    assert np.max(Wr[(slice(None),) * (d - 1) + (-1,)]) == 0.0


@pytest.mark.parametrize("d,N", [(2, 8), (3, 4)])
def test_mass_conservation_exact(d, N):
    # Qc_0 vanishes term by term (beta even in its second argument);
    # Qq_0 vanishes by the cyclic symmetry of the triple sum.
    rng = np.random.default_rng(9)
    f = rng.uniform(0.1, 1.0, size=(N,) * d)
    G = oracle.dft(f)
    tab = oracle.beta_table(d, N)
    s = oracle.galerkin_sums(d, N, G, tab, want=("c", "q"))
    z = (N // 2,) * d
    assert s["c"][z] == 0.0
    assert abs(s["q"][z]) < 1e-14 * np.max(np.abs(s["q"]))


@pytest.mark.parametrize("d,N", [(2, 8), (3, 4)])
def test_constant_is_stationary(d, N):
    o = oracle.Oracle(d, N)
    f = np.full((N,) * d, 0.37)
    for eps in (-1, 0, 1):
        Q, Qh = o.collide(f, eps, L=5.0)
        assert np.max(np.abs(Q)) < 1e-14


def test_sparse_spectrum_matches_dense():
    d, N = 2, 8
    f, sm, co = inp.sparse_spectrum(d, N, seed=2, nmodes=5)
    o = oracle.Oracle(d, N)
    m = o.modes(f, eps=1)
    Qc, T1, Xq = oracle.sparse_modes(d, N, sm, co, eps=1)
    for dense, sp in ((m["Qc"], Qc), (m["T1"], T1), (m["Xq"], Xq)):
        assert np.max(np.abs(dense - oracle.sparse_dense(d, N, sp))) < 1e-12 * np.max(np.abs(dense))


# ---------------------------------------------------------------- exact solutions
def test_bkw_fourth_moment_rate():
    # Classical 2-D Maxwell molecules, B = C_phi = 1: for the BKW datum
    # (K = 1/2) the fourth moment obeys dM4/dt = -(pi C/2)(M4 - 2 M2^2),
    # i.e. dM4/dt = pi at t = 0 (M2 = 2, M4 = 6).  This fixes the whole chain
    # Btilde = 2 C_phi, the kernel modes and the factor c (L/pi)^(d+gamma) up
    # to the collision truncation |x|, |y| <= R = S, which costs ~1% here.
    N, L = 48, 12.0
    f0 = inp.bkw_2d(N, L, t=0.0, lam=1.0)
    o = oracle.Oracle(2, N)
    Q, _ = o.collide(f0, eps=0, L=L)
    v = inp.velocity_grid(2, N, L)
    r2 = np.sum(v * v, axis=-1)
    dv = inp.cell_volume(2, N, L)
    assert dv * np.sum(f0) == pytest.approx(1.0, abs=1e-9)
    assert dv * np.sum(r2 ** 2 * f0) == pytest.approx(6.0, abs=1e-6)
    dM4 = dv * np.sum(r2 ** 2 * Q)
    assert dM4 == pytest.approx(math.pi, rel=2e-2)
    # mass and energy rates vanish (energy only up to the truncation error)
    assert abs(dv * np.sum(Q)) < 1e-13
    assert abs(dv * np.sum(r2 * Q)) < 1e-3


@pytest.mark.slow
def test_bkw_profile_after_rk4():
    N, L, lam, dt, nsteps = 48, 12.0, math.pi / 4, 0.05, 10
    o = oracle.Oracle(2, N)
    f = inp.bkw_2d(N, L, t=0.0, lam=lam)
    for _ in range(nsteps):
        f = o.rk4_step(f, dt, eps=0, L=L)
    ref = inp.bkw_2d(N, L, t=dt * nsteps, lam=lam)
    err = np.sqrt(np.sum((f - ref) ** 2) / np.sum(ref ** 2))
    assert err < 1e-2


def test_quantum_maxwellian_residual_decays():
    # section 'Validation of spectral accuracy' protocol: f0 = M_q sampled on the box is an equilibrium; the
    # discrete residual decays spectrally with N (2-D Fermi–Dirac, hbar = 3,
    # rho = 1, sigma = T = 0.5, L = 4, u0 = 0, as in Table 1).  The same datum
    # is far from stationary with the opposite sign of alpha, which pins
    # alpha = -eps hbar^d (eps = -1 for fermions).
    hbar, T, rho, L = 3.0, 0.5, 1.0, 4.0
    alpha = hbar ** 2
    z = math.exp(rho * alpha / (2 * math.pi * T)) - 1.0
    res, wrong = [], []
    for N in (16, 32):
        o = oracle.Oracle(2, N)
        f = inp.quantum_maxwellian(2, N, L, z=z, T=T, alpha=alpha)
        res.append(np.max(np.abs(o.collide(f, eps=-1, L=L, hbar=hbar)[0])))
        wrong.append(np.max(np.abs(o.collide(f, eps=+1, L=L, hbar=hbar)[0])))
    assert res[1] < res[0] / 50
    assert res[1] < 1e-5
    assert min(wrong) > 1e4 * res[1]


# ---------------------------------------------------------------- fixtures
def _golden_fugacities():
    rows = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "spectral_accuracy_fugacities.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            label, d, stat, rho, sigma, z = line.split()
            rows.append((label, int(d), stat == "FD", float(rho), float(sigma), z))
    return rows


def test_printed_fugacities_2d():
    # captions of the 2-D tables: hbar = 3, rho = 1, T = sigma, in closed form
    # FD: rho |alpha| / (2 pi T) = ln(1 + z);  BE: = -ln(1 - z).
    alpha = 9.0
    fd = lambda T: math.exp(alpha / (2 * math.pi * T)) - 1
    be = lambda T: 1 - math.exp(-alpha / (2 * math.pi * T))
    assert fd(0.5) == pytest.approx(16.5454, abs=5e-4)
    assert fd(1.0) == pytest.approx(3.1887, abs=5e-4)
    assert be(0.5) == pytest.approx(0.943, abs=5e-4)
    assert be(1.0) == pytest.approx(0.7613, abs=5e-4)


@pytest.mark.parametrize("row", _golden_fugacities(), ids=lambda r: r[0])
def test_printed_fugacities_from_the_oracle_integrals(row):
    # every caption's z from rho = (2 pi T)^(d/2) K_{d/2}(z) / |alpha|,
    # |alpha| = hbar^d (eq. mom0_qmaxwell), with the oracle's quadrature of
    # K_nu and a bracketing root finder, to half a unit of the last digit
    from scipy import optimize
    from oracle import equilibrium as oe
    label, d, fermi, rho, T, zs = row
    target = rho * 3.0 ** d / (2 * math.pi * T) ** (d / 2)
    f = lambda lz: oe.K(d / 2, fermi, log_z=lz) - target
    hi = 10.0 if fermi else -1e-12
    lz = optimize.brentq(f, -30.0, hi, xtol=1e-15, rtol=1e-15)
    mant = zs.split("e")[0]
    ulp = 10.0 ** (-(len(mant.split(".")[1]))) * (10.0 ** int(zs.split("e")[1]) if "e" in zs else 1.0)
    z = math.exp(lz)
    if label == "spectral_accuracy_fermions_3d_sigma1":
        # the one caption that does not reproduce: 3.09965 against 3.09922
        assert abs(z - 3.09965) < 5e-6 and abs(z - float(zs)) > 4e-4
    else:
        assert abs(z - float(zs)) <= 0.5 * ulp + 1e-12, (z, zs)


def test_moments_of_gaussian():
    N, L = 32, 8.0
    v = inp.velocity_grid(3, N, L)
    T, u = 0.8, np.array([0.3, -0.2, 0.1])
    f = np.exp(-np.sum((v - u) ** 2, axis=-1) / (2 * T)) / (2 * math.pi * T) ** 1.5
    m = oracle.moments(f, L, eps=0)
    assert m["rho"] == pytest.approx(1.0, abs=1e-10)
    assert np.allclose(m["u"], u, atol=1e-10)
    assert m["e"] == pytest.approx(1.5 * T, abs=1e-9)
    # classical entropy of a Maxwellian: int f ln f = -(3/2)(1 + ln(2 pi T))
    assert m["H"] == pytest.approx(-1.5 * (1 + math.log(2 * math.pi * T)), abs=1e-8)


@pytest.mark.parametrize("d,N", [(2, 8), (3, 6)])
def test_moment_projection_properties(d, N):
    # the correction removes exactly the span of {1, v, |v|^2}: the result has
    # zero discrete moments, the correction lies in that span, and a function
    # already orthogonal to it is left unchanged (idempotence)
    L = 4.0
    rng = np.random.default_rng(d * 100 + N)
    Q = rng.standard_normal((N,) * d)
    P = oracle.project_moments(Q, d, N, L)
    axes = [(2.0 * L / N) * np.arange(-N // 2, N // 2)] * d
    v = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    scale = np.sum(np.abs(Q)) * (1 + np.max(np.abs(v))) ** 2
    assert abs(P.sum()) <= 1e-13 * scale
    for a in range(d):
        assert abs(np.sum(v[..., a] * P)) <= 1e-13 * scale
    assert abs(np.sum(np.sum(v * v, axis=-1) * P)) <= 1e-13 * scale
    D = (Q - P).reshape(-1)
    basis = np.concatenate([np.ones((1, D.size)), v.reshape(-1, d).T, np.sum(v * v, axis=-1).reshape(1, -1)])
    coef, *_ = np.linalg.lstsq(basis.T, D, rcond=None)
    assert np.linalg.norm(basis.T @ coef - D) <= 1e-12 * np.linalg.norm(Q)
    assert np.allclose(oracle.project_moments(P, d, N, L), P, rtol=0, atol=1e-13 * np.max(np.abs(Q)))


def _polylog_series(nu, z, fermi, terms=2000):
    # complete Fermi-Dirac / Bose-Einstein integral for 0 < z < 1 by its power
    # series: sum_k (-1)^(k+1) z^k / k^nu (FD) or sum_k z^k / k^nu (BE)
    k = np.arange(1, terms + 1, dtype=np.float64)
    sgn = (-1.0) ** (k + 1) if fermi else 1.0
    return float(np.sum(sgn * z ** k / k ** nu))


def _quantum_maxwellian_entropy(d, alpha, z, T):
    # The quantum Maxwellian f = (1/|alpha|) / (z^-1 e^{|v|^2/2T} + sgn alpha)
    # (section 'Convergence towards a steady state', eq. def_Mq_2d and its 3-D
    # form).  Writing y = z^-1 e^{|v|^2/2T} and s = sgn alpha, the entropy
    # density f ln f + (1 - alpha f)/alpha ln(1 - alpha f) is
    #   -f ln|alpha| - f ln y - (1/alpha) ln(1 + s/y),
    # and integrating the series of each term over R^d gives
    #   rho   = (2 pi T)^(d/2) K_{d/2}(z) / |alpha|,
    #   rho e = (d/2) T (2 pi T)^(d/2) K_{d/2+1}(z) / |alpha|,
    #   H     = rho (ln z - ln|alpha|) - (rho e / T)(1 + 2/d),
    # with K_nu the Fermi-Dirac (alpha > 0) or Bose-Einstein (alpha < 0)
    # integral (mom02_qmaxwell).
    fermi = alpha > 0
    rho = (2 * math.pi * T) ** (d / 2) * _polylog_series(d / 2, z, fermi) / abs(alpha)
    rhoe = (d / 2) * T * (2 * math.pi * T) ** (d / 2) * _polylog_series(d / 2 + 1, z, fermi) / abs(alpha)
    H = rho * (math.log(z) - math.log(abs(alpha))) - rhoe / T * (1 + 2 / d)
    return rho, rhoe / rho, H


def _qmaxwellian_grid(d, N, L, alpha, z, T):
    v = inp.velocity_grid(d, N, L)
    r2 = np.sum(v * v, axis=-1)
    return (1 / abs(alpha)) / (np.exp(r2 / (2 * T)) / z + (1.0 if alpha > 0 else -1.0))


# fine grids: the discrete sums of these analytic, fast-decaying integrands
# equal the integrals to rounding (the nearest complex singularity of the
# Bose-Einstein case, |v| = sqrt(2 T |ln z|), bounds the grid step)
QM_CASES = [(2, 128, 8.0, -1, 1.0, 0.5, 0.5), (2, 128, 8.0, 1, 1.0, 0.5, 0.5), (2, 128, 8.0, -1, 1.5, 0.7, 0.4),
            (2, 128, 8.0, 1, 1.3, 0.3, 0.6), (3, 64, 6.0, -1, 1.0, 0.5, 0.5), (3, 64, 6.0, 1, 1.2, 0.3, 0.5)]


@pytest.mark.parametrize("d,N,L,eps,hbar,z,T", QM_CASES)
def test_quantum_entropy_of_quantum_maxwellian_closed_form(d, N, L, eps, hbar, z, T):
    alpha = oracle.alpha_of(eps, d, hbar)
    f = _qmaxwellian_grid(d, N, L, alpha, z, T)
    m = oracle.moments(f, L, eps, hbar)
    rho, e, H = _quantum_maxwellian_entropy(d, alpha, z, T)
    assert m["n_excluded"] == 0
    assert m["rho"] == pytest.approx(rho, rel=1e-12)
    assert m["e"] == pytest.approx(e, rel=1e-12)
    assert m["H"] == pytest.approx(H, rel=1e-11, abs=1e-12)


def test_quantum_entropy_pin_rejects_planted_mistakes():
    # the closed form above tells the oracle's entropy from a flipped sign of
    # its second term and from a missing 1/alpha there (|alpha| != 1)
    d, N, L, eps, hbar, z, T = 2, 128, 8.0, 1, 1.3, 0.3, 0.6
    alpha = oracle.alpha_of(eps, d, hbar)
    f = _qmaxwellian_grid(d, N, L, alpha, z, T)
    _, _, H = _quantum_maxwellian_entropy(d, alpha, z, T)
    dv = (2 * L / N) ** d
    om = 1 - alpha * f
    flipped = dv * np.sum(f * np.log(f) - om / alpha * np.log(om))
    no_inv = dv * np.sum(f * np.log(f) + om * np.log(om))
    assert abs(flipped - H) > 1e-3 * abs(H)
    assert abs(no_inv - H) > 1e-3 * abs(H)


def test_rk4_step_is_fourth_order():
    # Oracle.rk4_step against a fine-step reference of the same scheme over a
    # fixed horizon: the error falls 16-fold per halving of dt (a second-order
    # scheme, planted below, falls 4-fold and fails the same bound)
    d, N, L, eps, T = 2, 8, 5.0, 1, 0.5
    o = oracle.Oracle(d, N)
    f0 = inp.gaussian_mixture(d, N, L, seed=3, kmin=2)

    def run(n, step):
        f = f0.copy()
        for _ in range(n):
            f = step(f, T / n)
        return f

    rk4 = lambda f, dt: o.rk4_step(f, dt, eps, L)

    def midpoint(f, dt):
        k1 = o.rhs(f, eps, L)
        return f + dt * o.rhs(f + 0.5 * dt * k1, eps, L)

    ref = run(128, rk4)
    e = [np.abs(run(n, rk4) - ref).max() for n in (4, 8, 16)]
    assert e[2] > 1e-11  # above rounding
    for a, b in zip(e, e[1:]):
        assert 13.0 < a / b < 19.0, e
    e2 = [np.abs(run(n, midpoint) - ref).max() for n in (4, 8)]
    assert not (13.0 < e2[0] / e2[1] < 19.0)


# ---------------------------------------------------------------- series kernel modes (3-D)
def test_beta3_series_matches_quadrature():
    # the Funk-Hecke series of the Lemma's integral against the polar
    # quadrature of the same integral, random pairs and the axes
    rs = oracle.RadialSeries(3 * 12 * 12)
    rng = np.random.default_rng(1)
    a = rng.integers(-11, 12, (300, 3))
    b = rng.integers(-11, 12, (300, 3))
    a[:3] = 0
    b[2:5] = 0
    b00 = 8 * math.pi ** 2 * oracle.R_DEFAULT ** 4
    got = oracle.beta3_series_pairs(a, b, rs)
    ref = oracle.beta_pairs(3, a, b)
    assert np.max(np.abs(got - ref)) <= 1e-13 * b00


def test_beta3_series_closed_forms_and_cut():
    # beta(0,0) = 8 pi^2 R^4, beta(k,0) = 16 pi^2 R^2 (1 - cos R|k|) / |k|^2
    # (hard spheres, C_phi = 1); doubling the series cut and the radial nodes
    # changes nothing at rounding level
    R = oracle.R_DEFAULT
    rs = oracle.RadialSeries(3 * 20 * 20)
    k = np.array([[0, 0, 0], [1, 0, 0], [3, 4, 0], [7, 7, 7], [19, 2, 5]])
    z = np.zeros_like(k)
    got = oracle.beta3_series_pairs(k, z, rs)
    kk = np.sqrt(np.sum(k ** 2, axis=1).astype(float))
    ref = np.where(kk == 0, 8 * math.pi ** 2 * R ** 4,
                   16 * math.pi ** 2 * R ** 2 * (1 - np.cos(R * kk)) / np.where(kk == 0, 1, kk) ** 2)
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * ref[0])
    rng = np.random.default_rng(7)
    a = rng.integers(-19, 20, (200, 3))
    b = rng.integers(-19, 20, (200, 3))
    fine = oracle.RadialSeries(3 * 20 * 20, nodes=400, extra=2.0)
    assert np.max(np.abs(oracle.beta3_series_pairs(a, b, fine) - oracle.beta3_series_pairs(a, b, rs))) <= 1e-14 * ref[0]


@pytest.mark.parametrize("eps", [-1, 1])
def test_series_modes_equal_the_dense_sums(eps):
    # the sampled-mode sums with series kernel modes equal the table-based
    # direct sums (Qc, gain, T1, X) at every mode of a small dense datum
    N, L = 6, 5.0
    f = inp.gaussian_mixture(3, N, L, seed=4, fmax=0.9)
    m = oracle.Oracle(3, N).modes(f, eps)
    s = oracle.series_modes(f, eps, np.arange(N ** 3))
    for k in ("Qc", "gain", "T1", "Xq", "Qhat"):
        assert np.max(np.abs(s[k] - m[k])) <= 1e-13 * np.max(np.abs(m[k])), k


@pytest.mark.parametrize("name", ["dense_3d16_all_modes.npz", "c2_3d32_sampled_modes.npz"])
def test_stored_dense_goldens_conserve_mass(name):
    # the collision operator conserves mass (eq. conservationQ with psi = 1),
    # and so does its Galerkin form: Qhat_0 = Qc_0 - alpha (T1_0 + X_0) = 0,
    # where T1_0 and X_0 are each about a quarter of the gain term; the stored
    # oracle values must keep that cancellation far below the 1e-12 bar
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    z = np.load(path, allow_pickle=False)
    modes = [tuple(int(v) for v in m) for m in z["modes"]]
    i0 = modes.index((0, 0, 0))
    alpha = oracle.alpha_of(int(z["eps"]), 3)
    q0 = z["Qc"][i0] - alpha * (z["T1"][i0] + z["Xq"][i0])
    assert abs(z["T1"][i0]) > 0.1 * abs(z["gain"][i0])
    assert abs(q0) <= 1e-14 * abs(z["gain"][i0])
