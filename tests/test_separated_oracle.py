"""Pins for the oracle of the separated kernel modes and the transform route
of the trilinear term (section 'Fast computation of the collision modes',
eqs. betadD, alphap, alphapprime; appendix 'Fast evaluation of the collision
kernel').

The transform route is held to the direct trilinear sum of liboracle run on
the same rank-P table (two different computations of one finite sum); the
rank-P table is held to the converged kernel modes, which the oracle's own
pins tie to closed forms."""
import math

import numpy as np
import pytest

import oracle
from oracle import separated as sp


def _random_spectrum(d, N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N,) * d) + 1j * rng.standard_normal((N,) * d)


def test_beta_separated_2d_equals_converged_modes():
    # the rectangle rule in the angle is spectrally accurate for this
    # pi-periodic integrand: at angles_2d(N) it reproduces beta to rounding
    N = 16
    rng = np.random.default_rng(1)
    a = rng.integers(-N, N, size=(400, 2))
    b = rng.integers(-N, N, size=(400, 2))
    ref = oracle.beta_pairs(2, a, b)
    got = sp.beta_separated(2, a, b, sp.angles_2d(N))
    scale = oracle.beta_pairs(2, [[0, 0]], [[0, 0]])[0]
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale
    # too few angles: visibly off (the pin can fail)
    bad = sp.beta_separated(2, a, b, sp.angles_2d(N) // 4)
    assert np.max(np.abs(bad - ref)) > 1e-6 * scale


def test_beta_separated_3d_converges_at_second_order():
    # the polar rule of eq. alphapprime is a trapezoid rule in theta for an
    # integrand that is not smooth-periodic there: error ~ M1^-2
    rng = np.random.default_rng(2)
    a = rng.integers(-5, 6, size=(60, 3))
    b = rng.integers(-5, 6, size=(60, 3))
    ref = oracle.beta_pairs(3, a, b)
    scale = oracle.beta_pairs(3, [[0, 0, 0]], [[0, 0, 0]])[0]
    errs = []
    for m in (16, 32, 64, 128):
        got = sp.beta_separated(3, a, b, (m, 2 * m))
        errs.append(np.max(np.abs(got - ref)) / scale)
    print("3-D separated beta, max error / beta(0,0):", ", ".join(f"{e:.2e}" for e in errs))
    for e0, e1 in zip(errs[1:], errs[2:]):
        assert 3.0 < e0 / e1 < 5.0
    assert errs[-1] < 1e-3


def test_beta_separated_at_origin_closed_form():
    # beta(0, 0) = 8 pi C R^2 in 2-D for every angle count (constant integrand)
    R = oracle.R_DEFAULT
    for M in (1, 7, 40):
        assert sp.beta_separated(2, [[0, 0]], [[0, 0]], M)[0] == pytest.approx(8 * math.pi * R * R, rel=1e-14)


@pytest.mark.parametrize("d,N,M", [(2, 6, 9), (2, 8, 23), (3, 4, (4, 6)), (3, 6, (3, 4))])
def test_transform_route_equals_direct_sum_on_the_same_table(d, N, M):
    G = _random_spectrum(d, N, seed=N + 10 * d)
    table = sp.beta_separated_table(d, N, M)
    ref = oracle.galerkin_sums(d, N, G, table, want=("t1",))["t1"]
    got = sp.t1_transform(d, N, G, M)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-12, err


def test_transform_route_constant_datum():
    # G = g0 delta_0: the only surviving term is a = b = n = 0
    for d, N, M in ((2, 6, 11), (3, 4, (3, 5))):
        G = np.zeros((N,) * d, dtype=np.complex128)
        G[(N // 2,) * d] = 0.8 - 0.3j
        got = sp.t1_transform(d, N, G, M)
        ref = np.zeros_like(G)
        ref[(N // 2,) * d] = sp.beta_separated(d, np.zeros((1, d)), np.zeros((1, d)), M)[0] * G[(N // 2,) * d] ** 3
        assert np.max(np.abs(got - ref)) <= 1e-13 * abs(ref[(N // 2,) * d])


def test_transform_route_with_converged_angles_equals_the_direct_operator():
    # 2-D with angles_2d(N): the transform route gives the direct oracle's T1
    d, N = 2, 8
    G = _random_spectrum(d, N, seed=5)
    ref = oracle.galerkin_sums(d, N, G, oracle.beta_table(d, N), want=("t1",))["t1"]
    got = sp.t1_transform(d, N, G, sp.angles_2d(N))
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
