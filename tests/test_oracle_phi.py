"""Pins for oracle.phi: scalar phi_k and the three combination routes.

What pins what:
* mpmath closed forms at 150 digits pin phi_scalar (both branches).
* phi_k(0) = 1/k! and the recurrence of Section 3 (normalised form) pin the
  normalisation.
* Quadrature of the integral definition (eq. 3.4 with the 1/(k-1)! factor).
* The derivative identity phi_k' = phi_k - k phi_{k+1} by finite differences.
* The combination equals the time-1 solution of the ODE of Section 3.3,
  integrated by an independent high-order ODE solver (scipy DOP853).
* dense, eigh and Krylov routes agree; brute-force power series on a tiny
  matrix.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle.phi import (phi_combination, phi_combination_at, phi_combination_dense, phi_combination_eigh,
                        phi_combination_krylov, phi_scalar)

mpmath.mp.dps = 150


def phi_mp(k, z):
    z = mpmath.mpf(z)
    if z == 0:
        return mpmath.mpf(1) / mpmath.factorial(k)
    s = mpmath.exp(z)
    for j in range(1, k + 1):
        s = (s - mpmath.mpf(1) / mpmath.factorial(j - 1)) / z
    return s


ZS = [-700.0, -50.0, -7.5, -2.0, -1.999, -1.0, -0.999, -0.3, -1e-3, -1e-9, 0.0, 1e-8, 0.25, 0.9999,
      1.0, 1.999, 2.0, 3.0, 20.0]


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_phi_scalar_vs_mpmath(k):
    for z in ZS:
        ref = float(phi_mp(k, z))
        got = phi_scalar(k, z)
        assert abs(got - ref) <= 1e-14 * max(abs(ref), 1e-300), (k, z, got, ref)


def test_phi_closed_forms():
    for z in [-30.0, -2.0, 1.5, 4.0]:
        assert math.isclose(phi_scalar(1, z), (math.exp(z) - 1) / z, rel_tol=1e-14)
        assert math.isclose(phi_scalar(2, z), (math.exp(z) - 1 - z) / z ** 2, rel_tol=1e-13)
        assert math.isclose(phi_scalar(3, z), (math.exp(z) - 1 - z - z * z / 2) / z ** 3, rel_tol=1e-12)


def test_phi_at_zero_and_recurrence():
    for k in range(8):
        assert phi_scalar(k, 0.0) == pytest.approx(1.0 / math.factorial(k), rel=1e-15)
    for z in [-40.0, -3.0, -0.5, 0.7, 2.0]:
        for k in range(1, 6):
            lhs = phi_scalar(k, z)
            rhs = (phi_scalar(k - 1, z) - 1.0 / math.factorial(k - 1)) / z
            assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_phi_integral_definition(k):
    for z in [-20.0, -1.0, -0.1, 0.3, 2.0]:
        val, _ = quad(lambda s: math.exp((1 - s) * z) * s ** (k - 1) / math.factorial(k - 1), 0, 1,
                      epsabs=1e-15, epsrel=1e-14)
        assert phi_scalar(k, z) == pytest.approx(val, rel=1e-12)


def test_phi_derivative_identity():
    eps = 1e-5
    for z in [-10.0, -1.3, 0.4, 1.7]:
        for k in range(0, 4):
            fd = (phi_scalar(k, z + eps) - phi_scalar(k, z - eps)) / (2 * eps)
            ident = phi_scalar(k, z) - k * phi_scalar(k + 1, z)
            assert fd == pytest.approx(ident, rel=1e-8, abs=1e-10)


def _spd(n, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    return -(B @ B.T) / n * scale


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_combination_equals_ode_solution(p):
    """Section 3.3: y(1) of y' = A y + sum_k t^{k-1}/(k-1)! v_k, y(0) = v_0."""
    n = 12
    A = _spd(n, 1)
    rng = np.random.default_rng(2)
    vs = [rng.standard_normal(n) for _ in range(p + 1)]

    def rhs(t, y):
        out = A @ y
        for k in range(1, p + 1):
            out = out + t ** (k - 1) / math.factorial(k - 1) * vs[k]
        return out

    sol = solve_ivp(rhs, (0.0, 1.0), vs[0], method="DOP853", rtol=1e-13, atol=1e-14)
    ref = sol.y[:, -1]
    got = phi_combination_dense(A, 1.0, vs)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_three_routes_agree(p):
    n = 40
    A = _spd(n, 3, scale=20.0)
    rng = np.random.default_rng(4)
    bs = [rng.standard_normal(n) for _ in range(p + 1)]
    for t in [0.05, 1.0]:
        d = phi_combination_dense(A, t, bs)
        e = phi_combination_eigh(A, t, bs)
        k = phi_combination_krylov(A, t, bs, m=12)
        nrm = np.linalg.norm(e)
        assert np.linalg.norm(d - e) <= 1e-13 * nrm
        assert np.linalg.norm(k - e) <= 1e-12 * nrm


def test_power_series_brute_force():
    n = 5
    A = _spd(n, 5, scale=0.5)
    rng = np.random.default_rng(6)
    bs = [rng.standard_normal(n) for _ in range(4)]
    ref = np.zeros(n)
    for k, b in enumerate(bs):
        term = b.copy()
        acc = np.zeros(n)
        for j in range(60):
            acc += term / math.factorial(j + k)
            term = A @ term
        ref += acc
    got = phi_combination_dense(A, 1.0, bs)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


def test_dispatch_empty_and_zero():
    A = _spd(6, 7)
    z = np.zeros(6)
    assert np.all(phi_combination(A, 0.3, [z, z]) == 0.0)
    b0 = np.arange(6.0)
    # t = 0: every phi_k(0 A) is 1/k! I
    got = phi_combination(A, 0.0, [b0, b0, b0])
    assert np.allclose(got, b0 * (1 + 1 + 0.5), rtol=1e-15)


@pytest.mark.parametrize("p", [0, 1, 3])
def test_intermediate_time_is_the_ode_solution(p):
    """phi_combination_at: the ODE of Section 3.3 (its forcing scaled to end
    at t) integrated by DOP853 to an intermediate time s."""
    n = 25
    rng = np.random.default_rng(9)
    B = rng.standard_normal((n, n))
    A = -(B @ B.T) / n * 8.0
    bs = [rng.standard_normal(n) for _ in range(p + 1)]
    t, s = 0.9, 0.37

    def rhs(tau, y):
        out = A @ y
        for k in range(1, p + 1):
            out = out + tau ** (k - 1) / math.factorial(k - 1) * bs[k] / t ** k
        return out

    sol = solve_ivp(rhs, (0.0, s), bs[0], method="DOP853", rtol=1e-13, atol=1e-14)
    got = phi_combination_at(A, t, bs, s, method="dense")
    assert np.linalg.norm(got - sol.y[:, -1]) <= 1e-10 * np.linalg.norm(sol.y[:, -1])
    # at s = t it is the combination itself
    assert np.allclose(phi_combination_at(A, t, bs, t, method="dense"), phi_combination(A, t, bs, method="dense"),
                       rtol=1e-14, atol=1e-14)
