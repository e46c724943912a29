"""Pins for oracle.multispecies (Section 3, eq. 3.1 with u in R^m)."""
import numpy as np
import pytest

from oracle.etd import etd_step, logistic
from oracle.geometry import Grid
from oracle.multispecies import lotka_volterra, species_step
from oracle.operator import build_operator

SCHEMES = ["etd1", "etd2rk", "etd3rk", "etd4rk"]


def _disk_operator(n=20):
    g = Grid(2, (n, n), (-1.5, -1.5), (1.5, 1.5))
    X, Y = g.coords()
    op = build_operator(g, np.hypot(X, Y) - 1.1, 0.8)
    return op, X, Y


@pytest.mark.parametrize("scheme", SCHEMES)
def test_uncoupled_species_are_independent_runs(scheme):
    op, X, Y = _disk_operator()
    rng = np.random.default_rng(1)
    Us = [rng.uniform(0.1, 0.9, op.n) for _ in range(3)]
    a = [1.0, 0.7, 1.3]
    b = np.diag([1.0, 0.5, 2.0])
    h = 0.05
    got = species_step(op.A, h, Us, a, b, scheme, method="dense")
    for s in range(3):
        f, _ = logistic(a[s], b[s, s])
        ref = etd_step(op.A, h, Us[s], f, scheme, method="dense")
        assert np.linalg.norm(got[s] - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_conservative_coupling_keeps_the_sum_on_the_heat_flow(scheme):
    """f_0 = -k u_0 u_1, f_1 = k u_0 u_1: the sum S = U_0 + U_1 obeys S' = A S
    exactly, and the ETD schemes, linear in F with the same phi-functions for
    both blocks, give S_{n+1} = e^{hA} S_n (eigendecomposition)."""
    op, X, Y = _disk_operator()
    rng = np.random.default_rng(2)
    Us = [rng.uniform(0.1, 0.9, op.n) for _ in range(2)]
    k = 3.0
    a = [0.0, 0.0]
    b = np.array([[0.0, k], [-k, 0.0]])
    h = 0.08
    got = species_step(op.A, h, Us, a, b, scheme, method="dense")
    lam, Q = np.linalg.eigh(op.A.toarray())
    S = Us[0] + Us[1]
    ref = Q @ (np.exp(h * lam) * (Q.T @ S))
    assert np.linalg.norm(got[0] + got[1] - ref) <= 1e-12 * np.linalg.norm(ref)
    # the reaction does move the species (the pin is not vacuous)
    heat = Q @ (np.exp(h * lam) * (Q.T @ Us[0]))
    assert np.linalg.norm(got[0] - heat) > 1e-3 * np.linalg.norm(heat)


def test_zero_operator_is_heun_on_the_coupled_system():
    n = 5
    A = np.zeros((n, n))
    rng = np.random.default_rng(3)
    Us = [rng.uniform(0.1, 0.9, n) for _ in range(2)]
    a = [1.0, 0.6]
    b = np.array([[1.0, 0.4], [0.7, 1.2]])

    def f(u0, u1):
        return u0 * (a[0] - b[0, 0] * u0 - b[0, 1] * u1), u1 * (a[1] - b[1, 0] * u0 - b[1, 1] * u1)

    h = 0.3
    k1 = f(*Us)
    k2 = f(Us[0] + h * k1[0], Us[1] + h * k1[1])
    heun = [Us[s] + 0.5 * h * (k1[s] + k2[s]) for s in range(2)]
    got = species_step(A, h, Us, a, b, "etd2rk", method="dense")
    for s in range(2):
        assert np.allclose(got[s], heun[s], rtol=1e-14, atol=1e-15)


def test_lotka_volterra_single_species_is_logistic():
    U = np.linspace(0.0, 1.0, 11)
    f, _ = logistic(1.3, 0.8)
    assert np.array_equal(lotka_volterra([1.3], [[0.8]])(U), f(U))
