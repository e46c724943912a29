"""Pins for oracle.etd (Section 3 of the paper).

* C = 0: ETD1 is forward Euler, ETD2RK is Heun's method, ETD3RK is Kutta's
  third-order method and ETD4RK the classical fourth-order Runge-Kutta
  method (closed forms; F depends on U, so every stage value is tested).
* Diagonal C: ETD3RK and ETD4RK equal the ETDRK3 / ETDRK4 schemes of Cox and
  Matthews (J. Comput. Phys. 176, 2002) written in their own form, with the
  coefficients as explicit functions of hc per eigenvalue c.
* F = 0: one step is e^{hC} U (eigendecomposition route).
* F independent of U and polynomial in t: ETD1 exact for constant F, ETD2RK
  exact for linear F, ETD3RK / ETD4RK exact for quadratic F (exact solution
  by the eigendecomposition of C and exact integrals).
* ETD2 multistep (Section 3.1): eq. 3.6 with s = 2 evaluated by quadrature
  of its g_m integrals; C = 0 gives the two-step Adams-Bashforth method; exact for F independent of U and linear in t; order 2 on the
  logistic problem when started with one ETD2RK step.
* Logistic reaction: step-halving shows order 1 (ETD1) and 2 (ETD2RK) on the
  embedded-boundary operator, and orders 3 (ETD3RK) and 4 (ETD4RK) on a
  non-stiff symmetric operator (on the stiff embedded-boundary operator the
  higher-order schemes show the order reduction known for stiff problems).
* Section 4.2.1 peanut problem: second-order convergence and errors of the
  size printed in Table 1 (tests/golden/table1_etd2rk.json).
"""
import json
import math
import os

import numpy as np
import pytest
import sympy

from oracle.etd import etd1_step, etd2_step, etd2rk_step, etd3rk_step, etd4rk_step, logistic
from oracle.geometry import Grid
from oracle.operator import build_operator
from oracle.phi import phi_combination, phi_scalar
from paper_2209_15095_amd.inputs import peanut_level_set

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_etd2rk.json")


def _spd(n, seed, scale=5.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    return -(B @ B.T) / n * scale


def test_zero_operator_reduces_to_euler_and_heun():
    n = 7
    A = np.zeros((n, n))
    rng = np.random.default_rng(0)
    U = rng.uniform(0.1, 0.9, n)
    f, _ = logistic(1.0, 1.0)
    h = 0.3
    assert np.allclose(etd1_step(A, h, U, f), U + h * f(U), rtol=1e-14, atol=1e-15)
    heun = U + 0.5 * h * (f(U) + f(U + h * f(U)))
    assert np.allclose(etd2rk_step(A, h, U, f), heun, rtol=1e-14, atol=1e-15)


def test_zero_operator_reduces_to_kutta_rk3_and_classical_rk4():
    """C = 0 and U-dependent F: ETD3RK is Kutta's third-order method and
    ETD4RK the classical fourth-order Runge-Kutta method."""
    n = 9
    A = np.zeros((n, n))
    rng = np.random.default_rng(11)
    U = rng.uniform(0.1, 0.9, n)
    f, _ = logistic(1.3, 0.7)
    h = 0.35
    k1 = f(U)
    k2 = f(U + 0.5 * h * k1)
    k3 = f(U + h * (2.0 * k2 - k1))
    kutta = U + h * (k1 + 4.0 * k2 + k3) / 6.0
    assert np.allclose(etd3rk_step(A, h, U, f), kutta, rtol=1e-14, atol=1e-15)
    k3 = f(U + 0.5 * h * k2)
    k4 = f(U + h * k3)
    rk4 = U + h * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0
    assert np.allclose(etd4rk_step(A, h, U, f), rk4, rtol=1e-14, atol=1e-15)


def test_higher_order_match_cox_matthews_on_diagonal_operator():
    """Diagonal C = diag(c), logistic F: the ETDRK3 and ETDRK4 formulas of
    Cox and Matthews (2002) per component, coefficients in closed form in
    z = hc (no phi-function routine involved)."""
    rng = np.random.default_rng(5)
    n = 12
    c = -rng.uniform(0.5, 6.0, n)
    A = np.diag(c)
    U = rng.uniform(0.1, 0.9, n)
    f, _ = logistic(1.0, 1.0)
    h = 0.4
    z = h * c
    E, E2 = np.exp(z), np.exp(0.5 * z)
    q1 = (-4.0 - z + E * (4.0 - 3.0 * z + z * z)) / (h * h * c ** 3)
    q2 = (2.0 + z + E * (-2.0 + z)) / (h * h * c ** 3)
    q3 = (-4.0 - 3.0 * z - z * z + E * (4.0 - z)) / (h * h * c ** 3)
    a = E2 * U + (E2 - 1.0) * f(U) / c
    b3 = E * U + (E - 1.0) * (2.0 * f(a) - f(U)) / c
    cm3 = E * U + q1 * f(U) + 4.0 * q2 * f(a) + q3 * f(b3)
    b4 = E2 * U + (E2 - 1.0) * f(a) / c
    c4 = E2 * a + (E2 - 1.0) * (2.0 * f(b4) - f(U)) / c
    cm4 = E * U + q1 * f(U) + 2.0 * q2 * (f(a) + f(b4)) + q3 * f(c4)
    for method in ("dense", "eigh"):
        assert np.abs(etd3rk_step(A, h, U, f, method=method) - cm3).max() < 1e-12 * np.abs(cm3).max()
        assert np.abs(etd4rk_step(A, h, U, f, method=method) - cm4).max() < 1e-12 * np.abs(cm4).max()


def test_zero_reaction_is_exponential():
    A = _spd(20, 1)
    U = np.random.default_rng(1).standard_normal(20)
    lam, Q = np.linalg.eigh(A)
    h = 0.37
    exact = Q @ (np.exp(h * lam) * (Q.T @ U))
    zero = lambda u, t=0.0: np.zeros_like(u)
    for step in (etd1_step, etd2rk_step, etd3rk_step, etd4rk_step):
        assert np.linalg.norm(step(A, h, U, zero) - exact) < 1e-13 * np.linalg.norm(exact)


def _exact_poly_forcing(A, h, U, cs, t0):
    """Exact U(t0+h) for U' = A U + sum_j cs[j] t^j (t absolute)."""
    lam, Q = np.linalg.eigh(A)
    # rewrite sum_j c_j (t0 + s)^j = sum_k d_k s^k, then
    # U(h) = e^{hA}U + sum_k k! h^{k+1} phi_{k+1}(hA) d_k
    deg = len(cs) - 1
    d = [np.zeros_like(U) for _ in range(deg + 1)]
    for j, c in enumerate(cs):
        for k in range(j + 1):
            d[k] = d[k] + math.comb(j, k) * t0 ** (j - k) * c
    out = Q @ (np.exp(h * lam) * (Q.T @ U))
    for k in range(deg + 1):
        out += math.factorial(k) * h ** (k + 1) * (Q @ (phi_scalar(k + 1, h * lam) * (Q.T @ d[k])))
    return out


@pytest.mark.parametrize("step,deg", [(etd1_step, 0), (etd2rk_step, 1), (etd3rk_step, 2), (etd4rk_step, 2)])
def test_exact_for_polynomial_forcing(step, deg):
    n = 15
    A = _spd(n, 2)
    rng = np.random.default_rng(3)
    U = rng.standard_normal(n)
    cs = [rng.standard_normal(n) for _ in range(deg + 1)]
    t0, h = 0.4, 0.25
    F = lambda u, t: sum(c * t ** j for j, c in enumerate(cs))
    got = step(A, h, U, F, t0)
    ref = _exact_poly_forcing(A, h, U, cs, t0)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_logistic_temporal_orders():
    g = Grid(2, (24, 24), (-1.5, -1.5), (1.5, 1.5))
    X, Y = g.coords()
    op = build_operator(g, np.hypot(X, Y) - 1.0, 1.0)
    f, _ = logistic(1.0, 1.0)
    U0 = op.gather(0.5 + 0.3 * np.cos(X) * np.sin(2 * Y))
    T = 0.4

    def run(step, nsteps):
        U = U0.copy()
        for _ in range(nsteps):
            U = step(op.A, T / nsteps, U, f)
        return U

    for step, order in [(etd1_step, 1.0), (etd2rk_step, 2.0)]:
        ref = run(step, 64)
        e1 = np.linalg.norm(run(step, 4) - ref)
        e2 = np.linalg.norm(run(step, 8) - ref)
        assert abs(np.log2(e1 / e2) - order) < 0.25


def test_higher_order_temporal_orders():
    """Step halving on U' = C U + u(1 - u), C symmetric negative definite of
    moderate norm: orders 3 (ETD3RK) and 4 (ETD4RK)."""
    rng = np.random.default_rng(7)
    n = 10
    B = rng.standard_normal((n, n))
    A = -(B @ B.T) / n * 2.0
    f, _ = logistic(1.0, 1.0)
    U0 = rng.uniform(0.2, 0.8, n)
    T = 1.0

    def run(step, nsteps):
        U = U0.copy()
        for _ in range(nsteps):
            U = step(A, T / nsteps, U, f, method="dense")
        return U

    for step, order in [(etd2rk_step, 2.0), (etd3rk_step, 3.0), (etd4rk_step, 4.0)]:
        ref = run(step, 256)
        e1 = np.linalg.norm(run(step, 8) - ref)
        e2 = np.linalg.norm(run(step, 16) - ref)
        assert abs(np.log2(e1 / e2) - order) < 0.3, (step.__name__, np.log2(e1 / e2))


def test_etd2_multistep_zero_operator_is_adams_bashforth():
    n = 6
    A = np.zeros((n, n))
    rng = np.random.default_rng(4)
    U, Fn, Fm = (rng.standard_normal(n) for _ in range(3))
    h = 0.2
    ab2 = U + h * (1.5 * Fn - 0.5 * Fm)
    assert np.allclose(etd2_step(A, h, U, Fn, Fm), ab2, rtol=1e-14, atol=1e-15)


def test_etd2_multistep_is_eq_3_6_with_two_evaluations():
    """Eq. 3.6 with s = 2 evaluated as printed: U e^{hC} + h (g_0 F_n +
    g_1 (F_n - F_{n-1})), g_m = (-1)^m int_0^1 e^{(1-l)hC} binom(-l, m) dl,
    the integrals by 40-point Gauss-Legendre over the eigenvalues of C."""
    n = 12
    A = _spd(n, 7)
    rng = np.random.default_rng(8)
    U, Fn, Fm = (rng.standard_normal(n) for _ in range(3))
    h = 0.3
    lam, Q = np.linalg.eigh(A)
    x, wq = np.polynomial.legendre.leggauss(40)
    l = 0.5 * (x + 1.0)
    wq = 0.5 * wq
    E = np.exp(np.outer(1.0 - l, h * lam))            # e^{(1-l) h lam}, quadrature node by eigenvalue
    binom = [np.ones_like(l), -l]                       # binom(-l, 0), binom(-l, 1)
    g = [(-1) ** m * (wq * binom[m]) @ E for m in range(2)]
    diffs = [Fn, Fn - Fm]                               # sum_k (-1)^k binom(m, k) F_{n-k}
    ref = Q @ (np.exp(h * lam) * (Q.T @ U))
    for m in range(2):
        ref = ref + h * (Q @ (g[m] * (Q.T @ diffs[m])))
    got = etd2_step(A, h, U, Fn, Fm)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_etd2_multistep_exact_for_linear_forcing():
    n = 15
    A = _spd(n, 5)
    rng = np.random.default_rng(6)
    U = rng.standard_normal(n)
    cs = [rng.standard_normal(n) for _ in range(2)]
    t0, h = 0.4, 0.25
    F = lambda t: cs[0] + cs[1] * t
    got = etd2_step(A, h, U, F(t0), F(t0 - h))
    ref = _exact_poly_forcing(A, h, U, cs, t0)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)
    # a quadratic term is not integrated exactly (the scheme interpolates F
    # linearly through t0 - h and t0)
    cq = cs + [rng.standard_normal(n)]
    Fq = lambda t: cq[0] + cq[1] * t + cq[2] * t * t
    got = etd2_step(A, h, U, Fq(t0), Fq(t0 - h))
    assert np.linalg.norm(got - _exact_poly_forcing(A, h, U, cq, t0)) > 1e-6


def test_etd2_multistep_second_order():
    g = Grid(2, (24, 24), (-1.5, -1.5), (1.5, 1.5))
    X, Y = g.coords()
    op = build_operator(g, np.hypot(X, Y) - 1.0, 1.0)
    f, _ = logistic(1.0, 1.0)
    U0 = op.gather(0.5 + 0.3 * np.cos(X) * np.sin(2 * Y))
    T = 0.4

    def run(nsteps):
        h = T / nsteps
        U = etd2rk_step(op.A, h, U0, f)
        Fm = f(U0)
        for _ in range(nsteps - 1):
            Fn = f(U)
            U, Fm = etd2_step(op.A, h, U, Fn, Fm), Fn
        return U

    ref = run(512)
    e1 = np.linalg.norm(run(4) - ref)
    e2 = np.linalg.norm(run(8) - ref)
    assert abs(np.log2(e1 / e2) - 2.0) < 0.25


def _peanut_forcing():
    x, y, t = sympy.symbols("x y t")
    u = sympy.exp(-t) * (x ** 2 + y ** 2 - sympy.Rational(1, 4))
    beta = sympy.Rational(1, 4) - x ** 2 - y ** 2
    f = sympy.diff(u, t) - (sympy.diff(beta * sympy.diff(u, x), x) + sympy.diff(beta * sympy.diff(u, y), y))
    # the source term derived by hand: exp(-t)(7 r^2 - 3/4)
    assert sympy.simplify(f - sympy.exp(-t) * (7 * (x ** 2 + y ** 2) - sympy.Rational(3, 4))) == 0
    return (sympy.lambdify((x, y, t), u, "numpy"), sympy.lambdify((x, y, t), f, "numpy"))


def _peanut_errors(nodes, steps):
    uf, ff = _peanut_forcing()
    g = Grid(2, (nodes, nodes), (-1.0, -1.0), (1.0, 1.0))
    X, Y = g.coords()
    op = build_operator(g, peanut_level_set(X, Y), lambda P: 0.25 - P[:, 0] ** 2 - P[:, 1] ** 2)
    Xc, Yc = op.gather(X), op.gather(Y)
    T = 0.1
    h = T / steps
    method = "dense" if op.n < 1500 else "krylov"

    def F(u, t):
        return ff(Xc, Yc, t) + op.forcing(lambda P: uf(P[0], P[1], t))

    U = uf(Xc, Yc, 0.0)
    t = 0.0
    for _ in range(steps):
        U = etd2rk_step(op.A, h, U, F, t, method=method)
        t += h
    e = U - uf(Xc, Yc, T)
    return np.abs(e).max(), np.sqrt(np.mean(e * e))


def test_peanut_table1_etd2rk():
    """Section 4.2.1, Table 1 (ETD2RK): same problem, dt = h, t = 0.1."""
    rows = json.load(open(GOLDEN))["rows"]
    got = [_peanut_errors(r["nodes"], r["steps"]) for r in rows[:3]]
    for r, (linf, l2) in zip(rows[:3], got):
        assert r["linf"] / 3.0 < linf < r["linf"] * 3.0, (r, linf)
        assert r["l2"] / 4.0 < l2 < r["l2"] * 4.0, (r, l2)
    order = np.log2(got[0][0] / got[2][0]) / 2.0
    assert order > 1.5
