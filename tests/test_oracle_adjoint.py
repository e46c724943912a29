"""Pins for oracle.adjoint (discrete adjoint of ETD2RK, frozen domain).

* f = 0: ETD2RK is e^{hA} per step, so L = |e^{TA} U_0|^2 has the closed
  forms dL/dU_0 = 2 e^{2TA} U_0 and dL/dbeta = 2 T <e^{TA}U_0, A_1 e^{TA}U_0>.
* Logistic f: central finite differences of the forward map in U_0
  (directional) and in beta.
"""
import numpy as np

from oracle import adjoint as adj
from oracle.etd import logistic
from oracle.geometry import Grid
from oracle.operator import build_operator


def _problem(beta):
    g = Grid(2, (22, 22), (-1.5, -1.5), (1.5, 1.5))
    X, Y = g.coords()
    op1 = build_operator(g, np.hypot(X, Y) - 1.0, 1.0)
    rng = np.random.default_rng(0)
    U0 = rng.uniform(0.2, 0.8, op1.n)
    return op1.A, beta * op1.A, U0


def test_adjoint_closed_form_zero_reaction():
    beta, h, steps = 1.3, 0.02, 5
    A1, A, U0 = _problem(beta)
    zero = lambda u, t=0.0: np.zeros_like(u)
    L, gU, gb = adj.gradient(A, beta, h, U0, steps, zero, zero, method="eigh")
    lam, Q = np.linalg.eigh(A.toarray())
    T = h * steps
    eTA = lambda v, s=1.0: Q @ (np.exp(s * T * lam) * (Q.T @ v))
    UT = eTA(U0)
    assert abs(L - UT @ UT) < 1e-12 * L
    assert np.linalg.norm(gU - 2 * eTA(U0, 2.0)) < 1e-11 * np.linalg.norm(gU)
    gb_exact = 2 * T * (UT @ (A1 @ UT))
    assert abs(gb - gb_exact) < 1e-10 * abs(gb_exact)


def test_adjoint_matches_finite_differences_logistic():
    beta, h, steps = 0.8, 0.03, 4
    A1, A, U0 = _problem(beta)
    f, df = logistic(1.0, 1.0)
    L, gU, gb = adj.gradient(A, beta, h, U0, steps, f, df, method="dense")
    rng = np.random.default_rng(1)
    d = rng.standard_normal(U0.shape)
    eps = 1e-6

    def Lof(U, b):
        return adj.loss(adj.forward(b * A1, h, U, steps, f, method="dense")[-1])

    fd = (Lof(U0 + eps * d, beta) - Lof(U0 - eps * d, beta)) / (2 * eps)
    assert abs(fd - gU @ d) < 1e-7 * abs(fd)
    fdb = (Lof(U0, beta + eps) - Lof(U0, beta - eps)) / (2 * eps)
    assert abs(fdb - gb) < 1e-7 * abs(fdb)
