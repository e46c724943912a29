"""Exponential time differencing schemes on the semi-discrete system (oracle).

Section 3: after the spatial discretisation, U' = C U + F(U, t) (eq. 3.2);
the variation-of-constants formula (eq. 3.3) is approximated by
interpolating F.  Every scheme is written as phi-combinations, each
evaluated exactly (up to rounding) by ``oracle.phi``:

* ETD1 (Section 3.1): U+ = e^{hC} U + h phi_1(hC) F_n, i.e. the
  combination with b_0 = U, b_1 = h F_n.
* ETD2RK (Section 3.2): a = e^{hC} U + h phi_1(hC) F_n and
  U+ = e^{hC} U + h phi_1(hC) F_n + h phi_2(hC) (F(a, t+h) - F_n), the
  second line evaluated as one combination with b_2 = h (F(a) - F_n).
* ETD2 multistep (Section 3.1) and ETD3RK / ETD4RK (Section 3.2) are also
  given; the phi_3 of those two formulas is the paper's unnormalised one,
  which is 2 phi_3 in the standard normalisation used throughout here.

The reaction term of the free-boundary model (Section 4.3) is logistic,
f(u) = u (a - b u).

Pins (tests/test_oracle_etd.py): with C = 0 ETD1 is forward Euler and
ETD2RK is Heun's method; with F independent of U and polynomial in t of
degree below the order, the schemes are exact; with F = 0 a step is
e^{hC} U; the peanut reaction-diffusion problem of Section 4.2 converges at
second order with errors of the size printed in Table 1.
"""
from __future__ import annotations

import numpy as np

from .phi import phi_combination


def logistic(a: float = 1.0, b: float = 1.0):
    """f(u) = u (a - b u) and its derivative."""
    return (lambda u, t=0.0: u * (a - b * u)), (lambda u, t=0.0: a - 2.0 * b * u)


def etd1_step(A, h, U, F, t=0.0, method="auto"):
    """One ETD1 step for U' = A U + F(U, t)."""
    Fn = F(U, t)
    return phi_combination(A, h, [U, h * Fn], method)


def etd2rk_step(A, h, U, F, t=0.0, method="auto", return_stage=False):
    """One ETD2RK step for U' = A U + F(U, t)."""
    Fn = F(U, t)
    a = phi_combination(A, h, [U, h * Fn], method)
    Fa = F(a, t + h)
    Up = phi_combination(A, h, [U, h * Fn, h * (Fa - Fn)], method)
    return (Up, a) if return_stage else Up


def etd2_step(A, h, U, Fn, Fnm1, method="auto"):
    """One ETD2 multistep step given F_n and F_{n-1}."""
    return phi_combination(A, h, [U, h * Fn, h * (Fn - Fnm1)], method)


def etd3rk_step(A, h, U, F, t=0.0, method="auto"):
    """One ETD3RK step (Section 3.2); unnormalised phi_3 = 2 * standard phi_3."""
    Fn = F(U, t)
    a = phi_combination(A, h / 2, [U, (h / 2) * Fn], method)
    Fa = F(a, t + h / 2)
    b = phi_combination(A, h, [U, h * (2 * Fa - Fn)], method)
    Fb = F(b, t + h)
    return phi_combination(A, h, [U, h * Fn, h * (-3 * Fn + 4 * Fa - Fb),
                                  2.0 * h * (2 * Fn - 4 * Fa + 2 * Fb)], method)


def etd4rk_step(A, h, U, F, t=0.0, method="auto"):
    """One ETD4RK step (Section 3.2); unnormalised phi_3 = 2 * standard phi_3."""
    Fn = F(U, t)
    a = phi_combination(A, h / 2, [U, (h / 2) * Fn], method)
    Fa = F(a, t + h / 2)
    b = phi_combination(A, h / 2, [U, (h / 2) * Fa], method)
    Fb = F(b, t + h / 2)
    c = phi_combination(A, h / 2, [a, (h / 2) * (2 * Fb - Fn)], method)
    Fc = F(c, t + h)
    return phi_combination(A, h, [U, h * Fn, h * (-3 * Fn + 2 * (Fa + Fb) - Fc),
                                  2.0 * h * (2 * Fn - 2 * (Fa + Fb) + 2 * Fc)], method)


def etd_step(A, h, U, F, scheme: str, t=0.0, method="auto"):
    if scheme == "etd1":
        return etd1_step(A, h, U, F, t, method)
    if scheme == "etd2rk":
        return etd2rk_step(A, h, U, F, t, method)
    if scheme == "etd3rk":
        return etd3rk_step(A, h, U, F, t, method)
    if scheme == "etd4rk":
        return etd4rk_step(A, h, U, F, t, method)
    raise ValueError(scheme)
