"""Multi-species reaction-diffusion systems (oracle; test infrastructure).

Section 3, eq. 3.1: u in R^m with one diffusion coefficient beta for every
component, u_t = div(beta grad u) + f(u, t).  After the embedded-boundary
discretisation of Section 2 (the same operator A for each component) the
system is U' = C U + F(U) (eq. 3.2) with C = I_m (x) A, block diagonal, and
the stacked unknowns U = [U_0; U_1; ...; U_{m-1}] (species-major).  Every ETD
scheme of Section 3 applies unchanged to the stacked system (oracle.etd
with the block operator); phi_k(hC) acts block by block.

The reaction used here is the Lotka-Volterra family
f_s(u) = u_s (a_s - sum_j b_sj u_j), which for m = 1 is the logistic term of
the free-boundary model of Section 4.3.

Pins (tests/test_oracle_species.py): uncoupled species (b diagonal) equal
independent single-species runs; a conservative coupling (f_0 = -k u_0 u_1,
f_1 = k u_0 u_1) leaves the species sum evolving by e^{hA} alone, for every
scheme; with A = 0 ETD2RK is Heun's method on the coupled ODE system.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .etd import etd_step


def lotka_volterra(a, b):
    """F on the stacked vector: f_s(u) = u_s (a_s - sum_j b_sj u_j)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m = a.shape[0]

    def F(U, t=0.0):
        comps = np.split(U, m)
        out = []
        for s in range(m):
            acc = a[s]
            for j in range(m):
                acc = acc - b[s, j] * comps[j]
            out.append(comps[s] * acc)
        return np.concatenate(out)

    return F


def block_operator(A, m):
    """C = I_m (x) A (scipy sparse)."""
    return sp.block_diag([A] * m, format="csr")


def species_step(A, h, Us, a, b, scheme, method="auto"):
    """One ETD step of the m-species system; Us: list of m unknown vectors."""
    m = len(Us)
    U = etd_step(block_operator(A, m), h, np.concatenate(Us), lotka_volterra(a, b), scheme, method=method)
    return np.split(U, m)
