"""One step of the free-boundary algorithm (oracle).

Section 4.3, Algorithm: Step 1 extends the Stefan velocity and moves the
level set (HJ-WENO advection, then reinitialisation); Step 2 extends u to
the unknowns of the new domain by quadratic normal extrapolation and takes
an ETD step on the new domain.  Order used here and on the GPU: the
velocity comes from u^m on the old domain, then rho is advected over the
step, reinitialised when asked, u is extended from the old computational
points and restricted to the new ones, and the ETD step runs with the
operator of the new domain.  A frozen domain (mu = 0) skips Step 1.

A step whose maximum Stefan speed would move the boundary more than
MAX_FRONT_NODES nodes raises FrontTooFast before rho or u change.

Parity: "parity unpinned" as a coupled trajectory beyond the invariants of
its parts (see oracle.levelset and oracle.etd); the extension of
F(U_{n-1}) to the points that join the domain is pinned by the
truncation-order bound of tests/test_oracle_levelset.py.
"""
from __future__ import annotations

import numpy as np

from . import levelset as ls
from .etd import etd2_step, etd2rk_step, etd_step, logistic
from .geometry import Grid, classify
from .operator import build_operator


def levelset_advance(grid: Grid, rho, u_box, dt, mu, reinit: bool):
    """Steps 1 and 2a.  Returns (rho_new, u_new_box, info)."""
    h = grid.dx
    _, comp_old, _ = classify(grid, rho)
    u_ext = ls.aslam_extrapolate(u_box, comp_old, rho, h)
    V = ls.stefan_velocity(u_ext, rho, h, mu)
    ls.check_front_reach(V, dt, h)
    nsub = ls.advect_substeps(V, dt, h)
    rho_new = ls.advect(rho, V, dt, h)
    if reinit:
        rho_new = ls.reinitialize(rho_new, h)
    _, comp_new, _ = classify(grid, rho_new)
    u_new = np.where(comp_new, u_ext, 0.0)
    return rho_new, u_new, {"V": V, "nsub": nsub, "u_ext": u_ext}


def free_boundary_step(grid: Grid, rho, u_box, h, beta=1.0, mu=1.0, a=1.0, b=1.0,
                       scheme="etd2rk", reinit=False, frozen=False, method="auto"):
    """One full step; returns (rho_new, u_new_box, operator)."""
    if frozen:
        rho_new = rho
        u_new = u_box
    else:
        rho_new, u_new, _ = levelset_advance(grid, rho, u_box, h, mu, reinit)
    op = build_operator(grid, rho_new, beta)
    f, _ = logistic(a, b)
    U = op.gather(u_new)
    U = etd_step(op.A, h, U, f, scheme, method=method)
    return rho_new, op.scatter(U), op


def multistep_step(grid: Grid, rho, u_box, f_prev_box, h, beta=1.0, mu=1.0, a=1.0, b=1.0, first=False,
                   reinit=False, frozen=False, method="auto"):
    """One step with ETD2 multistep (Section 3.1) in the Section 4.3 algorithm.

    f_prev_box holds F(U_{n-1}) on the computational points of the current
    domain (not read when first).  On a moving domain it is carried to the
    new computational points by the quadratic normal extrapolation from the
    old computational points that carries u (Step 2), with the same sweeps.
    The first step is
    one ETD2RK step.  Returns (rho_new, u_new_box, f_new_box, op), f_new_box
    = F(U_n) on the new computational points and 0 elsewhere."""
    if frozen:
        rho_new, u_new, f_ext = rho, u_box, f_prev_box
    else:
        f_ext = None
        if not first:
            _, comp_old, _ = classify(grid, rho)
            f_ext = ls.aslam_extrapolate(f_prev_box, comp_old, rho, grid.dx)
        rho_new, u_new, _ = levelset_advance(grid, rho, u_box, h, mu, reinit)
    op = build_operator(grid, rho_new, beta)
    f, _ = logistic(a, b)
    U = op.gather(u_new)
    Fn = f(U)
    if first:
        U = etd2rk_step(op.A, h, U, f, method=method)
    else:
        U = etd2_step(op.A, h, U, Fn, op.gather(f_ext), method=method)
    return rho_new, op.scatter(U), op.scatter(Fn), op


def run(workload_grid: Grid, rho0, u0, steps, h, beta, mu, scheme, reinit_every=5,
        frozen=False, method="auto", callback=None):
    """Run `steps` free-boundary steps; reinit on steps whose 1-based index
    is a multiple of reinit_every."""
    rho, u = rho0, u0
    for m in range(steps):
        rho, u, op = free_boundary_step(workload_grid, rho, u, h, beta, mu, scheme=scheme,
                                        reinit=((m + 1) % reinit_every == 0) if reinit_every else False,
                                        frozen=frozen, method=method)
        if callback is not None:
            callback(m, rho, u, op)
    return rho, u
