"""Level-set sweeps that move the free boundary between ETD steps (oracle).

Section 4.3 of the paper, Algorithm, Steps 1-2: extend the Stefan velocity
off the interface, advect the level set rho with an HJ-WENO scheme,
reinitialise rho, and extend u to the new unknowns by quadratic
extrapolation in the normal direction (Aslam 2004).  The paper names these
building blocks and gives no parameters; the readings below are used both
here and on the GPU.

All sweeps act on whole box arrays; values beyond the box are the nearest
box value (constant extension).  Jacobi updates throughout (every node
updated from the previous iterate), so the result does not depend on a
visiting order.

* Normals: n = grad rho / max(|grad rho|, 1e-12), central differences.
* Aslam extrapolation: known set K0 = computational points of the current
  domain; u_n = n . grad u (central) where the stencil lies in K0 (set K1),
  u_nn = n . grad u_n where the stencil lies in K1 (set K2).  Then three
  extensions, each ASLAM_ITERS Jacobi iterations of v <- v - dtau (n . grad v
  - src) with first-order upwind differences along n, dtau = h/2, off the
  known set: u_nn (src 0, known K2), u_n (src u_nn, known K1), u (src u_n,
  known K0).  Unknown values start at 0.
* Reach: the extension is used only where the boundary moves by at most
  MAX_FRONT_NODES nodes in a step; a faster front is an error (FrontTooFast).
* Stefan velocity: V = mu |grad u_ext| (central differences) at nodes with
  |rho| < h, then constant extension along S(rho) n with S = sign(rho),
  VEL_ITERS Jacobi iterations, dtau = h/2; nodes farther than the extension
  reach keep V = 0.
* Advection: rho_t + V |grad rho| = 0 (the normal-speed form of
  rho_t + v . grad rho = 0 with v = V n), Godunov Hamiltonian for V >= 0,
  HJ-WENO5 one-sided derivatives (eps = 1e-6), TVD-RK3, substeps
  n_sub = max(1, ceil(max V * dt / (h/2))).
* Reinitialisation: rho_tau + S(rho_0)(|grad rho| - 1) = 0,
  S = rho_0 / sqrt(rho_0^2 + h^2), Godunov, HJ-WENO5, TVD-RK3,
  REINIT_ITERS iterations of dtau = h/2, in the narrow band
  |rho_0| < REINIT_BAND h (every stage keeps the other nodes at rho_0).

Pins (tests/test_oracle_levelset.py): WENO5 derivatives exact for cubics
and fifth-order accurate for smooth data; a circle under constant V grows to
radius R + V t; an exact signed distance is a fixed point of
reinitialisation away from the centre; a distorted level set is restored to
|grad rho| = 1 near the interface with its zero set kept; Aslam extension
reproduces a radial quadratic near the interface to truncation error; the
velocity of u = c (R - r) on a disk is mu c.  The coupled free-boundary
trajectory built from these sweeps is "parity unpinned" beyond those checks
(no trajectory in the paper survives: its figures are not available).
"""
from __future__ import annotations

import math

import numpy as np

ASLAM_ITERS = 25
# Largest front displacement per step, in nodes, that the extrapolation
# serves: with ASLAM_ITERS sweeps per stage the extension has converged to
# within truncation error at every point that joins the domain when the
# boundary moves at most this far (tests/test_oracle_levelset.py); a step
# whose maximum speed would move it farther (max V * dt > MAX_FRONT_NODES h)
# is refused.
MAX_FRONT_NODES = 2
VEL_ITERS = 20
REINIT_ITERS = 10
# Narrow band of the reinitialisation (units of h): only nodes with
# |rho_0| < REINIT_BAND h are updated; the interface region |rho| < 3h then
# agrees with a whole-box reinitialisation to well below 1e-4 h.
REINIT_BAND = 12
WENO_EPS = 1e-6


def _axes(a):
    """numpy axes of spatial axes x, y[, z]."""
    return [a.ndim - 1 - d for d in range(a.ndim)]


def _sh(a, ax, s):
    """b[i] = a[clamp(i + s)] along numpy axis ax."""
    n = a.shape[ax]
    idx = np.clip(np.arange(n) + s, 0, n - 1)
    return np.take(a, idx, axis=ax)


def normals(rho, h):
    g = [(_sh(rho, ax, 1) - _sh(rho, ax, -1)) / (2.0 * h) for ax in _axes(rho)]
    mag = np.sqrt(sum(c * c for c in g))
    mag = np.maximum(mag, 1e-12)
    return [c / mag for c in g]


def _central_dir(v, n, h):
    return sum(nd * (_sh(v, ax, 1) - _sh(v, ax, -1)) / (2.0 * h) for nd, ax in zip(n, _axes(v)))


def _upwind_dir(v, a, h):
    """First-order upwind a . grad v (information travels along +a)."""
    out = np.zeros_like(v)
    for ad, ax in zip(a, _axes(v)):
        out += np.maximum(ad, 0.0) * (v - _sh(v, ax, -1)) + np.minimum(ad, 0.0) * (_sh(v, ax, 1) - v)
    return out / h


def _stencil_known(known):
    k = known.copy()
    for ax in _axes(known):
        k &= _sh(known, ax, 1) & _sh(known, ax, -1)
    return k


def _extend(v, known, n, src, h, iters):
    dtau = 0.5 * h
    for _ in range(iters):
        upd = v - dtau * (_upwind_dir(v, n, h) - src)
        v = np.where(known, v, upd)
    return v


def aslam_extrapolate(u, known, rho, h, iters=ASLAM_ITERS):
    """Quadratic normal extrapolation of u off the known set."""
    n = normals(rho, h)
    u0 = np.where(known, u, 0.0)
    k1 = _stencil_known(known)
    un = np.where(k1, _central_dir(u0, n, h), 0.0)
    k2 = _stencil_known(k1)
    unn = np.where(k2, _central_dir(un, n, h), 0.0)
    unn = _extend(unn, k2, n, 0.0, h, iters)
    un = _extend(un, k1, n, unn, h, iters)
    return _extend(u0, known, n, un, h, iters)


def stefan_velocity(u_ext, rho, h, mu, iters=VEL_ITERS):
    """V = mu |grad u_ext| on |rho| < h, extended constant along normals."""
    g = [(_sh(u_ext, ax, 1) - _sh(u_ext, ax, -1)) / (2.0 * h) for ax in _axes(u_ext)]
    band = np.abs(rho) < h
    V = np.where(band, mu * np.sqrt(sum(c * c for c in g)), 0.0)
    n = normals(rho, h)
    S = np.sign(rho)
    a = [S * nd for nd in n]
    return _extend(V, band, a, 0.0, h, iters)


def _weno5(v1, v2, v3, v4, v5):
    """HJ-WENO5 combination of five divided differences (Jiang & Peng)."""
    p1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0
    p2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0
    p3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0
    s1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) ** 2 + 0.25 * (v1 - 4.0 * v2 + 3.0 * v3) ** 2
    s2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) ** 2 + 0.25 * (v2 - v4) ** 2
    s3 = 13.0 / 12.0 * (v3 - 2.0 * v4 + v5) ** 2 + 0.25 * (3.0 * v3 - 4.0 * v4 + v5) ** 2
    a1 = 0.1 / (s1 + WENO_EPS) ** 2
    a2 = 0.6 / (s2 + WENO_EPS) ** 2
    a3 = 0.3 / (s3 + WENO_EPS) ** 2
    return (a1 * p1 + a2 * p2 + a3 * p3) / (a1 + a2 + a3)


def weno_derivatives(phi, h):
    """[(D-, D+)] per spatial axis, HJ-WENO5, constant extension at the box."""
    out = []
    for ax in _axes(phi):
        d = [(_sh(phi, ax, k + 1) - _sh(phi, ax, k)) / h for k in range(-3, 3)]
        # d[j] = (phi_{i+j-2} - phi_{i+j-3})/h for j = 0..5
        dm = _weno5(d[0], d[1], d[2], d[3], d[4])
        dp = _weno5(d[5], d[4], d[3], d[2], d[1])
        out.append((dm, dp))
    return out


def godunov_grad(phi, h, sign):
    """|grad phi| by the Godunov rule for speed sign `sign` (array of +-1/0)."""
    acc_pos = np.zeros_like(phi)
    acc_neg = np.zeros_like(phi)
    for dm, dp in weno_derivatives(phi, h):
        acc_pos += np.maximum(np.maximum(dm, 0.0) ** 2, np.minimum(dp, 0.0) ** 2)
        acc_neg += np.maximum(np.minimum(dm, 0.0) ** 2, np.maximum(dp, 0.0) ** 2)
    return np.where(sign > 0, np.sqrt(acc_pos), np.where(sign < 0, np.sqrt(acc_neg), 0.0))


def _rk3(phi, L, dt):
    p1 = phi - dt * L(phi)
    p2 = 0.75 * phi + 0.25 * (p1 - dt * L(p1))
    return phi / 3.0 + 2.0 / 3.0 * (p2 - dt * L(p2))


class FrontTooFast(ValueError):
    """The boundary would move beyond the reach of the extrapolation."""


def check_front_reach(V, dt, h):
    """Raise FrontTooFast when max V * dt exceeds MAX_FRONT_NODES * h."""
    vmax = float(np.max(V)) if V.size else 0.0
    if vmax * dt > MAX_FRONT_NODES * h:
        raise FrontTooFast(f"front moves {vmax * dt / h:.2f} nodes in one step (limit {MAX_FRONT_NODES})")


def advect_substeps(V, dt, h) -> int:
    vmax = float(np.max(V)) if V.size else 0.0
    return max(1, int(math.ceil(vmax * dt / (0.5 * h))))


def advect(rho, V, dt, h):
    """rho_t + V |grad rho| = 0 over dt (V >= 0)."""
    nsub = advect_substeps(V, dt, h)
    ds = dt / nsub
    one = np.ones_like(rho)

    def L(phi):
        return V * godunov_grad(phi, h, one)

    for _ in range(nsub):
        rho = _rk3(rho, L, ds)
    return rho


def reinitialize(rho, h, iters=REINIT_ITERS, band=REINIT_BAND):
    """rho_tau + S(rho_0)(|grad rho| - 1) = 0, TVD-RK3 in pseudo-time.

    band (in units of h): the update is applied only at nodes with
    |rho_0| < band h (narrow band); every RK stage keeps the other nodes at
    their rho_0 values, which the WENO stencils of band nodes read.  None:
    the whole box."""
    rho0 = rho
    S = rho0 / np.sqrt(rho0 * rho0 + h * h)
    sgn = np.sign(S)
    if band is None:
        def L(phi):
            return S * (godunov_grad(phi, h, sgn) - 1.0)

        for _ in range(iters):
            rho = _rk3(rho, L, 0.5 * h)
        return rho
    inb = np.abs(rho0) < band * h

    def Lb(phi):
        return np.where(inb, S * (godunov_grad(phi, h, sgn) - 1.0), 0.0)

    dt = 0.5 * h
    for _ in range(iters):
        p1 = np.where(inb, rho - dt * Lb(rho), rho)
        p2 = np.where(inb, 0.75 * rho + 0.25 * (p1 - dt * Lb(p1)), rho)
        rho = np.where(inb, rho / 3.0 + 2.0 / 3.0 * (p2 - dt * Lb(p2)), rho)
    return rho
