"""Seeded synthetic workloads: grids, initial level sets and initial data.

This module generates inputs only; it holds none of the method's arithmetic
(no operator, no phi-function, no level-set PDE).  Both the CPU oracle and
the GPU path take their inputs from here, so initial data are never a source
of disagreement between them.  Everything is numpy float64 in box layout
((ny, nx) or (nz, ny, nx), x fastest).

Initial level sets are exact signed distances (negative inside): closed
forms for disks and spheres, dense curve sampling plus Newton refinement
for star-shaped curves, and the robust 2D ellipse distance in the meridian
plane for the prolate spheroid.  Random draws use numpy's default_rng with
the seed stated per workload.

Workloads (sizes as in the paper's setting of Section 4.3 and the
benchmark configurations):
  fisher64    2D 64^2 on [-8,8]^2, disk r=2, u0 = cos(pi r/4) inside, ETD1,
              h=0.01, 10 steps, beta=1, mu=1
  star512     2D 512^2 on [-16,16]^2, star r = 3 + 0.5 cos(5 theta),
              u0 = 0.5 inside, ETD2RK, h=0.005, 200 steps, beta=1, mu=2
  ellipsoid192  3D 192^3 on [-10,10]^3, spheroid semi-axes (3,2,2),
              u0 ~ U[0.2,0.8] (seed 0) inside, ETD2RK, h=0.01, 50 steps
  batch64     64 random 2D star domains (seed 0), sides in [96,384]
  sphere96    3D 96^3 on [-5,5]^3, frozen sphere r=4, u0 ~ U[0.2,0.8]
              (seed 0), ETD2RK, h=0.01, 40 steps (adjoint workload)
  disk4097    2D 4097^2 on [-16,16]^2, frozen disk r=15 (bandwidth scale)
  sphere385   3D 385^3 on [-10,10]^3, frozen sphere r=9.5 (bandwidth scale)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class GridSpec:
    dim: int
    n: tuple            # nodes per axis (x, y[, z])
    lo: tuple
    hi: tuple

    @property
    def dx(self) -> float:
        return (self.hi[0] - self.lo[0]) / (self.n[0] - 1)

    @property
    def shape(self) -> tuple:
        return tuple(reversed(self.n[: self.dim]))

    def coords(self):
        axes = [self.lo[d] + self.dx * np.arange(self.n[d]) for d in range(self.dim)]
        mesh = np.meshgrid(*reversed(axes), indexing="ij")
        return tuple(reversed(mesh))


@dataclass
class Workload:
    name: str
    grid: GridSpec
    rho0: np.ndarray
    u0: np.ndarray
    beta: float = 1.0
    mu: float = 1.0
    a: float = 1.0
    b: float = 1.0
    scheme: str = "etd2rk"
    h: float = 0.01
    steps: int = 10
    reinit_every: int = 5
    frozen: bool = False
    extra: dict = field(default_factory=dict)


# ---------------------------------------------------------------- distances

def sdf_disk(X, Y, r, cx=0.0, cy=0.0):
    return np.hypot(X - cx, Y - cy) - r


def sdf_sphere(X, Y, Z, r):
    return np.sqrt(X * X + Y * Y + Z * Z) - r


def sdf_star(X, Y, radius_fn, samples: int = 8192, newton: int = 8):
    """Signed distance to the polar curve r = radius_fn(theta) (star-shaped
    about the origin): nearest of `samples` curve points, then Newton on the
    curve parameter; negative inside."""
    from scipy.spatial import cKDTree

    th = np.linspace(0.0, 2.0 * np.pi, samples, endpoint=False)

    def curve(t):
        r = radius_fn(t)
        return r * np.cos(t), r * np.sin(t)

    def dcurve(t, eps=1e-6):
        x1, y1 = curve(t + eps)
        x0, y0 = curve(t - eps)
        return (x1 - x0) / (2 * eps), (y1 - y0) / (2 * eps)

    def ddcurve(t, eps=1e-4):
        x1, y1 = curve(t + eps)
        x0, y0 = curve(t)
        xm, ym = curve(t - eps)
        return (x1 - 2 * x0 + xm) / eps ** 2, (y1 - 2 * y0 + ym) / eps ** 2

    cx, cy = curve(th)
    tree = cKDTree(np.stack([cx, cy], axis=1))
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    _, k = tree.query(P)
    t = th[k]
    for _ in range(newton):
        x, y = curve(t)
        dx_, dy_ = dcurve(t)
        ddx, ddy = ddcurve(t)
        ex, ey = x - P[:, 0], y - P[:, 1]
        g = ex * dx_ + ey * dy_
        H = dx_ * dx_ + dy_ * dy_ + ex * ddx + ey * ddy
        step = np.where(H > 1e-12, g / np.where(H > 1e-12, H, 1.0), 0.0)
        step = np.clip(step, -0.05, 0.05)
        t = t - step
    x, y = curve(t)
    dist = np.hypot(x - P[:, 0], y - P[:, 1])
    ang = np.arctan2(P[:, 1], P[:, 0])
    rad = np.hypot(P[:, 0], P[:, 1])
    sign = np.where(rad < radius_fn(ang), -1.0, 1.0)
    return (sign * dist).reshape(X.shape)


def sdf_param_curve(X, Y, cx_fn, cy_fn, samples: int = 8192, newton: int = 8):
    """Signed distance to a closed parametric curve (cx_fn(t), cy_fn(t)),
    t in [0, 2 pi): nearest sample, Newton on t, sign by even-odd ray
    crossing of the sampled polygon; negative inside."""
    from scipy.spatial import cKDTree

    th = np.linspace(0.0, 2.0 * np.pi, samples, endpoint=False)
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    cx, cy = cx_fn(th), cy_fn(th)
    tree = cKDTree(np.stack([cx, cy], axis=1))
    _, k = tree.query(P)
    t = th[k]
    e1, e2 = 1e-6, 1e-4
    for _ in range(newton):
        x, y = cx_fn(t), cy_fn(t)
        dx_ = (cx_fn(t + e1) - cx_fn(t - e1)) / (2 * e1)
        dy_ = (cy_fn(t + e1) - cy_fn(t - e1)) / (2 * e1)
        ddx = (cx_fn(t + e2) - 2 * x + cx_fn(t - e2)) / e2 ** 2
        ddy = (cy_fn(t + e2) - 2 * y + cy_fn(t - e2)) / e2 ** 2
        ex, ey = x - P[:, 0], y - P[:, 1]
        g = ex * dx_ + ey * dy_
        H = dx_ * dx_ + dy_ * dy_ + ex * ddx + ey * ddy
        step = np.where(H > 1e-12, g / np.where(H > 1e-12, H, 1.0), 0.0)
        t = t - np.clip(step, -0.05, 0.05)
    dist = np.hypot(cx_fn(t) - P[:, 0], cy_fn(t) - P[:, 1])
    inside = np.zeros(P.shape[0], dtype=bool)
    x1, y1 = cx, cy
    x2, y2 = np.roll(cx, -1), np.roll(cy, -1)
    for c0 in range(0, samples, 512):
        sl = slice(c0, c0 + 512)
        a1, b1, a2, b2 = x1[sl][None, :], y1[sl][None, :], x2[sl][None, :], y2[sl][None, :]
        py = P[:, 1:2]
        px = P[:, 0:1]
        cond = (b1 > py) != (b2 > py)
        xint = (a2 - a1) * (py - b1) / np.where(b2 != b1, b2 - b1, 1.0) + a1
        inside ^= (np.count_nonzero(cond & (px < xint), axis=1) % 2).astype(bool)
    return np.where(inside, -dist, dist).reshape(X.shape)


def virus_level_set(X, Y):
    """Section 4.1 geometry: x = (0.6 + 0.1 sin 12t) cos t,
    y = (0.6 + 0.05 sin 12t) sin t."""
    return sdf_param_curve(X, Y, lambda t: (0.6 + 0.1 * np.sin(12 * t)) * np.cos(t),
                           lambda t: (0.6 + 0.05 * np.sin(12 * t)) * np.sin(t))


def peanut_level_set(X, Y):
    """Section 4.2 geometry (not a signed distance; used as given)."""
    return 0.5 - np.exp(-20 * (X ** 2 + (Y - 0.25) ** 2)) - np.exp(-20 * (X ** 2 + (Y + 0.25) ** 2))


def _ellipse_distance_first_quadrant(e0, e1, y0, y1, iters=64):
    """Distance from (y0, y1) (both >= 0) to the ellipse x^2/e0^2 + y^2/e1^2
    = 1 with e0 >= e1 > 0 (Eberly, 'Distance from a point to an ellipse'),
    vectorised; bisection on the Lagrange parameter."""
    y0 = np.asarray(y0, dtype=np.float64)
    y1 = np.asarray(y1, dtype=np.float64)
    out = np.empty_like(y0)
    pos1 = y1 > 0
    # generic case y1 > 0
    z0 = y0[pos1] / e0
    z1 = y1[pos1] / e1
    g = z0 * z0 + z1 * z1 - 1.0
    r0 = (e0 / e1) ** 2
    n0 = r0 * z0
    s0 = z1 - 1.0
    s1 = np.where(g < 0, 0.0, np.sqrt(n0 * n0 + z1 * z1) - 1.0)
    for _ in range(iters):
        s = 0.5 * (s0 + s1)
        ratio0 = n0 / (s + r0)
        ratio1 = z1 / (s + 1.0)
        gs = ratio0 * ratio0 + ratio1 * ratio1 - 1.0
        s0 = np.where(gs < 0, s0, s)
        s1 = np.where(gs < 0, s, s1)
    s = 0.5 * (s0 + s1)
    x0 = r0 * y0[pos1] / (s + r0)
    x1 = y1[pos1] / (s + 1.0)
    out[pos1] = np.hypot(x0 - y0[pos1], x1 - y1[pos1])
    # y1 == 0: point on the major axis
    zero = ~pos1
    yy = y0[zero]
    numer = e0 * yy
    denom = e0 * e0 - e1 * e1
    inner = numer < denom
    xr = np.where(inner, e0 * numer / np.where(inner, denom, 1.0), e0)
    x1r = np.where(inner, e1 * np.sqrt(np.clip(1.0 - (xr / e0) ** 2, 0.0, None)), 0.0)
    out[zero] = np.hypot(xr - yy, x1r)
    return out


def sdf_prolate_spheroid(X, Y, Z, a, b):
    """Signed distance to x^2/a^2 + (y^2+z^2)/b^2 = 1 with a >= b (axis x)."""
    rr = np.sqrt(Y * Y + Z * Z)
    d = _ellipse_distance_first_quadrant(a, b, np.abs(X).ravel(), rr.ravel()).reshape(X.shape)
    inside = (X / a) ** 2 + (rr / b) ** 2 < 1.0
    return np.where(inside, -d, d)


# ---------------------------------------------------------------- workloads

def _uniform_inside(rho, seed, lo=0.2, hi=0.8):
    rng = np.random.default_rng(seed)
    u = rng.uniform(lo, hi, size=rho.shape)
    return np.where(rho < 0, u, 0.0)


def fisher64(n: int = 64) -> Workload:
    g = GridSpec(2, (n, n), (-8.0, -8.0), (8.0, 8.0))
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 2.0
    u0 = np.where(rho < 0, np.cos(np.pi * r / 4.0), 0.0)
    return Workload("fisher64", g, rho, u0, beta=1.0, mu=1.0, scheme="etd1", h=0.01, steps=10)


def star512(n: int = 512) -> Workload:
    g = GridSpec(2, (n, n), (-16.0, -16.0), (16.0, 16.0))
    X, Y = g.coords()
    rho = sdf_star(X, Y, lambda t: 3.0 + 0.5 * np.cos(5.0 * t))
    u0 = np.where(rho < 0, 0.5, 0.0)
    return Workload("star512", g, rho, u0, beta=1.0, mu=2.0, scheme="etd2rk", h=0.005, steps=200)


def ellipsoid192(n: int = 192) -> Workload:
    g = GridSpec(3, (n, n, n), (-10.0,) * 3, (10.0,) * 3)
    X, Y, Z = g.coords()
    rho = sdf_prolate_spheroid(X, Y, Z, 3.0, 2.0)
    u0 = _uniform_inside(rho, 0)
    return Workload("ellipsoid192", g, rho, u0, beta=1.0, mu=1.0, scheme="etd2rk", h=0.01, steps=50)


def sphere96(n: int = 96) -> Workload:
    g = GridSpec(3, (n, n, n), (-5.0,) * 3, (5.0,) * 3)
    X, Y, Z = g.coords()
    rho = sdf_sphere(X, Y, Z, 4.0)
    u0 = _uniform_inside(rho, 0)
    return Workload("sphere96", g, rho, u0, beta=1.0, mu=0.0, scheme="etd2rk", h=0.01, steps=40,
                    frozen=True, extra={"checkpoint_every": 8})


def disk4097(n: int = 4097) -> Workload:
    g = GridSpec(2, (n, n), (-16.0, -16.0), (16.0, 16.0))
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 15.0
    u0 = np.where(rho < 0, 0.5 * (1.0 - (r / 15.0) ** 2), 0.0)
    return Workload("disk4097", g, rho, u0, beta=1.0, mu=0.0, scheme="etd2rk", h=5e-4, steps=5,
                    frozen=True)


def sphere385(n: int = 385) -> Workload:
    g = GridSpec(3, (n, n, n), (-10.0,) * 3, (10.0,) * 3)
    X, Y, Z = g.coords()
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = r - 9.5
    u0 = np.where(rho < 0, 0.5 * (1.0 - (r / 9.5) ** 2), 0.0)
    return Workload("sphere385", g, rho, u0, beta=1.0, mu=0.0, scheme="etd2rk", h=1e-3, steps=5,
                    frozen=True)


def batch_params(count: int = 64, seed: int = 0, n_lo: int = 96, n_hi: int = 384):
    """Per-instance draws, in order: side n, R0, a_2..a_6, p_2..p_6, beta."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        R0 = float(rng.uniform(2.0, 4.0))
        a = rng.uniform(0.0, 0.1, size=5)
        p = rng.uniform(0.0, 2.0 * np.pi, size=5)
        beta = float(rng.uniform(0.5, 2.0))
        out.append(dict(n=n, R0=R0, a=a, p=p, beta=beta))
    return out


def batch_instance(params: dict) -> Workload:
    n = params["n"]
    g = GridSpec(2, (n, n), (-8.0, -8.0), (8.0, 8.0))
    X, Y = g.coords()
    R0, a, p = params["R0"], params["a"], params["p"]

    def radius(t):
        acc = np.ones_like(t)
        for j in range(5):
            acc = acc + a[j] * np.cos((j + 2) * t + p[j])
        return R0 * acc

    rho = sdf_star(X, Y, radius)
    u0 = np.where(rho < 0, 0.5, 0.0)
    return Workload(f"batch_n{n}", g, rho, u0, beta=params["beta"], mu=1.0, scheme="etd2rk",
                    h=0.005, steps=100)


def batch64(count: int = 64, seed: int = 0, n_lo: int = 96, n_hi: int = 384):
    return [batch_instance(p) for p in batch_params(count, seed, n_lo, n_hi)]


def scaled(w: Workload, **kw) -> Workload:
    return replace(w, **kw)


WORKLOADS = {
    "fisher64": fisher64,
    "star512": star512,
    "ellipsoid192": ellipsoid192,
    "sphere96": sphere96,
    "disk4097": disk4097,
    "sphere385": sphere385,
}
