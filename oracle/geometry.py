"""Node grid, point classification and boundary geometry (oracle).

Section 2 of the paper: a uniform node grid x_i = x_L + (i-1) h covering a
box (eq. 2.3), the domain is where the level-set function rho < 0
(Section 4.3: rho < 0 inside, rho = 0 on the boundary), and grid points are
split into *interior ghost points* (inside, with at least one of the 2d
nearest neighbours outside) and *computational points* (inside, all 2d
neighbours inside).  The equations are solved at computational points only.

Arrays are numpy arrays in box layout: shape (ny, nx) in 2D and (nz, ny, nx)
in 3D, x fastest.  Spatial axis d (0 = x, 1 = y, 2 = z) is numpy axis
ndim - 1 - d.

Readings of the paper used here (both this oracle and the GPU path follow
them):
* inside <=> rho < 0 strictly; rho = 0 counts as outside.
* nodes of the outermost box layer are never computational (a missing
  neighbour counts as outside); a computational node closer than 2 layers to
  the box edge is a domain error (the Case-2/3 test looks two nodes out).
* the interface crossing on a grid line (the paper suggests a secant
  method) is the root of the linear interpolant of the grid values of rho.
* the closest boundary point of a node x is one projection step
  x - rho(x) g / |g|^2 with g the central-difference gradient of rho at x.

Pins (tests/test_oracle_operator.py): classification counts against brute
force loops; crossing fraction exact for linear rho; closest point exact for
a planar signed distance and within O(h^2) of the analytic point on a circle.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    """n[d] nodes on [lo[d], hi[d]] per axis d (x, y[, z]); equal spacing."""

    dim: int
    n: tuple
    lo: tuple
    hi: tuple

    @property
    def dx(self) -> float:
        return (self.hi[0] - self.lo[0]) / (self.n[0] - 1)

    @property
    def shape(self) -> tuple:
        return tuple(reversed(self.n[: self.dim]))

    def axis(self, d: int) -> np.ndarray:
        return self.lo[d] + self.dx * np.arange(self.n[d])

    def coords(self):
        """Coordinate arrays (x, y[, z]) in box layout."""
        axes = [self.axis(d) for d in range(self.dim)]
        mesh = np.meshgrid(*reversed(axes), indexing="ij")
        return tuple(reversed(mesh))

    def point(self, idx):
        """Coordinates of the node with numpy index tuple idx."""
        return np.array([self.lo[d] + self.dx * idx[self.dim - 1 - d] for d in range(self.dim)])


def np_axis(grid: Grid, d: int) -> int:
    return grid.dim - 1 - d


def shifted(a: np.ndarray, ax: int, s: int, fill):
    """b[i] = a[i + s] along numpy axis ax, with `fill` beyond the box."""
    b = np.full_like(a, fill)
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if s > 0:
        src[ax] = slice(s, None)
        dst[ax] = slice(None, -s)
    else:
        src[ax] = slice(None, s)
        dst[ax] = slice(-s, None)
    b[tuple(dst)] = a[tuple(src)]
    return b


def classify(grid: Grid, rho: np.ndarray):
    """Return (inside, comp, ghost) boolean box arrays (Section 2)."""
    inside = rho < 0.0
    comp = inside.copy()
    for d in range(grid.dim):
        ax = np_axis(grid, d)
        for s in (-1, 1):
            comp &= shifted(inside, ax, s, False)
    ghost = inside & ~comp
    return inside, comp, ghost


class DomainError(ValueError):
    """A computational node lies within 2 layers of the box edge."""


def check_domain(grid: Grid, comp: np.ndarray):
    """Raise DomainError if a computational node is in the two outer layers."""
    for d in range(grid.dim):
        ax = np_axis(grid, d)
        n = comp.shape[ax]
        for layer in (0, 1, n - 2, n - 1):
            if np.take(comp, layer, axis=ax).any():
                raise DomainError("computational node within 2 layers of the box edge")


def crossing_fraction(rho_near: float, rho_far: float) -> float:
    """Position of the interface between an inside node (rho_near < 0) and
    the next node on the line (rho_far >= 0), as a fraction of h measured
    from the inside node: root of the linear interpolant of rho."""
    return rho_near / (rho_near - rho_far)


def central_gradient(grid: Grid, rho: np.ndarray, idx) -> np.ndarray:
    """Central-difference gradient of rho at an interior node (idx = numpy
    index tuple); component d is the x/y/z derivative."""
    g = np.zeros(grid.dim)
    h = grid.dx
    for d in range(grid.dim):
        ax = np_axis(grid, d)
        ip = list(idx)
        im = list(idx)
        ip[ax] += 1
        im[ax] -= 1
        g[d] = (rho[tuple(ip)] - rho[tuple(im)]) / (2.0 * h)
    return g


def closest_point(grid: Grid, rho: np.ndarray, idx):
    """One projection step towards the zero level set from node idx.
    Returns (point, gradient); point is None when the gradient vanishes."""
    g = central_gradient(grid, rho, idx)
    gg = float(g @ g)
    x = grid.point(idx)
    if gg < 1e-300:
        return None, g
    return x - rho[idx] * g / gg, g
