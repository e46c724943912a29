"""Embedded-boundary discretisation of div(beta grad u) (oracle).

Section 2 of the paper.  Unknowns are the values at computational points, in
lexicographic box order (x fastest).  For a computational point p and each
axis direction +-e_d with neighbour q = p +- e_d and face coefficient
beta_pq (beta at the face midpoint):

* Case 1, q computational (eq. 2.4): off-diagonal beta_pq/h^2 and
  diagonal -beta_pq/h^2.
* Case 2, q an interior ghost point whose next node q2 = q +- e_d on the
  same line is outside (the ghost borders the interface on this line): the
  ghost value is the linear Lagrange interpolant of u_p and the boundary
  value u_G at the crossing, u_q = u_G h/s + u_p (s-h)/s with s in (h, 2h]
  the distance from p to the crossing.  Only the diagonal changes:
  -beta_pq/(h s); the boundary part beta_pq u_G/(h s) is forcing.
* Case 3, q a ghost whose next node q2 is inside: u_q is interpolated from
  u_p and the boundary values at the closest boundary points x_G1 of q and
  x_G2 of p.  In 2D this is the paper's RBF interpolant with a linear tail
  (eqs. 2.5-2.6, the 6 x 6 system, here with psi(r) = r^3); with three
  centres and a linear tail the RBF coefficients vanish, so the result is
  the linear interpolant and does not depend on psi.  The weight w_p of u_p
  enters the diagonal as -beta_pq (1 - w_p)/h^2 (symmetry is kept: only the
  diagonal changes), the boundary weights are forcing.

3D Case 3 is not defined by the paper (its examples are 2D): with three
centres a linear tail in 3D is under-determined.  Reading used here and on
the GPU: u_q is the linear function that vanishes on the plane containing
x_G1 and x_G2 whose normal is the part of the averaged level-set normal
orthogonal to x_G2 - x_G1, and equals u_p at p; so w_p is the ratio of the
signed distances of q and p to that plane.  In 2D that plane is the line
x_G1 x_G2 and the same ratio is exactly the RBF weight.  Degenerate
configurations (vanishing gradient, x_G1 = x_G2 in 2D, normal parallel to
the chord, p on the plane) fall back to w_p = rho_q / rho_p.

Pins (tests/test_oracle_operator.py): symmetry, negative definiteness and
Gershgorin bounds; exact discrete Laplacian of quadratics at Case-1 rows;
zero residual for linear functions with exact boundary data (pins the
Case-2 crossing distance and the Case-3 weights); the 2D RBF solve equal to
barycentric interpolation; eigenfunction decay on a disk and a sphere
converging at second order; Poisson convergence on the virus geometry of
Section 4.1 at order about 2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .geometry import (DomainError, Grid, check_domain, classify, closest_point,
                       crossing_fraction, np_axis)


@dataclass
class EBOperator:
    grid: Grid
    comp: np.ndarray            # bool box array
    inside: np.ndarray
    index: np.ndarray           # int box array, -1 off the unknowns
    A: sp.csr_matrix            # N_c x N_c
    taps: list = field(default_factory=list)   # (row, coef, point) boundary forcing taps
    counts: dict = field(default_factory=dict)
    case3_weights: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    def gather(self, box: np.ndarray) -> np.ndarray:
        return np.asarray(box)[self.comp]

    def scatter(self, vec: np.ndarray) -> np.ndarray:
        out = np.zeros(self.comp.shape)
        out[self.comp] = vec
        return out

    def forcing(self, u_boundary) -> np.ndarray:
        """Boundary forcing vector g for Dirichlet data u_boundary(point),
        so that the discrete operator applied to u is A u + g."""
        g = np.zeros(self.n)
        for row, coef, pt in self.taps:
            g[row] += coef * u_boundary(pt)
        return g


def _beta_at(beta, pts):
    """beta at an (m, dim) array of points: a constant or a vectorised callable."""
    pts = np.atleast_2d(pts)
    if callable(beta):
        return np.asarray(beta(pts), dtype=np.float64).reshape(pts.shape[0])
    return np.full(pts.shape[0], float(beta))


def rbf_weights_2d(x_p, x_g1, x_g2, x_q, psi=lambda r: r ** 3):
    """Weights (w_p, w_G1, w_G2) of the RBF interpolant with linear tail
    (eqs. 2.5-2.6) through x_p, x_G1, x_G2, evaluated at x_q (2D)."""
    pts = [np.asarray(x_p), np.asarray(x_g1), np.asarray(x_g2)]
    B = np.zeros((6, 6))
    for i in range(3):
        for j in range(3):
            B[i, j] = psi(np.linalg.norm(pts[i] - pts[j]))
        B[i, 3] = 1.0
        B[i, 4] = pts[i][0]
        B[i, 5] = pts[i][1]
        B[3, i] = 1.0
        B[4, i] = pts[i][0]
        B[5, i] = pts[i][1]
    row = np.array([psi(np.linalg.norm(x_q - pts[0])), psi(np.linalg.norm(x_q - pts[1])),
                    psi(np.linalg.norm(x_q - pts[2])), 1.0, x_q[0], x_q[1]])
    # u_q = row . B^{-1} [u; 0]  =>  weights = (B^{-T} row)[:3]
    w = np.linalg.solve(B.T, row)
    return w[:3]


def case3_weights(grid: Grid, rho: np.ndarray, p_idx, q_idx):
    """Interpolation weights (w_p, w_G1, w_G2) and points (x_G1, x_G2) for
    the ghost value at q from p and the closest boundary points."""
    h = grid.dx
    x_p = grid.point(p_idx)
    x_q = grid.point(q_idx)
    g1, gq = closest_point(grid, rho, q_idx)
    g2, gp = closest_point(grid, rho, p_idx)
    fallback = (rho[q_idx] / rho[p_idx], None, None)
    if g1 is None or g2 is None:
        return fallback
    ng = gq / np.linalg.norm(gq) + gp / np.linalg.norm(gp)
    if np.linalg.norm(ng) < 1e-12:
        return fallback
    nbar = ng / np.linalg.norm(ng)
    t = g2 - g1
    L = np.linalg.norm(t)
    if L < 1e-12 * h:
        if grid.dim == 2:
            return fallback
        nu = nbar
    else:
        that = t / L
        nu = nbar - (nbar @ that) * that
        nn = np.linalg.norm(nu)
        if nn < 1e-8:
            return fallback
        nu = nu / nn
    dp = (x_p - g1) @ nu
    dq = (x_q - g1) @ nu
    if abs(dp) < 1e-10 * h:
        return fallback
    if grid.dim == 2:
        w = rbf_weights_2d(x_p, g1, g2, x_q)
        return (float(w[0]), (float(w[1]), g1), (float(w[2]), g2))
    wp = dq / dp
    # boundary data (inhomogeneous case only): shared equally by the two feet
    return (float(wp), (0.5 * (1.0 - wp), g1), (0.5 * (1.0 - wp), g2))


def build_operator(grid: Grid, rho: np.ndarray, beta=1.0, check=True) -> EBOperator:
    """Assemble A (scipy CSR) for the domain rho < 0 (Section 2, Cases 1-3)."""
    rho = np.asarray(rho, dtype=np.float64)
    inside, comp, _ = classify(grid, rho)
    if check:
        check_domain(grid, comp)
    index = -np.ones(rho.shape, dtype=np.int64)
    n = int(comp.sum())
    index[comp] = np.arange(n)
    h = grid.dx
    h2 = h * h
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    taps = []
    counts = {"case1": 0, "case2": 0, "case3": 0, "case3_fallback": 0, "case3_w_gt1": 0}
    weights = []
    coords = grid.coords()
    p_all = np.argwhere(comp)                               # (m, ndim) numpy indices
    pt = tuple(p_all.T)
    xp = np.stack([c[pt] for c in coords], axis=1)
    r = index[pt]
    for d in range(grid.dim):
        ax = np_axis(grid, d)
        e_d = np.eye(grid.dim)[d]
        for s in (-1, 1):
            q_all = p_all.copy()
            q_all[:, ax] += s
            qt = tuple(q_all.T)
            xq = xp + s * h * e_d[None, :]
            # face midpoint from integer indices: identical from both sides
            mid = np.stack([grid.lo[dd] + h * 0.5 * (p_all[:, np_axis(grid, dd)] + q_all[:, np_axis(grid, dd)])
                            for dd in range(grid.dim)], axis=1)
            bf = _beta_at(beta, mid)
            # Case 1: neighbour computational
            c1 = comp[qt]
            rows.append(r[c1])
            cols.append(index[qt][c1])
            vals.append(bf[c1] / h2)
            np.subtract.at(diag, r[c1], bf[c1] / h2)
            counts["case1"] += int(c1.sum())
            assert inside[qt].all(), "neighbour of a computational point must be inside"
            # ghost neighbour: look one node further along the line
            q2_all = q_all.copy()
            q2_all[:, ax] += s
            q2t = tuple(q2_all.T)
            c2 = ~c1 & ~inside[q2t]
            c3 = ~c1 & inside[q2t]
            # Case 2: the ghost borders the interface on this line
            theta = crossing_fraction(rho[qt][c2], rho[q2t][c2])
            dist = (1.0 + theta) * h
            np.subtract.at(diag, r[c2], bf[c2] / (h * dist))
            xg = xq[c2] + (s * theta * h)[:, None] * e_d[None, :]
            for rr, cc, xx in zip(r[c2], bf[c2] / (h * dist), xg):
                taps.append((int(rr), float(cc), xx))
            counts["case2"] += int(c2.sum())
            # Case 3: the ghost does not border the interface on this line
            for k in np.nonzero(c3)[0]:
                p = tuple(p_all[k])
                q = tuple(q_all[k])
                wp, t1, t2 = case3_weights(grid, rho, p, q)
                rr = int(r[k])
                diag[rr] -= bf[k] * (1.0 - wp) / h2
                counts["case3"] += 1
                if t1 is None:
                    counts["case3_fallback"] += 1
                    g1, _ = closest_point(grid, rho, q)
                    taps.append((rr, bf[k] * (1.0 - wp) / h2, g1 if g1 is not None else xq[k]))
                else:
                    taps.append((rr, bf[k] * t1[0] / h2, t1[1]))
                    taps.append((rr, bf[k] * t2[0] / h2, t2[1]))
                if wp > 1.0:
                    counts["case3_w_gt1"] += 1
                weights.append(wp)
    rows = np.concatenate(rows + [np.arange(n)])
    cols = np.concatenate(cols + [np.arange(n)])
    vals = np.concatenate(vals + [diag])
    A = sp.csr_matrix((vals, (rows.astype(np.int64), cols.astype(np.int64))), shape=(n, n))
    A.sum_duplicates()
    return EBOperator(grid=grid, comp=comp, inside=inside, index=index, A=A, taps=taps,
                      counts=counts, case3_weights=weights)


def diagonal_box(op: EBOperator) -> np.ndarray:
    """Diagonal of A scattered to the box (0 off the unknowns)."""
    return op.scatter(op.A.diagonal())


__all__ = ["EBOperator", "build_operator", "case3_weights", "rbf_weights_2d",
           "diagonal_box", "DomainError"]
