"""Pins for oracle.geometry / oracle.operator (Section 2 of the paper).

A wrong sign, index, crossing distance, face coefficient or Case-3 weight
fails at least one of: brute-force classification, exact linear /
quadratic consistency, symmetry + definiteness, the 6x6 RBF solve vs
barycentric interpolation, second-order eigenfunction decay on a disk and a
sphere, and second-order convergence of the Poisson problem of Section 4.1.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy
from scipy.special import j0

from oracle.geometry import Grid, classify, closest_point, crossing_fraction
from oracle.operator import build_operator, rbf_weights_2d
from oracle.phi import phi_combination
from paper_2209_15095_amd.inputs import sdf_star, virus_level_set


def grid2(n, L):
    return Grid(2, (n, n), (-L, -L), (L, L))


def grid3(n, L):
    return Grid(3, (n, n, n), (-L, -L, -L), (L, L, L))


def test_classification_brute_force():
    for g in [grid2(23, 1.0), grid3(11, 1.0)]:
        C = g.coords()
        rho = sum(c * c for c in C) - 0.55 + 0.2 * C[0] * C[1]
        inside, comp, ghost = classify(g, rho)
        for idx in np.ndindex(*rho.shape):
            ins = rho[idx] < 0
            nb_in = True
            for ax in range(rho.ndim):
                for s in (-1, 1):
                    j = list(idx)
                    j[ax] += s
                    if j[ax] < 0 or j[ax] >= rho.shape[ax]:
                        nb_in = False
                    elif not rho[tuple(j)] < 0:
                        nb_in = False
            assert inside[idx] == ins
            assert comp[idx] == (ins and nb_in)
            assert ghost[idx] == (ins and not nb_in)


def test_crossing_fraction_linear():
    for r0, r1 in [(-0.3, 0.7), (-1e-3, 2.0), (-0.5, 0.0)]:
        th = crossing_fraction(r0, r1)
        assert r0 + th * (r1 - r0) == pytest.approx(0.0, abs=1e-15)


def test_closest_point_planar_exact():
    for g in [grid2(15, 1.0), grid3(9, 1.0)]:
        nrm = np.array([0.3, -0.8, 0.52][: g.dim])
        nrm /= np.linalg.norm(nrm)
        C = g.coords()
        rho = sum(nd * c for nd, c in zip(nrm, C)) - 0.1
        idx = tuple(s // 2 + 1 for s in rho.shape)
        pt, _ = closest_point(g, rho, idx)
        assert abs(pt @ nrm - 0.1) < 1e-14
        x = g.point(idx)
        assert np.linalg.norm((x - pt) - (x @ nrm - 0.1) * nrm) < 1e-14


def test_closest_point_circle_second_order():
    errs = []
    for n in [41, 81]:
        g = grid2(n, 2.0)
        X, Y = g.coords()
        rho = np.hypot(X, Y) ** 2 / 2.0 - 0.5 * 1.0  # not a distance: |grad| = r
        idx = (n // 2 + n // 8, n // 2 + n // 5)
        pt, _ = closest_point(g, rho, idx)
        errs.append(abs(np.linalg.norm(pt) - 1.0))
    assert errs[1] < errs[0]


def _domains():
    g = grid2(48, 2.0)
    X, Y = g.coords()
    yield g, sdf_star(X, Y, lambda t: 1.3 + 0.25 * np.cos(5 * t))
    g = grid3(22, 2.0)
    X, Y, Z = g.coords()
    yield g, np.sqrt((X / 1.2) ** 2 + Y ** 2 + (Z / 0.9) ** 2) - 1.3


@pytest.mark.parametrize("beta", [1.0, "var"])
def test_symmetric_negative_definite_gershgorin(beta):
    for g, rho in _domains():
        b = (lambda P: 1.0 + 0.3 * P[:, 0] ** 2 + 0.2 * P[:, 1]) if beta == "var" else beta
        op = build_operator(g, rho, b)
        A = op.A.toarray()
        assert np.abs(A - A.T).max() == 0.0
        lam = np.linalg.eigvalsh(A)
        assert lam.max() < 0.0
        bmax = 1.0 if beta == 1.0 else 1.0 + 0.3 * 4 + 0.2 * 2
        assert -lam.min() <= 4 * g.dim * bmax / g.dx ** 2 * 1.0001
        assert op.counts["case2"] > 0 and op.counts["case3"] > 0


def test_case1_rows_exact_for_quadratic_with_linear_beta():
    """Conservative face-midpoint scheme: exact for beta linear, u quadratic."""
    g = grid2(40, 2.0)
    X, Y = g.coords()
    rho = np.hypot(X, Y) - 1.5
    beta = lambda P: 1.0 + 0.3 * P[:, 0] - 0.2 * P[:, 1]
    op = build_operator(g, rho, beta)
    u = 1.0 + X - 2 * Y + 0.7 * X * X - 0.4 * X * Y + 1.3 * Y * Y
    Au = op.A @ op.gather(u)
    # exact div(beta grad u)
    ux = 1.0 + 1.4 * X - 0.4 * Y
    uy = -2.0 - 0.4 * X + 2.6 * Y
    bb = 1.0 + 0.3 * X - 0.2 * Y
    exact = 0.3 * ux + bb * 1.4 - 0.2 * uy + bb * 2.6
    # rows whose 4 neighbours are computational (pure Case 1)
    _, comp, _ = classify(g, rho)
    pure = comp.copy()
    for ax in (0, 1):
        for s in (-1, 1):
            pure &= np.roll(comp, s, axis=ax)
    sel = pure[comp]
    assert sel.sum() > 100
    assert np.abs(Au[sel] - exact[comp][sel]).max() < 1e-10


def test_linear_exact_with_boundary_data_2d():
    """Linear u with exact Dirichlet data: discrete residual vanishes at every
    row (pins Case-2 crossing distance and Case-3 weights)."""
    g = grid2(60, 2.0)
    X, Y = g.coords()
    rho = sdf_star(X, Y, lambda t: 1.2 + 0.3 * np.cos(5 * t))
    op = build_operator(g, rho, 1.7)
    assert op.counts["case3"] > 0 and op.counts["case2"] > 0
    uf = lambda P: 0.4 + 2.0 * P[0] - 3.0 * P[1]
    u = 0.4 + 2.0 * X - 3.0 * Y
    res = op.A @ op.gather(u) + op.forcing(uf)
    assert np.abs(res).max() < 1e-9 * (1.7 / g.dx ** 2)


def test_linear_exact_planar_3d():
    """3D, tilted planar boundary, u = distance to the plane (zero on it):
    A u = 0 exactly, including Case-3 rows (plane reading of Case 3)."""
    g = grid3(24, 1.0)
    X, Y, Z = g.coords()
    nrm = np.array([0.45, 0.6, 0.66])
    nrm /= np.linalg.norm(nrm)
    rho = nrm[0] * X + nrm[1] * Y + nrm[2] * Z - 0.35
    rho = np.maximum(rho, np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - 0.9)  # keep the domain off the box edge
    op = build_operator(g, rho, 1.0)
    assert op.counts["case3"] > 0
    u = -(nrm[0] * X + nrm[1] * Y + nrm[2] * Z - 0.35)
    Au = op.A @ op.gather(u)
    # rows whose ghost neighbours all see the plane (away from the sphere cap)
    _, comp, _ = classify(g, rho)
    near_plane = (np.abs(u) < 3 * g.dx) & (np.sqrt(X ** 2 + Y ** 2 + Z ** 2) < 0.9 - 4 * g.dx)
    sel = near_plane[comp]
    assert sel.sum() > 20
    assert np.abs(Au[sel]).max() < 1e-9 / g.dx ** 2


def test_rbf_equals_barycentric():
    rng = np.random.default_rng(0)
    for _ in range(50):
        P = rng.standard_normal((4, 2))
        w = rbf_weights_2d(P[0], P[1], P[2], P[3])
        T = np.array([[1, 1, 1], [P[0, 0], P[1, 0], P[2, 0]], [P[0, 1], P[1, 1], P[2, 1]]])
        bary = np.linalg.solve(T, np.array([1.0, P[3, 0], P[3, 1]]))
        assert np.allclose(w, bary, atol=1e-10)
        # independent of the radial function
        w2 = rbf_weights_2d(P[0], P[1], P[2], P[3], psi=lambda r: np.sqrt(r * r + 0.3))
        assert np.allclose(w2, bary, atol=1e-9)


def _decay_error_disk(n, R=1.0, T=0.05):
    g = grid2(n, 1.3)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - R
    op = build_operator(g, rho, 1.0)
    j01 = 2.404825557695773
    u0 = op.gather(j0(j01 * r / R))
    uT = phi_combination(op.A, T, [u0], method="krylov")
    exact = np.exp(-j01 ** 2 * T / R ** 2) * u0
    return np.abs(uT - exact).max()


def test_disk_eigenfunction_decay_second_order():
    """Observed order over a 4x refinement (EB errors oscillate between
    neighbouring resolutions, as in Table 1 of the paper)."""
    e1 = _decay_error_disk(41)
    e2 = _decay_error_disk(161)
    assert e2 < 2e-4
    assert np.log2(e1 / e2) / 2.0 > 1.4


def _decay_error_sphere(n, R=1.0, T=0.05):
    g = grid3(n, 1.3)
    X, Y, Z = g.coords()
    r = np.sqrt(X * X + Y * Y + Z * Z)
    op = build_operator(g, r - R, 1.0)
    rr = np.maximum(r, 1e-12)
    u0 = op.gather(np.sin(np.pi * rr / R) / (np.pi * rr / R))
    uT = phi_combination(op.A, T, [u0], method="krylov")
    exact = np.exp(-np.pi ** 2 * T / R ** 2) * u0
    return np.abs(uT - exact).max()


def test_sphere_eigenfunction_decay_second_order():
    e1 = _decay_error_sphere(21)
    e2 = _decay_error_sphere(41)
    assert e2 < 5e-3
    assert np.log2(e1 / e2) > 1.5


def _virus_problem():
    x, y = sympy.symbols("x y")
    u = sympy.exp(x) * (x ** 2 * sympy.sin(y) + y ** 2)
    beta = 2 + sympy.sin(x * y)
    f = sympy.diff(beta * sympy.diff(u, x), x) + sympy.diff(beta * sympy.diff(u, y), y)
    return (sympy.lambdify((x, y), u, "numpy"), sympy.lambdify((x, y), beta, "numpy"),
            sympy.lambdify((x, y), f, "numpy"))


def test_poisson_virus_second_order():
    """Section 4.1: second-order solution on the virus geometry."""
    uf, bf, ff = _virus_problem()
    errs = []
    for N in [50, 100, 200]:
        g = Grid(2, (N + 1, N + 1), (-1.0, -1.0), (1.0, 1.0))
        X, Y = g.coords()
        rho = virus_level_set(X, Y)
        op = build_operator(g, rho, lambda P: bf(P[:, 0], P[:, 1]))
        rhs = op.gather(ff(X, Y)) - op.forcing(lambda P: uf(P[0], P[1]))
        sol = spla.spsolve(op.A.tocsc(), rhs)
        errs.append(np.abs(sol - op.gather(uf(X, Y))).max())
    order = np.log2(errs[0] / errs[2]) / 2.0
    assert order > 1.7, errs
    assert errs[-1] < 5e-4
