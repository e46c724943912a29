"""Pins for oracle.levelset (Section 4.3, Algorithm Steps 1-2).

* HJ-WENO5 one-sided derivatives are exact for cubics and converge at fifth
  order for smooth data.
* A circle (sphere) moved by constant normal speed V has radius R + V t.
* An exact signed distance is (nearly) a fixed point of reinitialisation;
  a distorted level set regains |grad rho| = 1 near its zero set, which stays
  put.
* Aslam extrapolation reproduces a radial quadratic off the known set to
  truncation accuracy.
* The Stefan speed of u = c (R - r) on a disk is mu c near the interface and
  is extended constant along normals.
"""
import numpy as np
import pytest

from oracle import levelset as ls
from oracle.freeboundary import levelset_advance
from oracle.geometry import Grid, classify


def g2(n, L=2.0):
    return Grid(2, (n, n), (-L, -L), (L, L))


def test_weno5_exact_for_cubics():
    g = g2(40)
    X, Y = g.coords()
    phi = 0.3 * X ** 3 - X ** 2 * Y + 2 * Y ** 3 + X * Y - 0.5
    (dxm, dxp), (dym, dyp) = ls.weno_derivatives(phi, g.dx)
    ex = 0.9 * X ** 2 - 2 * X * Y + Y
    ey = -X ** 2 + 6 * Y ** 2 + X
    inner = (slice(3, -3), slice(3, -3))
    for d, e in [(dxm, ex), (dxp, ex), (dym, ey), (dyp, ey)]:
        assert np.abs(d[inner] - e[inner]).max() < 1e-10


def test_weno5_fifth_order_smooth():
    errs = []
    for n in [41, 81]:
        g = g2(n)
        X, Y = g.coords()
        phi = np.sin(1.3 * X) * np.cos(0.7 * Y)
        (dxm, dxp), _ = ls.weno_derivatives(phi, g.dx)
        ex = 1.3 * np.cos(1.3 * X) * np.cos(0.7 * Y)
        inner = (slice(4, -4), slice(4, -4))
        errs.append(max(np.abs(dxm - ex)[inner].max(), np.abs(dxp - ex)[inner].max()))
    assert np.log2(errs[0] / errs[1]) > 4.0


def _zero_radius(g, rho):
    """Radius of the zero set along the +x axis by linear interpolation."""
    j = rho.shape[0] // 2
    row = rho[j] if rho.ndim == 2 else rho[rho.shape[0] // 2, j]
    x = g.axis(0)
    i = np.nonzero((row[:-1] < 0) & (row[1:] >= 0))[0][-1]
    return x[i] - row[i] * (x[i + 1] - x[i]) / (row[i + 1] - row[i])


def test_constant_speed_circle_and_sphere():
    for g in [g2(81), Grid(3, (41, 41, 41), (-2.0,) * 3, (2.0,) * 3)]:
        C = g.coords()
        r = np.sqrt(sum(c * c for c in C))
        rho = r - 1.0
        V = np.full(rho.shape, 0.8)
        rho1 = ls.advect(rho, V, 0.25, g.dx)
        assert _zero_radius(g, rho1) == pytest.approx(1.2, abs=2e-3)


def test_reinit_keeps_signed_distance():
    g = g2(81)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 1.0
    out = ls.reinitialize(rho, g.dx)
    band = (np.abs(rho) < 0.4) & (r > 0.3)
    assert np.abs(out - rho)[band].max() < 2e-3


def test_reinit_restores_distance():
    g = g2(81)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = (r - 1.0) * (1.0 + 0.5 * X + 0.3 * Y * Y)
    out = ls.reinitialize(rho, g.dx, iters=40)
    near = np.abs(r - 1.0) < 3 * g.dx
    assert np.abs(out - (r - 1.0))[near].max() < 5e-3
    assert _zero_radius(g, out) == pytest.approx(1.0, abs=2e-3)


def test_aslam_extrapolates_radial_quadratic():
    g = g2(81)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 1.2
    _, comp, _ = classify(g, rho)
    u = 1.0 - 0.7 * r ** 2
    ext = ls.aslam_extrapolate(np.where(comp, u, 0.0), comp, rho, g.dx)
    band = (~comp) & (np.abs(rho) < 2.5 * g.dx)
    err = np.abs(ext - u)[band].max()
    assert err < 0.02
    # first-order upwind extension: halving h roughly halves the error
    g2_ = g2(161)
    X2, Y2 = g2_.coords()
    r2 = np.hypot(X2, Y2)
    rho2 = r2 - 1.2
    _, comp2, _ = classify(g2_, rho2)
    u2 = 1.0 - 0.7 * r2 ** 2
    ext2 = ls.aslam_extrapolate(np.where(comp2, u2, 0.0), comp2, rho2, g2_.dx, iters=30)
    band2 = (~comp2) & (np.abs(rho2) < 2.5 * g2_.dx)
    assert np.abs(ext2 - u2)[band2].max() < 0.75 * err


def _grown_extension_error(n, grow, shape, iters=ls.ASLAM_ITERS):
    """Max error of the extension of a smooth field F from the computational
    points of a domain to the computational points that a domain grown by
    `grow` cells adds, and the grid spacing."""
    g = Grid(2, (n, n), (-2.0, -2.0), (2.0, 2.0))
    X, Y = g.coords()
    dx = g.dx
    r = np.hypot(X - 0.1, Y + 0.05)
    if shape == "disk":
        rho = r - 1.0
    else:
        rho = r - (1.0 + 0.2 * np.cos(3.0 * np.arctan2(Y + 0.05, X - 0.1)))
    _, c0, _ = classify(g, rho)
    _, c1, _ = classify(g, rho - grow * dx)
    new = c1 & ~c0
    assert new.sum() > 50
    F = np.sin(1.3 * X + 0.4) * np.cos(0.7 * Y) + 0.5 * X * Y
    ext = ls.aslam_extrapolate(np.where(c0, F, 0.0), c0, rho, dx, iters=iters)
    return np.abs(ext - F)[new].max(), dx


@pytest.mark.parametrize("shape", ["disk", "flower"])
@pytest.mark.parametrize("grow", [1.0, float(ls.MAX_FRONT_NODES)])
def test_extension_converges_at_points_joining_the_domain(shape, grow):
    """Section 4.3, Step 2 (used for u and, by ETD2 multistep, for F(U_{n-1})):
    where the boundary moves by up to MAX_FRONT_NODES cells, the
    ASLAM_ITERS-sweep extension of a smooth field matches the field at every
    point that joins the domain to within truncation error, C dx^2 with C
    of the size of its second derivatives, at four resolutions (an
    extension with too few sweeps to converge there misses by 10 to 1000
    times that: 15 sweeps reach 79 dx^2 at two cells, 641^2)."""
    for n in (81, 161, 321, 641):
        err, dx = _grown_extension_error(n, grow, shape)
        assert err < 4.0 * dx * dx, (n, err / (dx * dx))


def test_front_reach_guard():
    """A step whose speed would move the boundary farther than
    MAX_FRONT_NODES nodes is refused before anything moves."""
    g = g2(81)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 1.0
    u = np.where(rho < 0, 0.5 * (1 - r ** 2), 0.0)
    # V ~ mu |du/dr| = mu at r = 1
    dt = 0.05
    mu_ok = 0.9 * ls.MAX_FRONT_NODES * g.dx / dt
    levelset_advance(g, rho, u, dt, mu_ok, reinit=False)
    with pytest.raises(ls.FrontTooFast):
        levelset_advance(g, rho, u, dt, 2.0 * ls.MAX_FRONT_NODES * g.dx / dt, reinit=False)


def test_stefan_velocity_linear_profile():
    g = g2(81)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 1.0
    c, mu = 0.6, 1.5
    u_ext = c * (1.0 - r)                     # |grad u| = c everywhere but r = 0
    V = ls.stefan_velocity(u_ext, rho, g.dx, mu)
    near = np.abs(rho) < 4 * g.dx
    assert np.abs(V[near] - mu * c).max() < 1e-3


def test_levelset_advance_grows_domain_monotonically():
    g = g2(81)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    rho = r - 1.0
    u = np.where(rho < 0, 0.5 * (1 - r ** 2), 0.0)
    _, comp0, _ = classify(g, rho)
    rho1, u1, info = levelset_advance(g, rho, u, 0.04, 1.0, reinit=True)
    _, comp1, _ = classify(g, rho1)
    assert (rho1 <= rho + 1e-12)[np.abs(rho) < 0.5].all()
    assert comp1.sum() >= comp0.sum()
    assert np.all(u1[~comp1] == 0.0)
    # velocity ~ mu |du/dr| = r at r = 1
    near = np.abs(rho) < g.dx
    assert np.abs(info["V"][near] - 1.0).max() < 0.1


def _distorted(dim):
    if dim == 2:
        g = g2(121, 2.5)
        X, Y = g.coords()
        r = np.hypot(X, Y)
        rho = (r - 1.0) * (1.0 + 0.3 * np.sin(2.0 * X) * np.cos(Y))
    else:
        g = Grid(3, (64, 64, 64), (-2.5,) * 3, (2.5,) * 3)
        X, Y, Z = g.coords()
        r = np.sqrt(X * X + Y * Y + Z * Z)
        rho = (r - 1.2) * (1.0 + 0.3 * np.sin(1.5 * X))
    return g, rho


@pytest.mark.parametrize("dim", [2, 3])
def test_banded_reinit_matches_whole_box_near_interface(dim):
    """The narrow band (|rho_0| < REINIT_BAND h) is wide enough: near the
    interface (|rho| < 3h) the banded and whole-box reinitialisations of a
    level set with a 30 % gradient distortion agree to 1e-4 h (a band of 4h
    misses by more), and outside the band rho is left bitwise as it was."""
    g, rho = _distorted(dim)
    h = g.dx
    full = ls.reinitialize(rho, h, band=None)
    bnd = ls.reinitialize(rho, h)
    near = np.abs(full) < 3 * h
    assert np.abs(bnd - full)[near].max() < 1e-4 * h
    outside = np.abs(rho) >= ls.REINIT_BAND * h
    assert np.array_equal(bnd[outside], rho[outside])
    narrow = ls.reinitialize(rho, h, band=4)
    assert np.abs(narrow - full)[near].max() > 1e-4 * h
