"""GPU parity of variable beta(x) and non-homogeneous Dirichlet data.

Section 2 (eq. 2.4 with beta at the face midpoints, the Case 2/3 ghost
closures with boundary data) and the accuracy test of Section 4.2.1: the
peanut domain rho = 0.5 - exp(-20(x^2+(y-1/4)^2)) - exp(-20(x^2+(y+1/4)^2))
< 0 in [-1,1]^2, beta = 1/4 - x^2 - y^2, exact u = e^{-t}(x^2+y^2-1/4),
source f = e^{-t}(7 r^2 - 3/4) (derived in tests/test_oracle_etd.py),
ETD2RK with dt = h to t = 0.1.

* etd_geometry_build_var: the operator against the oracle's CSR matrix, and
  the boundary forcing of etd_forcing_assemble against the oracle's taps,
  in 2D (peanut) and 3D (a spheroid with a variable beta), to rounding.
* Table 1 (ETD2RK rows 81^2 x 4, 161^2 x 8 and 321^2 x 16 steps): the GPU
  run through etd_step_forced against the oracle's run (1e-9 relative L2)
  and against the exact solution, inside the bands of the printed errors
  (tests/golden/table1_etd2rk.json).
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.etd import etd2rk_step
from oracle.geometry import Grid
from oracle.operator import build_operator
from paper_2209_15095_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_etd2rk.json")


def say(msg):
    print(f"[gpu-variable] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def u_exact(P, t):
    return np.exp(-t) * (np.sum(P * P, axis=-1) - 0.25)


def beta_peanut(P):
    return 0.25 - np.sum(P * P, axis=-1)


def source(X, Y, t):
    return np.exp(-t) * (7.0 * (X * X + Y * Y) - 0.75)


def face_betas(g, beta):
    """beta at node + h/2 e_d for every node (box arrays), the midpoints
    written as the oracle writes them (lo + h (i + 1/2))."""
    axes = [g.lo[d] + g.dx * np.arange(g.n[d]) for d in range(g.dim)]
    out = []
    for d in range(g.dim):
        ax = list(axes)
        ax[d] = g.lo[d] + g.dx * 0.5 * (2.0 * np.arange(g.n[d]) + 1.0)
        mesh = np.meshgrid(*reversed(ax), indexing="ij")
        P = np.stack(list(reversed(mesh)), axis=-1)
        out.append(beta(P))
    return out


def ctx_for(g, **kw):
    from paper_2209_15095_amd.api import Context
    return Context(g.dim, g.n, g.lo, g.hi, **kw)


def peanut(n):
    g = inputs.GridSpec(2, (n, n), (-1.0, -1.0), (1.0, 1.0))
    X, Y = g.coords()
    return g, X, Y, inputs.peanut_level_set(X, Y)


def spheroid3d(n=40):
    g = inputs.GridSpec(3, (n, n, n), (-1.0,) * 3, (1.0,) * 3)
    X, Y, Z = g.coords()
    return g, X, Y, Z, inputs.sdf_prolate_spheroid(X, Y, Z, 0.7, 0.5)


@pytest.mark.parametrize("case", ["peanut81", "spheroid40"])
def test_variable_operator_and_forcing_match_oracle(case):
    if case == "peanut81":
        g, X, Y, rho = peanut(81)
        beta = beta_peanut
    else:
        g, X, Y, Z, rho = spheroid3d()
        beta = lambda P: 1.0 + 0.5 * P[..., 0] - 0.3 * P[..., 1] * P[..., 2]
    og = Grid(g.dim, tuple(g.n), tuple(g.lo), tuple(g.hi))
    op = build_operator(og, rho, lambda P: beta(P))
    say(f"{case}: N {op.n}, taps {len(op.taps)}")
    ctx = ctx_for(g)
    ctx.geometry_build_var(dev(rho), [dev(b) for b in face_betas(g, beta)])
    rng = np.random.default_rng(2)
    v = rng.standard_normal(rho.shape)
    out = host(ctx.operator_apply(dev(v)))
    ref = op.scatter(op.A @ op.gather(v))
    say(f"  operator max diff {np.abs(out - ref).max() / np.abs(ref).max():.2e}")
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()
    pts = ctx.boundary_taps()
    assert pts.shape == (len(op.taps), g.dim)
    # same set of boundary points as the oracle's taps (nearest point both ways)
    from scipy.spatial import cKDTree
    opts = np.array([t[2] for t in op.taps])
    d1, _ = cKDTree(opts).query(pts)
    d2, _ = cKDTree(pts).query(opts)
    say(f"  tap points: max distance {max(d1.max(), d2.max()):.2e}")
    assert max(d1.max(), d2.max()) <= 1e-12
    t = 0.37
    src = rng.standard_normal(rho.shape)
    G = host(ctx.forcing_assemble(dev(u_exact(pts, t)), dev(src)))
    Gref = op.scatter(op.gather(src) + op.forcing(lambda P: u_exact(np.asarray(P), t)))
    say(f"  forcing max diff {np.abs(G - Gref).max() / np.abs(Gref).max():.2e}")
    assert np.abs(G - Gref).max() <= 1e-13 * np.abs(Gref).max()
    ctx.close()


def test_peanut_table1_etd2rk_on_gpu():
    rows = json.load(open(GOLDEN))["rows"][:3]
    T = 0.1
    for r in rows:
        n, steps = r["nodes"], r["steps"]
        h = T / steps
        g, X, Y, rho = peanut(n)
        og = Grid(2, (n, n), (-1.0, -1.0), (1.0, 1.0))
        op = build_operator(og, rho, lambda P: beta_peanut(P))
        Xc, Yc = op.gather(X), op.gather(Y)
        # oracle run (the Table 1 algorithm of tests/test_oracle_etd.py)
        F = lambda u, t: source(Xc, Yc, t) + op.forcing(lambda P: u_exact(np.asarray(P), t))
        U = u_exact(np.stack([Xc, Yc], axis=-1), 0.0)
        for m in range(steps):
            U = etd2rk_step(op.A, h, U, F, m * h, method="dense" if op.n < 1500 else "krylov")
        # GPU run
        ctx = ctx_for(g, a=0.0, b=0.0)
        ctx.geometry_build_var(dev(rho), [dev(b) for b in face_betas(g, beta_peanut)])
        pts = ctx.boundary_taps()

        def G(t):
            return ctx.forcing_assemble(dev(u_exact(pts, t)), dev(source(X, Y, t)))

        ud = dev(np.where(op.comp, u_exact(np.stack([X, Y], axis=-1), 0.0), 0.0))
        for m in range(steps):
            ctx.etd_step_forced("etd2rk", h, ud, [G(m * h), None, G((m + 1) * h)])
        ug = host(ud)
        ctx.close()
        e = ug[op.comp] - u_exact(np.stack([Xc, Yc], axis=-1), T)
        linf, l2 = float(np.abs(e).max()), float(np.sqrt(np.mean(e * e)))
        say(f"  {n}^2 x {steps}: GPU vs oracle {rel_l2(ug[op.comp], U):.2e}; "
            f"l_inf {linf:.3e} (printed {r['linf']:.3e}), l2 {l2:.3e} (printed {r['l2']:.3e})")
        assert rel_l2(ug[op.comp], U) <= 1e-9
        assert np.all(ug[~op.comp] == 0.0)
        assert r["linf"] / 3.0 < linf < r["linf"] * 3.0
        assert r["l2"] / 4.0 < l2 < r["l2"] * 4.0
