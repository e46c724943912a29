"""GPU parity at the full sizes of the 2D and 3D free-boundary workloads.

* star512 (512^2 star, ETD2RK h = 0.005, mu = 2, reinitialisation every 5
  steps): the first 10 steps of the workload, end to end, against the oracle
  (masks equal, rho to 1e-10, u to 1e-9 relative L2).
* ellipsoid192 (192^3 prolate spheroid, 38,824 unknowns): classification
  equal to the oracle's, the operator to rounding, one frozen ETD2RK step
  against the oracle's Krylov route to 1e-9, and the first free-boundary step
  of the workload (level set, geometry, ETD2RK) against the oracle's (masks
  equal, rho to 1e-10, u to 1e-9 relative L2); also a property of the
  full-size level set: with V >= 0 and no reinitialisation rho can only
  decrease, and the domain only grows.
* The 3D level-set step against the oracle at 64^3 (with reinitialisation)
  and a 3D free-boundary run of 4 steps at 48^3.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.etd import etd_step as oracle_etd_step, logistic
from oracle.freeboundary import free_boundary_step, levelset_advance as oracle_levelset_advance
from oracle.geometry import Grid, classify
from oracle.operator import build_operator
from paper_2209_15095_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-configs] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ogrid(g):
    return Grid(g.dim, tuple(g.n), tuple(g.lo), tuple(g.hi))


def ctx_for(grid, **kw):
    from paper_2209_15095_amd.api import Context
    return Context(grid.dim, grid.n, grid.lo, grid.hi, **kw)


def test_star512_first_steps_end_to_end():
    w = inputs.star512()
    steps = 10
    say(f"star512: {steps} free-boundary ETD2RK steps")
    og = ogrid(w.grid)
    rho, u = w.rho0.copy(), w.u0.copy()
    ctx = ctx_for(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu)
    rd, ud = dev(rho), dev(u)
    ctx.geometry_build(rd)
    for m in range(steps):
        reinit = (m + 1) % w.reinit_every == 0
        rho, u, op = free_boundary_step(og, rho, u, w.h, w.beta, w.mu, w.a, w.b, scheme=w.scheme,
                                        reinit=reinit, method="krylov")
        ctx.etd_step(w.scheme, w.h, ud, rho=rd, reinit=reinit)
    rg, ug = host(rd), host(ud)
    ctx.close()
    _, comp_g, _ = classify(og, rg)
    say(f"  N {op.n}  rho diff {np.abs(rg - rho).max():.3e}  u rel {rel_l2(ug[op.comp], u[op.comp]):.3e}")
    assert np.array_equal(comp_g, op.comp)
    assert np.abs(rg - rho).max() <= 1e-10
    assert rel_l2(ug[op.comp], u[op.comp]) <= 1e-9
    assert np.all(ug[~op.comp] == 0.0)


@pytest.fixture(scope="module")
def ellipsoid():
    say("ellipsoid192 inputs (exact signed distance)")
    return inputs.ellipsoid192()


def test_ellipsoid192_geometry_operator_and_step(ellipsoid):
    w = ellipsoid
    og = ogrid(w.grid)
    op = build_operator(og, w.rho0, w.beta)
    say(f"ellipsoid192: N {op.n}")
    ctx = ctx_for(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu)
    ctx.geometry_build(dev(w.rho0))
    # operator at full size
    rng = np.random.default_rng(11)
    v = rng.standard_normal(w.rho0.shape)
    out = host(ctx.operator_apply(dev(v)))
    ref = op.scatter(op.A @ op.gather(v))
    assert np.all((out != 0) <= op.comp)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()
    # one frozen ETD2RK step of the workload
    f, _ = logistic(w.a, w.b)
    U = oracle_etd_step(op.A, w.h, op.gather(w.u0), f, "etd2rk", method="krylov")
    ud = dev(w.u0)
    st = ctx.etd_step("etd2rk", w.h, ud, stats=True)
    ug = host(ud)
    say(f"  stats {st}  u rel {rel_l2(ug[op.comp], U):.3e}")
    assert st["n_unknowns"] == op.n
    assert rel_l2(ug[op.comp], U) <= 1e-9
    ctx.close()


def test_ellipsoid192_free_boundary_step_full_size(ellipsoid):
    """The first step of the workload at 192^3 (level set, geometry, ETD2RK)
    against the oracle's, in the oracle's order (its level set over the
    whole box takes about 2 minutes of host time)."""
    import time

    w = ellipsoid
    og = ogrid(w.grid)
    ctx = ctx_for(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu)
    rd, ud = dev(w.rho0), dev(w.u0)
    ctx.geometry_build(rd)
    ctx.etd_step("etd2rk", w.h, ud, rho=rd, reinit=False)
    rg, ug = host(rd), host(ud)
    ctx.close()
    say("ellipsoid192 full step: GPU done, oracle level set (whole box)")
    t0 = time.time()
    rho1, u1, _ = oracle_levelset_advance(og, w.rho0, w.u0, w.h, w.mu, False)
    say(f"  oracle level set {time.time() - t0:.0f} s; operator and ETD2RK (Krylov route)")
    op = build_operator(og, rho1, w.beta)
    f, _ = logistic(w.a, w.b)
    U = oracle_etd_step(op.A, w.h, op.gather(u1), f, "etd2rk", method="krylov")
    say(f"  oracle step {time.time() - t0:.0f} s; N {op.n}")
    _, comp_g, _ = classify(og, rg)
    say(f"  rho diff {np.abs(rg - rho1).max():.3e}  u rel {rel_l2(ug[op.comp], U):.3e}")
    assert np.array_equal(comp_g, op.comp)
    assert np.abs(rg - rho1).max() <= 1e-10
    assert rel_l2(ug[op.comp], U) <= 1e-9
    assert np.all(ug[~op.comp] == 0.0)


def test_ellipsoid192_levelset_monotone(ellipsoid):
    w = ellipsoid
    say("ellipsoid192: full-size level-set step, V >= 0 => rho non-increasing")
    ctx = ctx_for(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu)
    rd, ud = dev(w.rho0), dev(w.u0)
    ctx.geometry_build(rd)
    ctx.levelset_advance(rd, ud, w.h, False)
    rg, ug = host(rd), host(ud)
    ctx.close()
    drho = rg - w.rho0
    say(f"  max increase {drho.max():.3e}  max decrease {-drho.min():.3e}")
    assert drho.max() <= 1e-13
    assert -drho.min() > 0.0
    assert np.all((w.rho0 < 0) <= (rg < 0))
    _, comp_new, _ = classify(ogrid(w.grid), rg)
    assert np.all(ug[~comp_new] == 0.0)


def test_levelset_advance_parity_3d():
    g = inputs.GridSpec(3, (64, 64, 64), (-4.0,) * 3, (4.0,) * 3)
    X, Y, Z = g.coords()
    rho = inputs.sdf_prolate_spheroid(X, Y, Z, 2.5, 1.8)
    u = np.where(rho < 0, 0.8 * np.clip(-rho, 0, None) * (1 + 0.1 * np.cos(2 * X)), 0.0)
    say("levelset_advance 64^3 with reinitialisation")
    rho1, u1, info = oracle_levelset_advance(ogrid(g), rho, u, 0.05, 2.0, reinit=True)
    ctx = ctx_for(g, beta=1.0, mu=2.0)
    rd, ud = dev(rho), dev(u)
    ctx.geometry_build(rd)
    ctx.levelset_advance(rd, ud, 0.05, True)
    rg, ug = host(rd), host(ud)
    ctx.close()
    say(f"  nsub {info['nsub']} max|drho| {np.abs(rg - rho1).max():.3e} max|du| {np.abs(ug - u1).max():.3e}")
    assert np.abs(rg - rho1).max() <= 1e-11
    assert np.abs(ug - u1).max() <= 1e-11
    assert np.array_equal(rg < 0, rho1 < 0)


def test_free_boundary_3d_end_to_end():
    g = inputs.GridSpec(3, (48, 48, 48), (-5.0,) * 3, (5.0,) * 3)
    X, Y, Z = g.coords()
    rho = inputs.sdf_prolate_spheroid(X, Y, Z, 2.5, 1.8)
    u = np.where(rho < 0, np.random.default_rng(0).uniform(0.2, 0.8, rho.shape), 0.0)
    say("3D free boundary 48^3, 4 ETD2RK steps, mu = 1")
    og = ogrid(g)
    ctx = ctx_for(g, beta=1.0, mu=1.0)
    rd, ud = dev(rho), dev(u)
    ctx.geometry_build(rd)
    for m in range(4):
        reinit = m == 3
        rho, u, op = free_boundary_step(og, rho, u, 0.01, 1.0, 1.0, scheme="etd2rk", reinit=reinit,
                                        method="krylov")
        ctx.etd_step("etd2rk", 0.01, ud, rho=rd, reinit=reinit)
    rg, ug = host(rd), host(ud)
    ctx.close()
    _, comp_g, _ = classify(og, rg)
    say(f"  N {op.n} rho diff {np.abs(rg - rho).max():.3e}  u rel {rel_l2(ug[op.comp], u[op.comp]):.3e}")
    assert np.array_equal(comp_g, op.comp)
    assert np.abs(rg - rho).max() <= 1e-10
    assert rel_l2(ug[op.comp], u[op.comp]) <= 1e-9
