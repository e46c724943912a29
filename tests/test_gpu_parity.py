"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bars: operator and level-set sweeps to rounding (<= 1e-12 relative / abs);
phi-combinations and ETD steps to 1e-9 relative L2 over computational
points at Krylov tolerance 1e-10; classification masks exactly equal.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import levelset as ols
from oracle.etd import etd_step as oracle_etd_step, logistic
from oracle.freeboundary import levelset_advance as oracle_levelset_advance
from oracle.geometry import Grid, classify
from oracle.operator import build_operator
from oracle.phi import phi_combination, phi_combination_at
from paper_2209_15095_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ctx_for(grid, **kw):
    from paper_2209_15095_amd.api import Context
    return Context(grid.dim, grid.n, grid.lo, grid.hi, **kw)


def ogrid(g):
    return Grid(g.dim, tuple(g.n), tuple(g.lo), tuple(g.hi))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_star2d(n=96):
    g = inputs.GridSpec(2, (n, n), (-4.0, -4.0), (4.0, 4.0))
    X, Y = g.coords()
    rho = inputs.sdf_star(X, Y, lambda t: 2.0 + 0.4 * np.cos(5 * t))
    return g, rho


def small_ellipsoid3d(n=40):
    g = inputs.GridSpec(3, (n, n, n), (-4.0,) * 3, (4.0,) * 3)
    X, Y, Z = g.coords()
    return g, inputs.sdf_prolate_spheroid(X, Y, Z, 3.0, 2.0)


@pytest.mark.parametrize("case", ["star2d", "ellipsoid3d", "fisher64"])
def test_operator_apply_parity(case):
    say(f"operator_apply {case}")
    if case == "star2d":
        g, rho = small_star2d()
    elif case == "ellipsoid3d":
        g, rho = small_ellipsoid3d()
    else:
        w = inputs.fisher64()
        g, rho = w.grid, w.rho0
    op = build_operator(ogrid(g), rho, 1.3)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(rho.shape)
    ctx = ctx_for(g, beta=1.3)
    ctx.geometry_build(dev(rho))
    out = host(ctx.operator_apply(dev(v)))
    ref = op.scatter(op.A @ op.gather(v))
    assert np.all(out[~op.comp] == 0.0)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("t", [0.01, 1.0])
def test_phi_combination_parity_fisher64(p, t):
    say(f"phi_combination fisher64 p={p} t={t}")
    w = inputs.fisher64()
    op = build_operator(ogrid(w.grid), w.rho0, 1.0)
    rng = np.random.default_rng(p)
    bs = [rng.standard_normal(w.rho0.shape) for _ in range(p + 1)]
    ref = op.scatter(phi_combination(op.A, t, [op.gather(b) for b in bs], method="dense"))
    ctx = ctx_for(w.grid, beta=1.0)
    ctx.geometry_build(dev(w.rho0))
    out, st = ctx.phi_combination_apply(t, [dev(b) for b in bs], stats=True)
    out = host(out)
    say(f"  stats {st}")
    assert np.all(out[~op.comp] == 0.0)
    assert rel_l2(out[op.comp], ref[op.comp]) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("case,t", [("fisher64", 0.05), ("star2d", 2.0), ("ellipsoid3d", 2.0)])
@pytest.mark.parametrize("p", [0, 1, 3])
def test_phi_combination_multi_parity(case, t, p):
    """phi_combination_apply_multi: the value at t and at t_mid (inside a
    substep, or at its end) from one integration, against the oracle's
    phi_combination and phi_combination_at; t = 2 takes several substeps."""
    if case == "fisher64":
        w = inputs.fisher64()
        g, rho = w.grid, w.rho0
    else:
        g, rho = small_star2d() if case == "star2d" else small_ellipsoid3d()
    op = build_operator(ogrid(g), rho, 1.0)
    rng = np.random.default_rng(8)
    bs = [rng.standard_normal(rho.shape) for _ in range(p + 1)]
    vs = [op.gather(b) for b in bs]
    method = "dense" if op.n < 2500 else "krylov"
    ctx = ctx_for(g, beta=1.0)
    ctx.geometry_build(dev(rho))
    for frac in (0.5, 0.3, 1.0):
        ref = phi_combination(op.A, t, vs, method=method)
        ref_mid = phi_combination_at(op.A, t, vs, frac * t, method=method)
        out, mid, st = ctx.phi_combination_apply_multi(t, [dev(b) for b in bs], frac * t, stats=True)
        out, mid = host(out), host(mid)
        say(f"multi {case} p {p} t_mid {frac}t: substeps {st['substeps']} out {rel_l2(out[op.comp], ref):.2e} "
            f"mid {rel_l2(mid[op.comp], ref_mid):.2e}")
        assert rel_l2(out[op.comp], ref) <= 1e-9
        assert rel_l2(mid[op.comp], ref_mid) <= 1e-9
        assert np.all(mid[~op.comp] == 0.0)
    ctx.close()


@pytest.mark.parametrize("case", ["star2d", "ellipsoid3d"])
def test_phi_combination_parity_stiff(case):
    """Large |tA| (several substeps / large m) on 2D and 3D domains."""
    say(f"phi_combination stiff {case}")
    g, rho = small_star2d() if case == "star2d" else small_ellipsoid3d()
    op = build_operator(ogrid(g), rho, 1.0)
    rng = np.random.default_rng(5)
    bs = [rng.standard_normal(rho.shape) for _ in range(3)]
    t = 2.0
    ref = op.scatter(phi_combination(op.A, t, [op.gather(b) for b in bs], method="krylov"))
    ctx = ctx_for(g, beta=1.0)
    ctx.geometry_build(dev(rho))
    out, st = ctx.phi_combination_apply(t, [dev(b) for b in bs], stats=True)
    say(f"  stats {st}")
    out = host(out)
    assert rel_l2(out[op.comp], ref[op.comp]) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("scheme", ["etd1", "etd2rk", "etd3rk", "etd4rk", "etd3rk_simul", "etd4rk_simul"])
@pytest.mark.parametrize("case", ["fisher64", "ellipsoid3d"])
def test_etd_step_frozen_parity(scheme, case):
    say(f"etd_step frozen {case} {scheme}")
    if case == "fisher64":
        w = inputs.fisher64()
        g, rho, u0 = w.grid, w.rho0, w.u0
    else:
        g, rho = small_ellipsoid3d()
        u0 = np.where(rho < 0, np.random.default_rng(0).uniform(0.2, 0.8, rho.shape), 0.0)
    op = build_operator(ogrid(g), rho, 1.0)
    f, _ = logistic(1.0, 1.0)
    h = 0.05
    U = op.gather(u0)
    ctx = ctx_for(g, beta=1.0)
    ctx.geometry_build(dev(rho))
    ud = dev(u0)
    for k in range(3):
        # the _simul variants compute the same schemes (Section 3.3 simultaneous output)
        U = oracle_etd_step(op.A, h, U, f, scheme.replace("_simul", ""), method="dense" if op.n < 2500 else "krylov")
        st = ctx.etd_step(scheme, h, ud, stats=True)
        say(f"  step {k} stats {st}")
    out = host(ud)
    assert np.all(out[~op.comp] == 0.0)
    assert rel_l2(out[op.comp], U) <= 1e-9
    ctx.close()


def test_levelset_advance_parity_2d():
    say("levelset_advance star2d")
    g, rho = small_star2d(128)
    X, Y = g.coords()
    r = np.hypot(X, Y)
    u = np.where(rho < 0, 0.8 * np.clip(-rho, 0, None) * (1 + 0.1 * np.cos(3 * X)), 0.0)
    rho1, u1, info = oracle_levelset_advance(ogrid(g), rho, u, 0.05, 2.0, reinit=True)
    ctx = ctx_for(g, beta=1.0, mu=2.0)
    rd, ud = dev(rho), dev(u)
    ctx.geometry_build(rd)
    ctx.levelset_advance(rd, ud, 0.05, True)
    rg, ug = host(rd), host(ud)
    say(f"  nsub {info['nsub']} max|drho| {np.abs(rg - rho1).max():.3e} max|du| {np.abs(ug - u1).max():.3e}")
    assert np.abs(rg - rho1).max() <= 1e-11
    assert np.abs(ug - u1).max() <= 1e-11
    assert np.array_equal(rg < 0, rho1 < 0)
    ctx.close()


@pytest.mark.parametrize("scheme", [None, "etd4rk", "etd4rk_simul"])
def test_free_boundary_fisher64_end_to_end(scheme):
    """Config fisher64 in full: 10 ETD1 steps, mu = 1, moving boundary; and
    the same run with ETD4RK steps."""
    say(f"free boundary fisher64 10 steps {scheme or 'etd1'}")
    from oracle.freeboundary import free_boundary_step
    w = inputs.fisher64()
    if scheme is not None:
        w.scheme = scheme
    og = ogrid(w.grid)
    rho, u = w.rho0.copy(), w.u0.copy()
    ctx = ctx_for(w.grid, beta=w.beta, mu=w.mu)
    rd, ud = dev(rho), dev(u)
    ctx.geometry_build(rd)
    for m in range(w.steps):
        reinit = (m + 1) % w.reinit_every == 0
        rho, u, op = free_boundary_step(og, rho, u, w.h, w.beta, w.mu, scheme=w.scheme.replace("_simul", ""),
                                        reinit=reinit, method="dense")
        ctx.etd_step(w.scheme, w.h, ud, rho=rd, reinit=reinit)
    rg, ug = host(rd), host(ud)
    _, comp_g, _ = classify(og, rg)
    assert np.array_equal(comp_g, op.comp)
    say(f"  rho diff {np.abs(rg - rho).max():.3e}  u rel {rel_l2(ug[op.comp], u[op.comp]):.3e}")
    assert np.abs(rg - rho).max() <= 1e-10
    assert rel_l2(ug[op.comp], u[op.comp]) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("case", ["fisher64", "ellipsoid3d"])
def test_etd2_multistep_frozen_parity(case):
    """ETD2 multistep (Section 3.1) on a frozen domain: an ETD2RK start,
    then three two-step updates; u and the returned F(U_n) against the
    oracle step by step."""
    say(f"etd2 multistep frozen {case}")
    from oracle.freeboundary import multistep_step
    if case == "fisher64":
        w = inputs.fisher64()
        g, rho, u0 = w.grid, w.rho0, w.u0
    else:
        g, rho = small_ellipsoid3d()
        u0 = np.where(rho < 0, np.random.default_rng(0).uniform(0.2, 0.8, rho.shape), 0.0)
    og = ogrid(g)
    ctx = ctx_for(g, beta=1.0)
    ctx.geometry_build(dev(rho))
    ud, fd = dev(u0), dev(np.full_like(u0, np.nan))
    u, fp = u0.copy(), np.zeros_like(u0)
    for k in range(4):
        _, u, fp, op = multistep_step(og, rho, u, fp, 0.05, first=(k == 0), frozen=True)
        st = ctx.multistep_step(0.05, ud, fd, first=(k == 0), stats=True)
        say(f"  step {k} stats {st}")
        ug, fg = host(ud), host(fd)
        assert np.all(ug[~op.comp] == 0.0) and np.all(fg[~op.comp] == 0.0)
        assert rel_l2(ug[op.comp], u[op.comp]) <= 1e-9
        assert rel_l2(fg[op.comp], fp[op.comp]) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("case", ["fisher64", "ellipsoid3d"])
def test_etd2_multistep_free_boundary_growing(case):
    """ETD2 multistep steps on a moving boundary (mu = 2, h = 0.05,
    reinitialisation on step 4): on the fisher64 grid and initial data the
    domain grows (164, 184, 208, 208, 216 unknowns), so F(U_{n-1}) is carried
    to the points that join it by the extrapolation that carries u; the 3D
    case (a 32^3 prolate spheroid, 3 steps) runs the same path in 3D."""
    say(f"etd2 multistep free boundary, growing domain, {case}")
    from oracle.freeboundary import multistep_step
    if case == "fisher64":
        w = inputs.fisher64()
        g, rho, u, beta, nsteps = w.grid, w.rho0.copy(), w.u0.copy(), w.beta, 5
    else:
        g, _ = small_ellipsoid3d(32)
        X, Y, Z = g.coords()
        rho = inputs.sdf_prolate_spheroid(X, Y, Z, 3.0, 2.0)
        u = np.where(rho < 0, 0.5 + 0.2 * np.cos(X) * np.cos(Y), 0.0)
        beta, nsteps = 1.0, 3
    og = ogrid(g)
    mu, h = 2.0, 0.05
    fp = np.zeros_like(u)
    ctx = ctx_for(g, beta=beta, mu=mu)
    rd, ud, fd = dev(rho), dev(u), dev(np.zeros_like(u))
    ctx.geometry_build(rd)
    ns = []
    for m in range(nsteps):
        reinit = m == 3
        rho, u, fp, op = multistep_step(og, rho, u, fp, h, beta, mu, first=(m == 0), reinit=reinit,
                                        method="dense" if case == "fisher64" else "auto")
        ns.append(op.n)
        ctx.multistep_step(h, ud, fd, first=(m == 0), rho=rd, reinit=reinit)
    rg, ug, fg = host(rd), host(ud), host(fd)
    _, comp_g, _ = classify(og, rg)
    assert np.array_equal(comp_g, op.comp)
    say(f"  unknowns {ns}  rho diff {np.abs(rg - rho).max():.3e}  "
        f"u rel {rel_l2(ug[op.comp], u[op.comp]):.3e}  f rel {rel_l2(fg[op.comp], fp[op.comp]):.3e}")
    if case == "fisher64":
        assert ns[2] > ns[1] > ns[0] and ns[4] > ns[3]   # two-step updates that meet new points
    assert np.abs(rg - rho).max() <= 1e-10
    assert rel_l2(ug[op.comp], u[op.comp]) <= 1e-9
    assert rel_l2(fg[op.comp], fp[op.comp]) <= 1e-9
    ctx.close()


def test_bitwise_deterministic():
    say("determinism")
    g, rho = small_star2d()
    u0 = np.where(rho < 0, 0.5, 0.0)
    outs = []
    for _ in range(2):
        ctx = ctx_for(g, beta=1.0, mu=1.0)
        rd, ud = dev(rho), dev(u0)
        ctx.geometry_build(rd)
        for m in range(3):
            ctx.etd_step("etd2rk", 0.01, ud, rho=rd, reinit=(m == 2))
        outs.append((host(rd), host(ud)))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_domain_error_and_no_geometry():
    say("error paths")
    from paper_2209_15095_amd._lib import EtdError, ETD_ERR_DOMAIN, ETD_ERR_NO_GEOMETRY
    g = inputs.GridSpec(2, (40, 40), (-1.0, -1.0), (1.0, 1.0))
    X, Y = g.coords()
    ctx = ctx_for(g)
    u = dev(np.zeros(X.shape))
    with pytest.raises(EtdError) as e:
        ctx.etd_step("etd1", 0.1, u)
    assert e.value.code == ETD_ERR_NO_GEOMETRY
    rho = np.hypot(X, Y) - 1.3      # covers all but the corners: computational points at layer 1
    with pytest.raises(EtdError) as e:
        ctx.geometry_build(dev(rho))
    assert e.value.code == ETD_ERR_DOMAIN
    ctx.close()


@pytest.mark.parametrize("case", ["fisher64", "ellipsoid3d"])
def test_both_krylov_builds_match_oracle(case):
    """The persistent kernels are built with 512-thread blocks (used when
    every active tile fits one loop trip of them) and 1024-thread blocks;
    each build, forced through ETDFB_KBLOCK, takes three frozen ETD2RK steps
    against the oracle (1e-9) and against the other build (1e-12)."""
    import os
    if case == "fisher64":
        w = inputs.fisher64()
        g, rho, u0 = w.grid, w.rho0, w.u0
    else:
        g, rho = small_ellipsoid3d()
        u0 = np.where(rho < 0, np.random.default_rng(4).uniform(0.2, 0.8, rho.shape), 0.0)
    op = build_operator(ogrid(g), rho, 1.0)
    f, _ = logistic(1.0, 1.0)
    h = 0.05
    U = op.gather(u0)
    for _ in range(3):
        U = oracle_etd_step(op.A, h, U, f, "etd2rk", method="dense" if op.n < 2500 else "krylov")
    outs = {}
    for kblock in (512, 1024):
        old = os.environ.get("ETDFB_KBLOCK")
        os.environ["ETDFB_KBLOCK"] = str(kblock)
        try:
            ctx = ctx_for(g, beta=1.0)
            ctx.geometry_build(dev(rho))
        finally:
            os.environ.pop("ETDFB_KBLOCK", None)
            if old is not None:
                os.environ["ETDFB_KBLOCK"] = old
        ud = dev(u0)
        for _ in range(3):
            st = ctx.etd_step("etd2rk", h, ud, stats=True)
        outs[kblock] = host(ud)
        say(f"  {case} {kblock}-thread blocks: {st}  rel {rel_l2(outs[kblock][op.comp], U):.3e}")
        ctx.close()
        assert rel_l2(outs[kblock][op.comp], U) <= 1e-9
    assert rel_l2(outs[512], outs[1024]) <= 1e-12
