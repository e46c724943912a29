"""GPU parity of the LDS-staged Lanczos pass.

The persistent kernel stages each tile and its face halo in LDS when the
problem is large (2048 active tiles or more) and a block works on several
loop trips (more active tiles than 4 per block of the grid), which happens
at the bandwidth-scale sizes.  Here the size threshold is taken to 0
(ETDFB_STAGE_MIN, read at every launch) and the block count forced down
(ETDFB_GRID, read when the geometry is built) so that small problems take
that path: phi-combinations and frozen ETD2RK steps against
the oracle at 1e-9 relative L2 (Krylov tolerance 1e-10), and the staged
launch against the one-trip launch of the same problem to 1e-12, with each
build of the persistent kernels (blocks of 512 and of 1024 threads).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.etd import etd_step as oracle_etd_step, logistic
from oracle.geometry import Grid
from oracle.operator import build_operator
from oracle.phi import phi_combination
from paper_2209_15095_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-staged] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ogrid(g):
    return Grid(g.dim, tuple(g.n), tuple(g.lo), tuple(g.hi))


@pytest.fixture(autouse=True)
def staged_from_any_size():
    """The staged pass from any size (it is used from 2048 active tiles by
    default); read by every launch."""
    old = os.environ.get("ETDFB_STAGE_MIN")
    os.environ["ETDFB_STAGE_MIN"] = "0"
    yield
    if old is None:
        os.environ.pop("ETDFB_STAGE_MIN", None)
    else:
        os.environ["ETDFB_STAGE_MIN"] = old


def ctx_with_blocks(g, rho, blocks, kblock=None, **kw):
    """A context whose persistent launches use `blocks` blocks (None:
    default) of the Krylov build with `kblock` threads per block (None: the
    library's choice); both are read when the geometry is built."""
    from paper_2209_15095_amd.api import Context
    old = {k: os.environ.pop(k, None) for k in ("ETDFB_GRID", "ETDFB_KBLOCK")}
    try:
        if blocks is not None:
            os.environ["ETDFB_GRID"] = str(blocks)
        if kblock is not None:
            os.environ["ETDFB_KBLOCK"] = str(kblock)
        ctx = Context(g.dim, g.n, g.lo, g.hi, **kw)
        ctx.geometry_build(dev(rho))
    finally:
        for k, v in old.items():
            os.environ.pop(k, None)
            if v is not None:
                os.environ[k] = v
    return ctx


def disk2d(n):
    g = inputs.GridSpec(2, (n, n), (-8.0, -8.0), (8.0, 8.0))
    X, Y = g.coords()
    return g, np.sqrt(X * X + Y * Y) - 6.5


def ellipsoid3d(n):
    g = inputs.GridSpec(3, (n, n, n), (-4.0,) * 3, (4.0,) * 3)
    X, Y, Z = g.coords()
    return g, inputs.sdf_prolate_spheroid(X, Y, Z, 3.0, 2.0)


@pytest.mark.parametrize("kblock", [512, 1024])
@pytest.mark.parametrize("blocks", [1, 3])
@pytest.mark.parametrize("case", ["disk2d", "ellipsoid3d"])
def test_staged_phi_combination_parity(case, blocks, kblock):
    if case == "disk2d":
        g, rho = disk2d(97)
    else:
        g, rho = ellipsoid3d(32)
    op = build_operator(ogrid(g), rho, 1.0)
    rng = np.random.default_rng(5)
    bs = [np.where(op.comp, rng.standard_normal(rho.shape), 0.0) for _ in range(3)]
    t = 0.2
    ref = phi_combination(op.A, t, [op.gather(b) for b in bs])
    ctx = ctx_with_blocks(g, rho, blocks, kblock)
    out, st = ctx.phi_combination_apply(t, [dev(b) for b in bs], stats=True)
    o = out.cpu().numpy()
    say(f"{case} blocks {blocks} x {kblock}: active tiles {st['n_active_tiles']} m {st['m_last']} "
        f"rel {rel_l2(o[op.comp], ref):.3e}")
    assert st["n_active_tiles"] > (kblock // 256) * blocks   # several loop trips per block
    assert np.all(o[~op.comp] == 0.0)
    assert rel_l2(o[op.comp], ref) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("kblock", [512, 1024])
def test_staged_etd2rk_steps_disk257(kblock):
    g, rho = disk2d(257)
    op = build_operator(ogrid(g), rho, 1.0)
    u0 = np.where(op.comp, np.random.default_rng(2).uniform(0.2, 0.8, rho.shape), 0.0)
    f, _ = logistic(1.0, 1.0)
    h = 0.002
    say(f"disk257: {op.n} unknowns, 2 ETD2RK steps, 8 blocks against the default launch and the oracle")
    U = op.gather(u0)
    for _ in range(2):
        U = oracle_etd_step(op.A, h, U, f, "etd2rk", method="krylov")
    outs = []
    for blocks in (8, None):
        ctx = ctx_with_blocks(g, rho, blocks, kblock)
        ud = dev(u0)
        for _ in range(2):
            st = ctx.etd_step("etd2rk", h, ud, stats=True)
        outs.append(ud.cpu().numpy())
        say(f"  blocks {blocks}: active tiles {st['n_active_tiles']} m {st['m_last']} "
            f"rel {rel_l2(outs[-1][op.comp], U):.3e}")
        ctx.close()
    assert rel_l2(outs[0][op.comp], U) <= 1e-9
    assert rel_l2(outs[1][op.comp], U) <= 1e-9
    assert rel_l2(outs[0], outs[1]) <= 1e-12


@pytest.mark.parametrize("name", ["disk4097", "sphere385"])
def test_staged_matches_one_by_one_loads_at_full_size(name):
    """The bandwidth-scale workloads in the launch bench.py times: one frozen
    ETD2RK step with the staged Lanczos passes (their default at this size)
    against the same step with the stencil loaded point by point (staging
    switched off), to 1e-10 relative L2; both also against the step's
    invariant u = 0 off the computational points."""
    from paper_2209_15095_amd.api import Context
    w = inputs.WORKLOADS[name]()
    say(f"{name}: one ETD2RK step, staged against point-by-point stencil loads")
    outs = []
    for stage_min in ("2048", str(1 << 30)):
        os.environ["ETDFB_STAGE_MIN"] = stage_min
        ctx = Context.from_grid(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu)
        ctx.geometry_build(dev(w.rho0))
        ud = dev(w.u0)
        st = ctx.etd_step(w.scheme, w.h, ud, stats=True)
        torch.cuda.synchronize()
        say(f"  stage_min {stage_min}: active tiles {st['n_active_tiles']} m {st['m_last']} "
            f"substeps {st['substeps']}")
        outs.append(ud.cpu().numpy())
        del ud
        ctx.close()
    comp = outs[1] != 0.0
    assert np.all(outs[0][~comp] == 0.0)
    rel = rel_l2(outs[0], outs[1])
    say(f"  rel L2 difference {rel:.3e}")
    assert rel <= 1e-10
