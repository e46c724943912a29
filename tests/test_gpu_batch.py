"""GPU parity of the batched entry points (etd_batch_*) against the oracle.

The batch of 64 randomly perturbed stars (seeded draws: side n in
[96, 384], radius, five Fourier modes, beta in [0.5, 2]; box [-8, 8]^2,
ETD2RK h = 0.005, mu = 1) is advanced on the GPU for two free-boundary steps;
every instance is compared with the oracle run instance by instance (1e-9
relative L2 over computational points, level set to 1e-10, masks equal).  The one-block-per-instance launch (group limit 1)
must agree with the grouped launch to rounding, and a batch of one with
etd_step.  Free-boundary steps replayed from recorded graphs (launch sizes
found on the device) must match eager steps, and a front beyond the guard
must latch its error for its instance only.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.freeboundary import free_boundary_step
from oracle.geometry import Grid, classify
from paper_2209_15095_amd import inputs

pytestmark = pytest.mark.gpu

STEPS = 2


def say(msg):
    print(f"[gpu-batch] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ogrid(g):
    return Grid(g.dim, tuple(g.n), tuple(g.lo), tuple(g.hi))


def run_batch(ws, steps, group_limit=0):
    from paper_2209_15095_amd.api import Batch
    b = Batch([w.grid for w in ws], [dict(beta=w.beta, mu=w.mu) for w in ws])
    b.set_group_limit(group_limit)
    rhos = [dev(w.rho0) for w in ws]
    us = [dev(w.u0) for w in ws]
    b.geometry_build(rhos)
    for m in range(steps):
        st = b.step("etd2rk", ws[0].h, us, rhos, reinit=((m + 1) % 5 == 0 or m == steps - 1), stats=True)
    torch.cuda.synchronize()
    out = [(r.cpu().numpy(), u.cpu().numpy()) for r, u in zip(rhos, us)]
    b.close()
    return out, st


@pytest.fixture(scope="module")
def batch_result():
    ws = inputs.batch64()
    say(f"batch64: {len(ws)} instances, n in [{min(w.grid.n[0] for w in ws)}, {max(w.grid.n[0] for w in ws)}]")
    out, st = run_batch(ws, STEPS)
    say(f"  m_last per instance {[s['m_last'] for s in st][:8]} ...")
    return ws, out


def test_batch64_every_instance_matches_oracle(batch_result):
    """All 64 instances, each run by the oracle for the same free-boundary
    steps (about 1 s of host time per instance)."""
    ws, out = batch_result
    worst_u, worst_rho = 0.0, 0.0
    for i, w in enumerate(ws):
        og = ogrid(w.grid)
        rho, u = w.rho0.copy(), w.u0.copy()
        for m in range(STEPS):
            rho, u, op = free_boundary_step(og, rho, u, w.h, w.beta, w.mu, scheme="etd2rk",
                                            reinit=((m + 1) % 5 == 0 or m == STEPS - 1), method="krylov")
        rg, ug = out[i]
        _, comp_g, _ = classify(og, rg)
        du, dr = rel_l2(ug[op.comp], u[op.comp]), float(np.abs(rg - rho).max())
        worst_u, worst_rho = max(worst_u, du), max(worst_rho, dr)
        if i % 8 == 7:
            say(f"  instances 0..{i}: worst rho diff {worst_rho:.3e}, worst u rel {worst_u:.3e}")
        assert np.array_equal(comp_g, op.comp), i
        assert dr <= 1e-10, (i, dr)
        assert du <= 1e-9, (i, du)
        assert np.all(ug[~op.comp] == 0.0), i


def test_batch_single_block_groups_agree(batch_result):
    ws, out = batch_result
    say("group limit 1 (one block per instance, ordinary launch)")
    out1, _ = run_batch(ws, STEPS, group_limit=1)
    for i, ((r0, u0), (r1, u1)) in enumerate(zip(out, out1)):
        # the launches differ only in reduction order (rounding), which reaches
        # rho through the speed of the second step
        assert np.abs(r1 - r0).max() <= 1e-12, i
        assert rel_l2(u1, u0) <= 1e-10, i


def test_batch_of_one_matches_etd_step():
    from paper_2209_15095_amd.api import Context
    w = inputs.star512()
    say("batch of one vs etd_step (star512, 2 steps)")
    out, _ = run_batch([w], 2)
    ctx = Context.from_grid(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu)
    rho, u = dev(w.rho0), dev(w.u0)
    ctx.geometry_build(rho)
    for m in range(2):
        ctx.etd_step("etd2rk", w.h, u, rho=rho, reinit=(m == 1))
    torch.cuda.synchronize()
    ctx.close()
    assert np.abs(out[0][0] - rho.cpu().numpy()).max() <= 1e-12
    assert rel_l2(out[0][1], u.cpu().numpy()) <= 1e-10


def _frozen_batch(ws, limit=None, stage_min=None):
    from paper_2209_15095_amd.api import Batch
    b = Batch([w.grid for w in ws], [dict(beta=w.beta, mu=0.0) for w in ws])
    if limit is not None:
        b.set_group_limit(limit)
    if stage_min is not None:
        b.set_stage_min(stage_min)
    b.geometry_build([dev(w.rho0) for w in ws])
    return b, [dev(w.u0) for w in ws]


def test_graph_steps_replay_eager_steps():
    ws = inputs.batch64()[:12]
    h = ws[0].h
    say("graph replay: 12 frozen instances, 5 steps, eager work between replays")
    a, ua = _frozen_batch(ws)
    b, ub = _frozen_batch(ws)
    ref = []
    for k in range(5):
        a.step("etd2rk", h, ua)
        torch.cuda.synchronize()
        ref.append([u.cpu().numpy() for u in ua])
    # replays one at a time with the program's own work and synchronisations in between
    for k in range(3):
        b.graph_steps("etd2rk", h, ub, 1)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        got = [u.cpu().numpy() for u in ub]
        assert all(np.array_equal(g, r) for g, r in zip(got, ref[k])), k
        del junk
    b.graph_steps("etd2rk", h, ub, 2)
    b.sync()
    got = [u.cpu().numpy() for u in ub]
    assert all(np.array_equal(g, r) for g, r in zip(got, ref[4]))
    a.close()
    b.close()


def test_autotune_leaves_state_and_chooses_a_limit():
    ws = inputs.batch64()[:16]
    h = ws[0].h
    c, uc = _frozen_batch(ws)
    before = [u.cpu().numpy() for u in uc]
    res = c.autotune("etd2rk", h, uc, trials=2)
    say(f"autotune: {res}")
    assert res["limit"] in c.AUTOTUNE_LIMITS and res["stage_min"] in c.AUTOTUNE_STAGES
    assert len(res["ms"]) == 18 and all(ms > 0.0 for ms in res["ms"].values())
    assert res["ms"][(res["limit"], res["stage_min"])] == min(res["ms"].values())
    assert all(np.array_equal(u.cpu().numpy(), v) for u, v in zip(uc, before))
    # the tuned batch steps exactly as a fresh batch with that schedule
    d, ud = _frozen_batch(ws, limit=res["limit"], stage_min=res["stage_min"])
    for _ in range(2):
        c.step("etd2rk", h, uc)
        d.step("etd2rk", h, ud)
    torch.cuda.synchronize()
    for x, y in zip(uc, ud):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    c.close()
    d.close()


def test_batch_multistep_growing_domains_match_oracle():
    """etd_batch_multistep_step on two batch64 instances (n = 97 and 102,
    their own beta) with mu = 2, h = 0.05: an ETD2RK start and two ETD2
    multistep steps on growing domains, u, F(U_n) and rho against the
    oracle's multistep_step instance by instance."""
    from oracle.freeboundary import multistep_step
    from paper_2209_15095_amd.api import Batch
    ws = inputs.batch64()
    ws = [ws[49], ws[22]]
    mu, h, steps = 2.0, 0.05, 3
    say(f"batch multistep: instances n={[w.grid.n[0] for w in ws]}")
    b = Batch([w.grid for w in ws], [dict(beta=w.beta, mu=mu) for w in ws])
    rhos = [dev(w.rho0) for w in ws]
    us = [dev(w.u0) for w in ws]
    fs = [dev(np.full_like(w.u0, np.nan)) for w in ws]
    b.geometry_build(rhos)
    for m in range(steps):
        b.multistep_step(h, us, fs, first=(m == 0), rhos=rhos)
    torch.cuda.synchronize()
    for k, w in enumerate(ws):
        og = ogrid(w.grid)
        rho, u, fp, ns = w.rho0.copy(), w.u0.copy(), np.zeros_like(w.u0), []
        for m in range(steps):
            rho, u, fp, op = multistep_step(og, rho, u, fp, h, w.beta, mu, first=(m == 0))
            ns.append(op.n)
        rg, ug, fg = rhos[k].cpu().numpy(), us[k].cpu().numpy(), fs[k].cpu().numpy()
        _, comp_g, _ = classify(og, rg)
        say(f"  instance {k}: unknowns {ns}  rho diff {np.abs(rg - rho).max():.3e}  "
            f"u rel {rel_l2(ug[op.comp], u[op.comp]):.3e}  f rel {rel_l2(fg[op.comp], fp[op.comp]):.3e}")
        assert ns[1] > ns[0]
        assert np.array_equal(comp_g, op.comp)
        assert np.abs(rg - rho).max() <= 1e-10
        assert rel_l2(ug[op.comp], u[op.comp]) <= 1e-9
        assert rel_l2(fg[op.comp], fp[op.comp]) <= 1e-9
        assert np.all(fg[~op.comp] == 0.0)
    b.close()


@pytest.mark.parametrize("scheme", ["etd3rk", "etd4rk"])
def test_batch_higher_order_frozen_match_oracle(scheme):
    """etd_batch_step with ETD3RK / ETD4RK on three frozen batch64 instances
    (the smallest grids, their own beta), two steps of h = 0.1, against the
    oracle's etd_step instance by instance; at this step ETD3RK and ETD4RK
    differ by about 2e-6, so the tolerance tells the schemes apart.  Then the
    same steps replayed from a recorded graph agree with the eager ones bit
    for bit."""
    from oracle.etd import etd_step as oracle_etd_step, logistic
    from oracle.operator import build_operator
    ws = inputs.batch64()
    order = np.argsort([w.grid.n[0] for w in ws])[:3]
    ws = [ws[int(i)] for i in order]
    h = 0.1
    say(f"batch {scheme}: frozen instances n={[w.grid.n[0] for w in ws]}")
    b, ub = _frozen_batch(ws)
    for _ in range(2):
        b.step(scheme, h, ub)
    torch.cuda.synchronize()
    f, _ = logistic(1.0, 1.0)
    for k, w in enumerate(ws):
        op = build_operator(ogrid(w.grid), w.rho0, w.beta)
        U = op.gather(w.u0)
        for _ in range(2):
            U = oracle_etd_step(op.A, h, U, f, scheme, method="krylov")
        got = ub[k].cpu().numpy()
        say(f"  instance {k}: N={op.n} rel {rel_l2(got[op.comp], U):.3e}")
        assert np.all(got[~op.comp] == 0.0)
        assert rel_l2(got[op.comp], U) <= 1e-9
    g, ug = _frozen_batch(ws)
    g.graph_steps(scheme, h, ug, 2)
    g.sync()
    for x, y in zip(ug, ub):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    b.close()
    g.close()


def _free_batch(ws, limit=0, mu=None):
    from paper_2209_15095_amd.api import Batch
    b = Batch([w.grid for w in ws], [dict(beta=w.beta, mu=(w.mu if mu is None else mu[i]))
                                     for i, w in enumerate(ws)])
    b.set_group_limit(limit)
    rhos = [dev(w.rho0) for w in ws]
    us = [dev(w.u0) for w in ws]
    b.geometry_build(rhos)
    return b, rhos, us


def test_graph_free_steps_match_eager_steps():
    """etd_batch_graph_free_steps (level set, geometry and ETD2RK step
    recorded as graphs whose launch sizes are found on the device) against
    eager etd_batch_step on 8 batch64 instances: 10 free-boundary steps with
    reinitialisation every 5 (both recordings replayed), in two calls
    (steps 0-5, then 6-9) with an eager step on another batch and a
    synchronisation in between.  rho to 1e-12, u to 1e-10 relative L2 (the
    graph keeps the block schedule of the recording, so its reductions may
    be ordered differently), masks equal; nothing latched."""
    ws = inputs.batch64()[:8]
    h = ws[0].h
    steps = 10
    say(f"graph free steps: {len(ws)} instances, {steps} steps, reinit every 5")
    a, ra, ua = _free_batch(ws, limit=2)
    for m in range(steps):
        a.step("etd2rk", h, ua, ra, reinit=(m + 1) % 5 == 0)
    torch.cuda.synchronize()
    b, rb, ub = _free_batch(ws, limit=2)
    b.graph_free_steps("etd2rk", h, ub, rb, reinit_every=5, step0=0, nsteps=6)
    torch.cuda.synchronize()
    c, rc, uc = _free_batch(ws[:2])
    c.step("etd2rk", h, uc, rc)   # eager work of another batch between the replays
    torch.cuda.synchronize()
    b.graph_free_steps("etd2rk", h, ub, rb, reinit_every=5, step0=6, nsteps=4)
    b.sync()
    a.sync()
    for i, w in enumerate(ws):
        og = ogrid(w.grid)
        rg, ug = rb[i].cpu().numpy(), ub[i].cpu().numpy()
        re, ue = ra[i].cpu().numpy(), ua[i].cpu().numpy()
        _, cg, _ = classify(og, rg)
        _, ce, _ = classify(og, re)
        assert np.array_equal(cg, ce), i
        assert np.abs(rg - re).max() <= 1e-12, (i, np.abs(rg - re).max())
        err = rel_l2(ug[ce], ue[ce])
        assert err <= 1e-10, (i, err)
        assert np.all(ug[~cg] == 0.0)
    say("  graph steps equal the eager steps")
    # an eager step after the replays (the host re-reads the moved lists)
    b.step("etd2rk", h, ub, rb, reinit=False)
    a.step("etd2rk", h, ua, ra, reinit=False)
    torch.cuda.synchronize()
    for i in range(len(ws)):
        assert rel_l2(ub[i].cpu().numpy(), ua[i].cpu().numpy()) <= 1e-10
    for x in (a, b, c):
        x.close()


def test_graph_free_steps_front_error_latched():
    """A replayed free-boundary step whose front would move farther than the
    guard allows latches ETD_ERR_FRONT for its instance (reported by
    etd_batch_sync); the other instance of the batch matches eager steps."""
    from paper_2209_15095_amd._lib import ETD_ERR_FRONT, EtdError
    ws = inputs.batch64()[:2]
    h = ws[0].h
    b, rb, ub = _free_batch(ws, mu=[ws[0].mu, 500.0])
    b.graph_free_steps("etd2rk", h, ub, rb, reinit_every=5, step0=0, nsteps=2)
    with pytest.raises(EtdError) as ei:
        b.sync()
    assert ei.value.code == ETD_ERR_FRONT
    a, ra, ua = _free_batch(ws[:1])
    for m in range(2):
        a.step("etd2rk", h, ua, ra, reinit=False)
    torch.cuda.synchronize()
    assert np.abs(rb[0].cpu().numpy() - ra[0].cpu().numpy()).max() <= 1e-12
    assert rel_l2(ub[0].cpu().numpy(), ua[0].cpu().numpy()) <= 1e-10
    a.close()
    b.close()
