"""The allocation-free entry point phi_combination_apply_static against
phi_combination_apply on a context (the same operator and combination,
eq. 3.7): two calls in a row through the C-ABI, the second on a smaller grid
(the shared static array keeps the first call's contents), then a 3D call;
and a grid over the size limit refused before any device work."""
import ctypes as C
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_15095_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def case(grid, rho, beta, t, p, seed):
    from paper_2209_15095_amd.api import Context, phi_combination_apply_static
    rng = np.random.default_rng(seed)
    bs = [dev(rng.standard_normal(rho.shape)) for _ in range(p + 1)]
    rd = dev(rho)
    ctx = Context(grid.dim, grid.n, grid.lo, grid.hi, beta=beta)
    ctx.geometry_build(rd)
    ref = ctx.phi_combination_apply(t, bs).cpu().numpy()
    ctx.close()
    out = torch.full_like(rd, 7.0)
    phi_combination_apply_static(grid, beta, rd, t, bs, out)
    got = out.cpu().numpy()
    comp = ref != 0
    say(f"grid {grid.n[:grid.dim]} p {p}: rel {rel_l2(got[comp], ref[comp]):.2e}, "
        f"off-domain max {np.abs(got[~comp]).max():.1e}")
    assert rel_l2(got[comp], ref[comp]) <= 1e-9
    assert np.all(got[~comp] == 0.0)


def test_static_entry_matches_context_entry():
    w = inputs.fisher64()
    case(w.grid, w.rho0, 1.0, 0.05, 2, 1)
    g = inputs.GridSpec(2, (40, 40), (-5.0, -5.0), (5.0, 5.0))
    X, Y = g.coords()
    case(g, np.hypot(X, Y) - 3.0, 1.3, 0.02, 1, 2)
    g3 = inputs.GridSpec(3, (20, 20, 20), (-3.0,) * 3, (3.0,) * 3)
    X, Y, Z = g3.coords()
    case(g3, inputs.sdf_prolate_spheroid(X, Y, Z, 2.0, 1.5), 0.8, 0.03, 3, 3)


def test_static_entry_refuses_grids_over_the_limit():
    from paper_2209_15095_amd import _lib as L
    from paper_2209_15095_amd.api import _grid_struct
    lib = L.load()
    g = _grid_struct(2, (512, 512), (-1.0, -1.0), (1.0, 1.0))
    one = torch.zeros((512, 512), dtype=torch.float64, device="cuda")
    arr = (C.c_void_p * 1)(one.data_ptr())
    out = torch.zeros_like(one)
    r = lib.phi_combination_apply_static(C.byref(g), 1.0, C.c_void_p(one.data_ptr()), 0.1, 0, arr,
                                         C.c_void_p(out.data_ptr()), None, None)
    assert r == L.ETD_ERR_INVALID
