"""Host-only checks of the C-ABI (no GPU needed, no compute calls):
the in-tree library loads, exports every function include/etdfb.h declares,
the Python binding declares exactly that set, and host argument checks
return ETD_ERR_INVALID before any device work."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2209_15095_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etdfb.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libetdfb.so is not built; run python -m paper_2209_15095_amd.build")
    return L.load()


def test_header_and_binding_agree():
    assert header_functions() == sorted(L.SIGNATURES)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in header_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_status_strings(lib):
    for code in range(0, -10, -1):
        s = lib.etd_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.etd_status_string(-99).decode() == "unknown status"


def test_host_argument_checks(lib):
    h = C.c_void_p()
    g = L.EtdGrid()
    g.dim = 4
    ph = L.EtdPhysics(1.0, 1.0, 1.0, 0.0)
    assert lib.etd_ctx_create(C.byref(g), C.byref(ph), None, None, C.byref(h)) == L.ETD_ERR_INVALID
    g.dim = 2
    g.n[0] = g.n[1] = 64
    g.lo[0] = g.lo[1] = -1.0
    g.hi[0] = g.hi[1] = 1.0
    bad = L.EtdPhysics(-1.0, 1.0, 1.0, 0.0)
    assert lib.etd_ctx_create(C.byref(g), C.byref(bad), None, None, C.byref(h)) == L.ETD_ERR_INVALID
    g.hi[1] = 2.0   # unequal spacing
    assert lib.etd_ctx_create(C.byref(g), C.byref(ph), None, None, C.byref(h)) == L.ETD_ERR_INVALID
    g.hi[1] = 1.0
    op = L.EtdKrylovOpts(1e-10, 8, 65, 4, 64)   # m_max above 64
    assert lib.etd_ctx_create(C.byref(g), C.byref(ph), C.byref(op), None, C.byref(h)) == L.ETD_ERR_INVALID
    assert lib.etd_ctx_create(None, C.byref(ph), None, None, C.byref(h)) == L.ETD_ERR_INVALID
    # NULL contexts
    assert lib.etd_ctx_destroy(None) == L.ETD_ERR_INVALID
    assert lib.etd_ctx_sync(None) == L.ETD_ERR_INVALID
    assert lib.etd_geometry_build(None, None) == L.ETD_ERR_INVALID
    assert lib.etd_step(None, 2, 0.1, None, None, 0, None) == L.ETD_ERR_INVALID
    assert lib.phi_combination_apply(None, 0.1, 1, None, None, None) == L.ETD_ERR_INVALID
    assert lib.levelset_advance(None, None, None, 0.1, 0) == L.ETD_ERR_INVALID
    assert lib.etd_operator_apply(None, None, None) == L.ETD_ERR_INVALID
    assert lib.etd_adjoint_step(None, 2, 0.1, None, None, None, None) == L.ETD_ERR_INVALID
    assert lib.etd_multistep_step(None, 0.1, None, None, 1, None, 0, None) == L.ETD_ERR_INVALID
    assert lib.etd_batch_multistep_step(None, 0.1, None, None, 1, None, 0, None) == L.ETD_ERR_INVALID


def test_batch_host_argument_checks(lib):
    h = C.c_void_p()
    g = (L.EtdGrid * 2)()
    for i in range(2):
        g[i].dim = 2
        g[i].n[0] = g[i].n[1] = 64
        g[i].lo[0] = g[i].lo[1] = -1.0
        g[i].hi[0] = g[i].hi[1] = 1.0
    ph = (L.EtdPhysics * 2)(L.EtdPhysics(1.0, 1.0, 1.0, 0.0), L.EtdPhysics(1.0, 1.0, 1.0, 0.0))
    assert lib.etd_batch_create(0, g, ph, None, None, C.byref(h)) == L.ETD_ERR_INVALID
    assert lib.etd_batch_create(2, None, ph, None, None, C.byref(h)) == L.ETD_ERR_INVALID
    g[1].dim = 3   # mixed dimensions
    assert lib.etd_batch_create(2, g, ph, None, None, C.byref(h)) == L.ETD_ERR_INVALID
    assert lib.etd_batch_destroy(None) == L.ETD_ERR_INVALID
    assert lib.etd_batch_sync(None) == L.ETD_ERR_INVALID
    assert lib.etd_batch_step(None, 2, 0.1, None, None, 0, None) == L.ETD_ERR_INVALID
    assert lib.etd_batch_geometry_build(None, None) == L.ETD_ERR_INVALID
    assert lib.etd_batch_set_group_limit(None, 1) == L.ETD_ERR_INVALID
    assert lib.etd_batch_graph_steps(None, 2, 0.1, None, 1) == L.ETD_ERR_INVALID
    assert lib.etd_batch_autotune(None, 2, 0.1, None, 1, None, None, None) == L.ETD_ERR_INVALID
    assert lib.etd_batch_set_stage_min(None, 0) == L.ETD_ERR_INVALID
    assert lib.etd_batch_graph_free_steps(None, 2, 0.1, None, None, 5, 0, 1) == L.ETD_ERR_INVALID
