"""Python binding of libetdfb (same names as the C-ABI in include/etdfb.h).

Argument marshalling only: tensors are torch float64 CUDA (HIP) tensors in
box layout, passed by device pointer together with the current torch
stream; every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


# ETD schemes of the boundary (Section 3)
SCHEMES = {"etd1": L.ETD_SCHEME_ETD1, "etd2rk": L.ETD_SCHEME_ETD2RK, "etd3rk": L.ETD_SCHEME_ETD3RK,
           "etd4rk": L.ETD_SCHEME_ETD4RK, "etd3rk_simul": L.ETD_SCHEME_ETD3RK_SIMUL,
           "etd4rk_simul": L.ETD_SCHEME_ETD4RK_SIMUL}


class Context:
    """One etd_ctx: a grid, physics, Krylov options and device workspaces."""

    def __init__(self, dim, n, lo, hi, beta=1.0, a=1.0, b=1.0, mu=0.0, tol=1e-10, m_min=8, m_max=64,
                 m_step=4, max_substeps=64, stream=None, species=None):
        """species: None (scalar u), or (a, B) of an m-species Lotka-Volterra
        reaction f_s(u) = u_s (a[s] - sum_j B[s][j] u_j), m <= 4."""
        self.lib = L.load()
        g = L.EtdGrid()
        g.dim = dim
        for d in range(3):
            g.n[d] = int(n[d]) if d < dim else 1
            g.lo[d] = float(lo[d]) if d < dim else 0.0
            g.hi[d] = float(hi[d]) if d < dim else 1.0
        ph = L.EtdPhysics(float(beta), float(a), float(b), float(mu))
        op = L.EtdKrylovOpts(float(tol), int(m_min), int(m_max), int(m_step), int(max_substeps))
        self.dim = dim
        self.beta = float(beta)
        self.shape = tuple(reversed([int(x) for x in n[:dim]]))
        self.handle = C.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream()
        self.species = 1
        if species is None:
            L.check(self.lib.etd_ctx_create(C.byref(g), C.byref(ph), C.byref(op), C.c_void_p(s.cuda_stream),
                                            C.byref(self.handle)), "etd_ctx_create")
        else:
            sa, sb = species
            m = len(sa)
            sp = L.EtdSpecies()
            sp.m = m
            for i in range(m):
                sp.a[i] = float(sa[i])
                for j in range(m):
                    sp.b[i * L.ETD_MAX_SPECIES + j] = float(sb[i][j])
            L.check(self.lib.etd_ctx_create_species(C.byref(g), C.byref(ph), C.byref(sp), C.byref(op),
                                                    C.c_void_p(s.cuda_stream), C.byref(self.handle)),
                    "etd_ctx_create_species")
            self.species = m
        self._stream = s

    @classmethod
    def from_grid(cls, grid, **kw):
        return cls(grid.dim, grid.n, grid.lo, grid.hi, **kw)

    def _check_box(self, t: torch.Tensor, name: str):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name}: expected a float64 CUDA tensor")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor of shape {self.shape}, got {tuple(t.shape)}")

    def _sync_stream(self):
        cur = torch.cuda.current_stream()
        if cur.cuda_stream != self._stream.cuda_stream:
            self._stream = cur
            L.check(self.lib.etd_ctx_set_stream(self.handle, C.c_void_p(cur.cuda_stream)), "etd_ctx_set_stream")

    def close(self):
        if self.handle:
            self.lib.etd_ctx_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_beta(self, beta: float):
        L.check(self.lib.etd_ctx_set_beta(self.handle, float(beta)), "etd_ctx_set_beta")
        self.beta = float(beta)

    def geometry_build(self, rho: torch.Tensor):
        self._check_box(rho, "rho")
        self._sync_stream()
        L.check(self.lib.etd_geometry_build(self.handle, C.c_void_p(_ptr(rho))), "etd_geometry_build")

    def geometry_build_var(self, rho: torch.Tensor, beta_face):
        """Variable-beta geometry: beta_face[d] holds beta(x + h/2 e_d) at each node x."""
        self._check_box(rho, "rho")
        if len(beta_face) != self.dim:
            raise ValueError(f"beta_face: expected {self.dim} box tensors")
        for d, b in enumerate(beta_face):
            self._check_box(b, f"beta_face[{d}]")
        self._sync_stream()
        arr = (C.c_void_p * self.dim)(*[_ptr(b) for b in beta_face])
        L.check(self.lib.etd_geometry_build_var(self.handle, C.c_void_p(_ptr(rho)), arr), "etd_geometry_build_var")

    def boundary_taps(self):
        """(count, dim) float64 numpy array of the Dirichlet data points."""
        import numpy as np
        n = C.c_int32()
        L.check(self.lib.etd_boundary_taps(self.handle, 0, None, C.byref(n)), "etd_boundary_taps")
        pts = np.zeros((max(n.value, 1), self.dim))
        L.check(self.lib.etd_boundary_taps(self.handle, n.value, pts.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.byref(n)), "etd_boundary_taps")
        return pts[: n.value]

    def forcing_assemble(self, ub, src=None, out=None):
        """out = src + boundary forcing of the data ub (one value per tap)."""
        if ub is not None and (ub.dtype != torch.float64 or not ub.is_cuda or not ub.is_contiguous()):
            raise TypeError("ub: expected a contiguous float64 CUDA tensor")
        if src is not None:
            self._check_box(src, "src")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        self._check_box(out, "out")
        self._sync_stream()
        L.check(self.lib.etd_forcing_assemble(self.handle, C.c_void_p(_ptr(ub)) if ub is not None else None,
                                              C.c_void_p(_ptr(src)) if src is not None else None,
                                              C.c_void_p(_ptr(out))), "etd_forcing_assemble")
        return out

    def etd_step_forced(self, scheme: str, h: float, u: torch.Tensor, g, stats=False):
        """One step of u_t = A u + f(u) + G(t); g = [G(t_n), G(t_n + h/2), G(t_n + h)] (None where unused)."""
        code = SCHEMES[scheme]
        self._check_box(u, "u")
        if len(g) != 3:
            raise ValueError("g: expected [G(t_n), G(t_n + h/2), G(t_n + h)]")
        for k, t in enumerate(g):
            if t is not None:
                self._check_box(t, f"g[{k}]")
        self._sync_stream()
        arr = (C.c_void_p * 3)(*[_ptr(t) if t is not None else None for t in g])
        st = L.EtdStats() if stats else None
        L.check(self.lib.etd_step_forced(self.handle, code, float(h), C.c_void_p(_ptr(u)), arr,
                                         C.byref(st) if st is not None else None), "etd_step_forced")
        return st.as_dict() if stats else None

    def operator_apply(self, v: torch.Tensor, out=None):
        """out = A v on the current geometry."""
        self._check_box(v, "v")
        if out is None:
            out = torch.empty_like(v)
        self._check_box(out, "out")
        self._sync_stream()
        L.check(self.lib.etd_operator_apply(self.handle, C.c_void_p(_ptr(v)), C.c_void_p(_ptr(out))),
                "etd_operator_apply")
        return out

    def phi_combination_apply(self, t: float, bs, out=None, stats: bool = False):
        """out = sum_k phi_k(t A) b_k on the current geometry."""
        for i, b in enumerate(bs):
            self._check_box(b, f"b[{i}]")
        if out is None:
            out = torch.empty_like(bs[0])
        self._check_box(out, "out")
        self._sync_stream()
        arr = (C.c_void_p * len(bs))(*[_ptr(b) for b in bs])
        st = L.EtdStats() if stats else None
        L.check(self.lib.phi_combination_apply(self.handle, float(t), len(bs) - 1, arr, C.c_void_p(_ptr(out)),
                                               C.byref(st) if st is not None else None),
                "phi_combination_apply")
        return (out, st.as_dict()) if stats else out

    def phi_combination_apply_multi(self, t: float, bs, t_mid: float, out=None, out_mid=None, stats=False):
        """(out at t, out_mid at t_mid) of the combination's ODE, from one integration."""
        for i, b in enumerate(bs):
            self._check_box(b, f"b[{i}]")
        out = torch.empty_like(bs[0]) if out is None else out
        out_mid = torch.empty_like(bs[0]) if out_mid is None else out_mid
        self._check_box(out, "out")
        self._check_box(out_mid, "out_mid")
        self._sync_stream()
        arr = (C.c_void_p * len(bs))(*[_ptr(b) for b in bs])
        st = L.EtdStats() if stats else None
        L.check(self.lib.phi_combination_apply_multi(self.handle, float(t), len(bs) - 1, arr, float(t_mid),
                                                     C.c_void_p(_ptr(out_mid)), C.c_void_p(_ptr(out)),
                                                     C.byref(st) if st is not None else None),
                "phi_combination_apply_multi")
        return (out, out_mid, st.as_dict()) if stats else (out, out_mid)

    def levelset_advance(self, rho: torch.Tensor, u: torch.Tensor, dt: float, reinit: bool):
        self._check_box(rho, "rho")
        self._check_box(u, "u")
        self._sync_stream()
        L.check(self.lib.levelset_advance(self.handle, C.c_void_p(_ptr(rho)), C.c_void_p(_ptr(u)), float(dt),
                                          int(bool(reinit))), "levelset_advance")

    def etd_step(self, scheme: str, h: float, u: torch.Tensor, rho=None, reinit=False, stats=False):
        code = SCHEMES[scheme]
        self._check_box(u, "u")
        if rho is not None:
            self._check_box(rho, "rho")
        self._sync_stream()
        st = L.EtdStats() if stats else None
        L.check(self.lib.etd_step(self.handle, code, float(h), C.c_void_p(_ptr(u)),
                                  C.c_void_p(_ptr(rho)) if rho is not None else None, int(bool(reinit)),
                                  C.byref(st) if st is not None else None), "etd_step")
        return st.as_dict() if stats else None

    def etd_step_species(self, scheme: str, h: float, us, stats=False):
        """One step of the m-species system (etd_step_species); us: m box tensors, in place."""
        code = SCHEMES[scheme]
        if len(us) != self.species:
            raise ValueError(f"us: expected {self.species} tensors")
        for k, t in enumerate(us):
            self._check_box(t, f"u[{k}]")
        self._sync_stream()
        arr = (C.c_void_p * self.species)(*[_ptr(t) for t in us])
        st = L.EtdStats() if stats else None
        L.check(self.lib.etd_step_species(self.handle, code, float(h), arr, C.byref(st) if st is not None else None),
                "etd_step_species")
        return st.as_dict() if stats else None

    def multistep_step(self, h: float, u: torch.Tensor, f_prev: torch.Tensor, first: bool, rho=None,
                       reinit=False, stats=False):
        """One ETD2 multistep step (etd_multistep_step): u in place; f_prev
        holds F(U_{n-1}) on entry (ignored when first) and F(U_n) on return."""
        self._check_box(u, "u")
        self._check_box(f_prev, "f_prev")
        if rho is not None:
            self._check_box(rho, "rho")
        self._sync_stream()
        st = L.EtdStats() if stats else None
        L.check(self.lib.etd_multistep_step(self.handle, float(h), C.c_void_p(_ptr(u)), C.c_void_p(_ptr(f_prev)),
                                            int(bool(first)),
                                            C.c_void_p(_ptr(rho)) if rho is not None else None, int(bool(reinit)),
                                            C.byref(st) if st is not None else None), "etd_multistep_step")
        return st.as_dict() if stats else None

    def adjoint_step(self, h: float, u_n: torch.Tensor, gbar_np1: torch.Tensor, dbeta: torch.Tensor,
                     gbar_n=None, scheme: str = "etd2rk"):
        """gbar_n = dL/dU_n from gbar_np1 = dL/dU_{n+1}; dbeta (0-dim float64
        CUDA tensor) accumulates dL/dbeta.  Returns gbar_n."""
        code = SCHEMES[scheme]
        self._check_box(u_n, "u_n")
        self._check_box(gbar_np1, "gbar_np1")
        if gbar_n is None:
            gbar_n = torch.empty_like(gbar_np1)
        self._check_box(gbar_n, "gbar_n")
        if dbeta.dtype != torch.float64 or not dbeta.is_cuda or dbeta.numel() != 1:
            raise TypeError("dbeta: expected a one-element float64 CUDA tensor")
        self._sync_stream()
        L.check(self.lib.etd_adjoint_step(self.handle, code, float(h), C.c_void_p(_ptr(u_n)),
                                          C.c_void_p(_ptr(gbar_np1)), C.c_void_p(_ptr(gbar_n)),
                                          C.c_void_p(_ptr(dbeta))), "etd_adjoint_step")
        return gbar_n

    def profile_enable(self, on: bool = True):
        L.check(self.lib.etd_ctx_profile_enable(self.handle, int(bool(on))), "etd_ctx_profile_enable")

    def profile_read(self, reset: bool = False):
        pr = L.EtdProfile()
        L.check(self.lib.etd_ctx_profile_read(self.handle, C.byref(pr), int(bool(reset))), "etd_ctx_profile_read")
        return pr.as_dict()

    def sync(self):
        L.check(self.lib.etd_ctx_sync(self.handle), "etd_ctx_sync")

    def stats(self):
        st = L.EtdStats()
        L.check(self.lib.etd_ctx_stats(self.handle, C.byref(st)), "etd_ctx_stats")
        return st.as_dict()


def _grid_struct(dim, n, lo, hi):
    g = L.EtdGrid()
    g.dim = dim
    for d in range(3):
        g.n[d] = int(n[d]) if d < dim else 1
        g.lo[d] = float(lo[d]) if d < dim else 0.0
        g.hi[d] = float(hi[d]) if d < dim else 1.0
    return g


class Batch:
    """One etd_batch: independent instances advanced by shared launches.

    grids: list of objects with dim, n, lo, hi; phys: list of dicts with
    beta, a, b, mu (one per instance).
    """

    def __init__(self, grids, phys, tol=1e-10, m_min=8, m_max=64, m_step=4, max_substeps=64, stream=None):
        self.lib = L.load()
        n = len(grids)
        if n < 1 or len(phys) != n:
            raise ValueError("grids and phys must be non-empty lists of equal length")
        ga = (L.EtdGrid * n)(*[_grid_struct(g.dim, g.n, g.lo, g.hi) for g in grids])
        pa = (L.EtdPhysics * n)(*[L.EtdPhysics(float(p.get("beta", 1.0)), float(p.get("a", 1.0)),
                                               float(p.get("b", 1.0)), float(p.get("mu", 0.0))) for p in phys])
        op = L.EtdKrylovOpts(float(tol), int(m_min), int(m_max), int(m_step), int(max_substeps))
        self.count = n
        self.shapes = [tuple(reversed([int(x) for x in g.n[:g.dim]])) for g in grids]
        self.handle = C.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream()
        L.check(self.lib.etd_batch_create(n, ga, pa, C.byref(op), C.c_void_p(s.cuda_stream), C.byref(self.handle)),
                "etd_batch_create")
        self._stream = s

    def _ptrs(self, ts, name):
        if len(ts) != self.count:
            raise ValueError(f"{name}: expected {self.count} tensors")
        for i, t in enumerate(ts):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
                raise TypeError(f"{name}[{i}]: expected a float64 CUDA tensor")
            if tuple(t.shape) != self.shapes[i] or not t.is_contiguous():
                raise ValueError(f"{name}[{i}]: expected a contiguous tensor of shape {self.shapes[i]}")
        return (C.c_void_p * self.count)(*[_ptr(t) for t in ts])

    def _sync_stream(self):
        cur = torch.cuda.current_stream()
        if cur.cuda_stream != self._stream.cuda_stream:
            self._stream = cur
            L.check(self.lib.etd_batch_set_stream(self.handle, C.c_void_p(cur.cuda_stream)), "etd_batch_set_stream")

    def close(self):
        if self.handle:
            self.lib.etd_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_group_limit(self, max_blocks: int):
        L.check(self.lib.etd_batch_set_group_limit(self.handle, int(max_blocks)), "etd_batch_set_group_limit")

    def geometry_build(self, rhos):
        arr = self._ptrs(rhos, "rho")
        self._sync_stream()
        L.check(self.lib.etd_batch_geometry_build(self.handle, arr), "etd_batch_geometry_build")

    def step(self, scheme: str, h: float, us, rhos=None, reinit=False, stats=False):
        code = SCHEMES[scheme]
        ua = self._ptrs(us, "u")
        ra = self._ptrs(rhos, "rho") if rhos is not None else None
        self._sync_stream()
        st = (L.EtdStats * self.count)() if stats else None
        L.check(self.lib.etd_batch_step(self.handle, code, float(h), ua, ra, int(bool(reinit)), st), "etd_batch_step")
        return [x.as_dict() for x in st] if stats else None

    def multistep_step(self, h: float, us, fs, first: bool, rhos=None, reinit=False, stats=False):
        """One ETD2 multistep step of every instance (etd_batch_multistep_step):
        us in place; fs[i] holds F(U_{n-1}) on entry (ignored when first) and
        F(U_n) on return."""
        ua = self._ptrs(us, "u")
        fa = self._ptrs(fs, "f_prev")
        ra = self._ptrs(rhos, "rho") if rhos is not None else None
        self._sync_stream()
        st = (L.EtdStats * self.count)() if stats else None
        L.check(self.lib.etd_batch_multistep_step(self.handle, float(h), ua, fa, int(bool(first)), ra,
                                                  int(bool(reinit)), st), "etd_batch_multistep_step")
        return [x.as_dict() for x in st] if stats else None

    def graph_steps(self, scheme: str, h: float, us, nsteps: int = 1):
        """nsteps frozen-domain steps, each one replay of a recorded HIP graph."""
        code = SCHEMES[scheme]
        ua = self._ptrs(us, "u")
        self._sync_stream()
        L.check(self.lib.etd_batch_graph_steps(self.handle, code, float(h), ua, int(nsteps)),
                "etd_batch_graph_steps")

    def graph_free_steps(self, scheme: str, h: float, us, rhos, reinit_every: int = 0, step0: int = 0,
                         nsteps: int = 1):
        """nsteps free-boundary steps (global steps step0 .. step0 + nsteps - 1,
        reinitialising rho after every reinit_every-th), each one replay of a
        recorded HIP graph with launch sizes found on the device."""
        code = SCHEMES[scheme]
        ua = self._ptrs(us, "u")
        ra = self._ptrs(rhos, "rho")
        self._sync_stream()
        L.check(self.lib.etd_batch_graph_free_steps(self.handle, code, float(h), ua, ra, int(reinit_every),
                                                    int(step0), int(nsteps)), "etd_batch_graph_free_steps")

    def set_stage_min(self, min_tiles: int):
        L.check(self.lib.etd_batch_set_stage_min(self.handle, int(min_tiles)), "etd_batch_set_stage_min")

    AUTOTUNE_LIMITS = (1, 2, 4, 8, 16, 0)
    AUTOTUNE_STAGES = (0, 2048, 2 ** 31 - 1)

    def autotune(self, scheme: str, h: float, us, trials: int = 3):
        """Pick the group limit (blocks per instance) and the stage threshold
        (LDS-staged Lanczos passes from this many active tiles) with the
        fastest batched Krylov launch; returns {"limit": chosen, "stage_min":
        chosen, "ms": {(limit, stage_min): mean ms}}."""
        code = SCHEMES[scheme]
        ua = self._ptrs(us, "u")
        self._sync_stream()
        lim = C.c_int32()
        stg = C.c_int32()
        ms = (C.c_double * L.ETD_AUTOTUNE_CANDIDATES)()
        L.check(self.lib.etd_batch_autotune(self.handle, code, float(h), ua, int(trials), C.byref(lim),
                                            C.byref(stg), ms), "etd_batch_autotune")
        keys = [(l_, s_) for l_ in self.AUTOTUNE_LIMITS for s_ in self.AUTOTUNE_STAGES]
        return {"limit": int(lim.value), "stage_min": int(stg.value), "ms": dict(zip(keys, list(ms)))}

    def sync(self):
        L.check(self.lib.etd_batch_sync(self.handle), "etd_batch_sync")

    def stats(self, i: int):
        st = L.EtdStats()
        L.check(self.lib.etd_batch_stats(self.handle, int(i), C.byref(st)), "etd_batch_stats")
        return st.as_dict()

    def profile_enable(self, on: bool = True):
        L.check(self.lib.etd_batch_profile_enable(self.handle, int(bool(on))), "etd_batch_profile_enable")

    def profile_read(self, reset: bool = False):
        pr = L.EtdProfile()
        L.check(self.lib.etd_batch_profile_read(self.handle, C.byref(pr), int(bool(reset))), "etd_batch_profile_read")
        return pr.as_dict()


def phi_combination_apply_static(grid, beta: float, rho: torch.Tensor, t: float, bs, out: torch.Tensor,
                                 tol=1e-10, m_min=8, m_max=64, m_step=4, max_substeps=64):
    """out = sum_k phi_k(t A) b_k without a context (phi_combination_apply_static):
    no device memory is allocated by the call (out must be given)."""
    lib = L.load()
    g = _grid_struct(grid.dim, grid.n, grid.lo, grid.hi)
    shape = tuple(reversed([int(x) for x in grid.n[: grid.dim]]))
    for name, tt in [("rho", rho), ("out", out)] + [(f"b[{i}]", b) for i, b in enumerate(bs)]:
        if not isinstance(tt, torch.Tensor) or tt.dtype != torch.float64 or not tt.is_cuda:
            raise TypeError(f"{name}: expected a float64 CUDA tensor")
        if tuple(tt.shape) != shape or not tt.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor of shape {shape}")
    op = L.EtdKrylovOpts(float(tol), int(m_min), int(m_max), int(m_step), int(max_substeps))
    arr = (C.c_void_p * len(bs))(*[_ptr(b) for b in bs])
    s = torch.cuda.current_stream()
    L.check(lib.phi_combination_apply_static(C.byref(g), float(beta), C.c_void_p(_ptr(rho)), float(t), len(bs) - 1,
                                             arr, C.c_void_p(_ptr(out)), C.byref(op), C.c_void_p(s.cuda_stream)),
            "phi_combination_apply_static")
    return out


class ETDSolve(torch.autograd.Function):
    """u_T = ETD2RK^steps(u0) on a frozen domain, differentiable in u0 and beta.

    Forward keeps a checkpoint every `checkpoint_every` steps; backward
    recomputes each segment from its checkpoint and runs the discrete
    adjoint (etd_adjoint_step) step by step in reverse.  Call as
    ETDSolve.apply(u0, beta, context, h, steps, checkpoint_every) with a
    Context whose geometry is built; beta is a one-element float64 tensor.
    """

    @staticmethod
    def forward(fctx, u0, beta, context, h, steps, checkpoint_every=8):
        beta_value = float(beta.detach().reshape(-1)[0].item())
        context.set_beta(beta_value)
        u = u0.detach().clone()
        ckpt = {0: u.clone()}
        for n in range(steps):
            context.etd_step("etd2rk", h, u)
            if (n + 1) % checkpoint_every == 0 and n + 1 < steps:
                ckpt[n + 1] = u.clone()
        fctx.context, fctx.h, fctx.steps, fctx.every = context, h, steps, checkpoint_every
        fctx.ckpt = ckpt
        fctx.beta_shape = beta.shape
        fctx.beta_value = beta_value
        return u

    @staticmethod
    def backward(fctx, grad_out):
        context, h, steps, every = fctx.context, fctx.h, fctx.steps, fctx.every
        g = grad_out.detach().contiguous().clone()
        dbeta = torch.zeros(1, dtype=torch.float64, device=g.device)
        starts = sorted(fctx.ckpt)
        # the recomputation and the adjoint run at the forward's beta, whatever
        # the context was set to in between; the caller's value is restored
        beta_before = context.beta
        context.set_beta(fctx.beta_value)
        try:
            for s0 in reversed(starts):
                e = min(s0 + every, steps)
                states = [fctx.ckpt[s0].clone()]
                for n in range(s0, e - 1):
                    u = states[-1].clone()
                    context.etd_step("etd2rk", h, u)
                    states.append(u)
                for n in range(e - 1, s0 - 1, -1):
                    context.adjoint_step(h, states[n - s0], g, dbeta, gbar_n=g)
        finally:
            context.set_beta(beta_before)
        return g, dbeta.reshape(fctx.beta_shape), None, None, None, None

