"""ctypes declarations of libetdfb (include/etdfb.h).  Argument marshalling
only; the library must be built in-tree (paper_2209_15095_amd/build.py).
Loading fails loudly when it is missing: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetdfb.so")

ETD_OK = 0
ETD_ERR_INVALID = -1
ETD_ERR_HIP = -2
ETD_ERR_NO_DEVICE = -3
ETD_ERR_KRYLOV = -4
ETD_ERR_NONFINITE = -5
ETD_ERR_DOMAIN = -6
ETD_ERR_BARRIER = -7
ETD_ERR_NO_GEOMETRY = -8
ETD_ERR_FRONT = -9

ETD_STATIC_MAX_TILES = 64
ETD_STATIC_SCRATCH_BYTES = 12 << 20

ETD_SCHEME_ETD1 = 1
ETD_SCHEME_ETD2RK = 2
ETD_SCHEME_ETD3RK = 3
ETD_SCHEME_ETD4RK = 4
ETD_SCHEME_ETD3RK_SIMUL = 5
ETD_SCHEME_ETD4RK_SIMUL = 6


class EtdGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class EtdPhysics(C.Structure):
    _fields_ = [("beta", C.c_double), ("a", C.c_double), ("b", C.c_double), ("mu", C.c_double)]


ETD_MAX_SPECIES = 4
ETD_AUTOTUNE_CANDIDATES = 18


class EtdSpecies(C.Structure):
    _fields_ = [("m", C.c_int32), ("a", C.c_double * ETD_MAX_SPECIES),
                ("b", C.c_double * (ETD_MAX_SPECIES * ETD_MAX_SPECIES))]


class EtdKrylovOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("m_min", C.c_int32), ("m_max", C.c_int32), ("m_step", C.c_int32),
                ("max_substeps", C.c_int32)]


class EtdStats(C.Structure):
    _fields_ = [("substeps", C.c_int32), ("rejected", C.c_int32), ("matvecs", C.c_int32),
                ("m_last", C.c_int32), ("expms", C.c_int32), ("n_active_tiles", C.c_int32),
                ("n_unknowns", C.c_int32), ("status", C.c_int32), ("err_est", C.c_double),
                ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EtdProfile(C.Structure):
    _fields_ = [("krylov_ms", C.c_double), ("levelset_ms", C.c_double), ("geometry_ms", C.c_double),
                ("alg_bytes", C.c_double), ("krylov_launches", C.c_int32), ("levelset_calls", C.c_int32),
                ("geometry_calls", C.c_int32), ("n_unknowns", C.c_int32),
                ("krylov_device_ms", C.c_double), ("krylov_sync_ms", C.c_double), ("krylov_expm_ms", C.c_double),
                ("krylov_pass_ms", C.c_double), ("krylov_prologue_ms", C.c_double),
                ("krylov_syncs", C.c_int32), ("krylov_expms", C.c_int32), ("krylov_gap_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); the set of symbols include/etdfb.h declares
SIGNATURES = {
    "etd_ctx_create": (C.c_int, [C.POINTER(EtdGrid), C.POINTER(EtdPhysics), C.POINTER(EtdKrylovOpts),
                                 C.c_void_p, C.POINTER(C.c_void_p)]),
    "etd_ctx_create_species": (C.c_int, [C.POINTER(EtdGrid), C.POINTER(EtdPhysics), C.POINTER(EtdSpecies),
                                         C.POINTER(EtdKrylovOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "etd_step_species": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_void_p), C.POINTER(EtdStats)]),
    "etd_ctx_destroy": (C.c_int, [C.c_void_p]),
    "etd_ctx_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "etd_ctx_set_beta": (C.c_int, [C.c_void_p, C.c_double]),
    "etd_geometry_build": (C.c_int, [C.c_void_p, C.c_void_p]),
    "etd_operator_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "etd_geometry_build_var": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "etd_boundary_taps": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "etd_forcing_assemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "etd_step_forced": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.POINTER(C.c_void_p),
                                  C.POINTER(EtdStats)]),
    "phi_combination_apply": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p,
                                        C.POINTER(EtdStats)]),
    "phi_combination_apply_multi": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.POINTER(C.c_void_p), C.c_double,
                                              C.c_void_p, C.c_void_p, C.POINTER(EtdStats)]),
    "levelset_advance": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32]),
    "etd_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_int32,
                           C.POINTER(EtdStats)]),
    "etd_multistep_step": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_int32, C.POINTER(EtdStats)]),
    "etd_adjoint_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "etd_ctx_sync": (C.c_int, [C.c_void_p]),
    "etd_ctx_stats": (C.c_int, [C.c_void_p, C.POINTER(EtdStats)]),
    "etd_ctx_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "etd_ctx_profile_read": (C.c_int, [C.c_void_p, C.POINTER(EtdProfile), C.c_int32]),
    "etd_status_string": (C.c_char_p, [C.c_int]),
    "phi_combination_apply_static": (C.c_int, [C.POINTER(EtdGrid), C.c_double, C.c_void_p, C.c_double, C.c_int32,
                                               C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(EtdKrylovOpts),
                                               C.c_void_p]),
    "etd_batch_create": (C.c_int, [C.c_int32, C.POINTER(EtdGrid), C.POINTER(EtdPhysics), C.POINTER(EtdKrylovOpts),
                                   C.c_void_p, C.POINTER(C.c_void_p)]),
    "etd_batch_destroy": (C.c_int, [C.c_void_p]),
    "etd_batch_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "etd_batch_set_group_limit": (C.c_int, [C.c_void_p, C.c_int32]),
    "etd_batch_set_stage_min": (C.c_int, [C.c_void_p, C.c_int32]),
    "etd_batch_geometry_build": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "etd_batch_multistep_step": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(EtdStats)]),
    "etd_batch_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_void_p), C.c_int32, C.POINTER(EtdStats)]),
    "etd_batch_sync": (C.c_int, [C.c_void_p]),
    "etd_batch_graph_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_void_p), C.c_int32]),
    "etd_batch_graph_free_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_void_p),
                                             C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32]),
    "etd_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_void_p), C.c_int32,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "etd_batch_stats": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(EtdStats)]),
    "etd_batch_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "etd_batch_profile_read": (C.c_int, [C.c_void_p, C.POINTER(EtdProfile), C.c_int32]),
}

_lib = None


class EtdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.etd_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")


def load(path: str = LIB_PATH):
    """Load libetdfb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libetdfb.so not built at {path}; run python -m paper_2209_15095_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, where: str):
    if code != ETD_OK:
        raise EtdError(code, where)
