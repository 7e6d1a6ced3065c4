"""ctypes declarations of the C ABI in include/biot_pint.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbiot_pint.so")

BIOT_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EDIVERGED", -5: "ENOTCONVERGED", -6: "ESTATE"}
SCHED = {"jacobi": 0, "wavefront": 1}
PRECOND = {"P1": 1, "P2": 2}
PRECISION = {"fp64": 0, "mixed": 1}
INNER = {"richardson": 0, "gmres": 1}
PROBES = ["residual", "cheb_u", "cheb_p", "levres_u", "levres_p", "pstage", "post_u", "post_p"]
PROBE_STRIDE_SHIFT = 16  # BIOT_PROBE_STRIDE_SHIFT: bits of the probe mask holding the wave stride

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int32), ("n_elems", C.c_int32),
                ("grid_n", C.c_int32), ("xyz", _dp), ("conn", _ip), ("dirichlet", _up)]


class Materials(C.Structure):
    _fields_ = [("young", _dp), ("poisson", _dp), ("perm", _dp), ("beta", _dp),
                ("alpha", C.c_double), ("stab_h", C.c_double), ("lame_lambda", _dp),
                ("lame_mu", _dp)]


class Load(C.Structure):
    _fields_ = [("n_facets", C.c_int32), ("facet_nodes", _ip), ("traction", _dp), ("coef", _dp),
                ("n_terms", C.c_int32), ("terms", _dp), ("term_coef", _dp),
                ("n_prescribed", C.c_int32), ("prescribed", _dp), ("prescribed_coef", _dp),
                ("x0", _dp)]


class Options(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("depth", C.c_int32), ("precond", C.c_int32),
                ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
                ("lmax_safety", C.c_double), ("power_iters", C.c_int32),
                ("max_batch", C.c_int32), ("omega", C.c_double), ("wg_per_cu", C.c_int32),
                ("coarse_cells", C.c_int32), ("use_graph", C.c_int32),
                ("precision", C.c_int32), ("adjoint", C.c_int32), ("ckpt_stride", C.c_int32),
                ("replay_segments", C.c_int32), ("max_sensors", C.c_int32),
                ("inner", C.c_int32), ("gmres_k", C.c_int32),
                ("fuse_post", C.c_int32)]


class Objective(C.Structure):
    _fields_ = [("n_sensors", C.c_int32), ("nodes", _ip), ("p_obs", _dp)]


class AdjointStats(C.Structure):
    _fields_ = [("J", C.c_double), ("adjoint_sweeps", C.c_int32), ("replay_sweeps", C.c_int32),
                ("replay_groups", C.c_int32), ("adjoint_rel_resid", C.c_double),
                ("replay_rel_resid", C.c_double), ("seconds_adjoint", C.c_double),
                ("seconds_replay", C.c_double), ("seconds", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("converged", C.c_int32), ("rel_resid_u", C.c_double),
                ("rel_resid_p", C.c_double), ("seconds", C.c_double), ("alg_bytes", C.c_double)]


class Info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int32), ("n_steps", C.c_int32),
                ("n_levels", C.c_int32), ("level_cells", C.c_int32 * 16),
                ("level_nodes", C.c_int32 * 16), ("slots", C.c_int32),
                ("lmax_A", C.c_double * 16), ("lmax_S", C.c_double * 16),
                ("workspace_bytes", C.c_uint64), ("n_samples", C.c_int32),
                ("nodes_per_sample", C.c_int32)]


# name -> (restype, argtypes)
SIGNATURES = {
    "biot_default_options": (C.c_int, [C.POINTER(Options)]),
    "biot_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Materials), C.POINTER(Load), C.c_double,
                              C.c_int32, C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "biot_create_batch": (C.c_int, [C.POINTER(Mesh), C.c_int32, C.POINTER(Materials),
                                    C.POINTER(Load), _dp, _ip, C.POINTER(Options),
                                    C.POINTER(C.c_void_p)]),
    "biot_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "biot_sample_layout": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]),
    "biot_bind": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]),
    "biot_reset": (C.c_int, [C.c_void_p]),
    "biot_sweep": (C.c_int, [C.c_void_p, C.c_int32]),
    "biot_residual_norms": (C.c_int, [C.c_void_p, _dp]),
    "biot_solve_to_tol": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_int32, C.POINTER(Stats)]),
    "biot_get_trajectory": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32]),
    "biot_set_trajectory": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32]),
    "biot_get_sample_trajectory": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                             C.c_void_p, C.c_int32]),
    "biot_apply_operator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "biot_apply_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "biot_apply_precond_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "biot_get_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "biot_export_level": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "biot_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "biot_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_char_p)]),
    "biot_objective_value": (C.c_int, [C.c_void_p, C.POINTER(Objective), C.POINTER(C.c_double)]),
    "biot_adjoint": (C.c_int, [C.c_void_p, C.POINTER(Objective), C.c_double, C.c_int32,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                               C.POINTER(AdjointStats)]),
    "biot_get_adjoint": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32]),
    "biot_last_error": (C.c_char_p, [C.c_void_p]),
    "biot_version": (C.c_char_p, []),
    "biot_destroy": (None, [C.c_void_p]),
}

_LIB = None


def load():
    """Load libbiot_pint.so from the package directory; raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python __graft_entry__.py` "
                           "(build()) to compile the HIP library")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class BiotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(lib, rc, handle=None):
    if rc != BIOT_OK:
        msg = lib.biot_last_error(handle)
        raise BiotError(rc, msg.decode() if msg else "")
    return rc


def dptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def iptr(a):
    return a.ctypes.data_as(_ip)


def uptr(a):
    return a.ctypes.data_as(_up)
