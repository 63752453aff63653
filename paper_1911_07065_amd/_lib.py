"""ctypes declarations of libppgmres.so (argument marshalling only).

The library must have been built in-tree (``python -m paper_1911_07065_amd.build``
or ``__graft_entry__.build()``); importing this module without it raises
ImportError: there is no fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppgmres.so")

PP_OK, PP_NOCONV, PP_BREAKDOWN, PP_UNSTABLE = 0, 1, 2, 3
PP_EINVAL, PP_ENOMEM, PP_EDEVICE, PP_ESINGULAR = -1, -2, -3, -4
STATUS_NAMES = {0: "OK", 1: "NOCONV", 2: "BREAKDOWN", 3: "UNSTABLE", -1: "EINVAL", -2: "ENOMEM",
                -3: "EDEVICE", -4: "ESINGULAR"}

c_int, c_double, c_void_p, c_int64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64
P_int = ctypes.POINTER(ctypes.c_int)
P_double = ctypes.POINTER(ctypes.c_double)


class SetupInfo(ctypes.Structure):
    _fields_ = [("d", c_int), ("d_eff", c_int), ("n_added", c_int), ("breakdown", c_int),
                ("mvps", c_int64), ("dots", c_int64), ("t_setup_s", c_double)]


class StchOpts(ctypes.Structure):
    _fields_ = [("b", c_void_p), ("tol", c_double), ("d_step", c_int), ("d_min", c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("m", c_int), ("max_cycles", c_int), ("tol", c_double), ("inner", c_int),
                ("stall_cycles", c_int), ("inner_eta", c_double), ("history", P_double), ("history_cap", c_int),
                ("new_poly_degree", c_int), ("new_poly_add", c_int), ("graphs", c_int), ("graph_steps", c_int),
                ("lookahead", c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("cycles", c_int), ("iters", c_int), ("fp64_cycles", c_int),
                ("mvps", c_int64), ("vops", c_int64), ("dots", c_int64), ("relres", c_double),
                ("relres_shortcut", c_double), ("t_solve_s", c_double), ("lookahead_discarded", c_int)]


# name -> (restype, argtypes); must mirror include/ppgmres.h
SIGNATURES = {
    "pp_matrix_create": (c_int, [c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "pp_matrix_set_values": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pp_matrix_destroy": (None, [c_void_p]),
    "pp_matrix_tune": (c_int, [c_void_p, c_int, c_void_p, P_int, P_int, P_double]),
    "pp_matrix_set_variant": (c_int, [c_void_p, c_int, c_int, c_int]),
    "pp_matrix_variant": (c_int, [c_void_p, c_int, P_int, P_int, P_double]),
    "pp_matrix_set_pair_steps": (c_int, [c_void_p, c_int, c_int]),
    "pp_matrix_pair_steps": (c_int, [c_void_p, c_int, P_int, P_int, P_double]),
    "pp_matrix_set_march": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
    "pp_matrix_march": (c_int, [c_void_p, c_int, P_int, P_int, P_double, P_int]),
    "pp_matrix_set_march_shape": (c_int, [c_void_p, c_int, c_int]),
    "pp_launch_floor": (c_int, [c_int, c_int64, c_int, c_void_p]),
    "pp_solve_workspace_bytes": (c_int, [c_void_p, c_void_p, ctypes.POINTER(SolveOpts), ctypes.POINTER(c_int64),
                                         ctypes.POINTER(c_int64)]),
    "pp_matrix_march_shape": (c_int, [c_void_p, c_int, P_int]),
    "pp_matrix_right_scale": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pp_matrix_scale": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pp_chain_variant_name": (ctypes.c_char_p, [c_int]),
    "pp_matrix_transpose": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pp_gather": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pp_adjoint_values": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pp_gmres_setup": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, ctypes.POINTER(c_void_p),
                               ctypes.POINTER(SetupInfo)]),
    "pp_gmres_setup_basis": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, ctypes.POINTER(c_void_p),
                                     ctypes.POINTER(SetupInfo)]),
    "pp_batch_set_orth": (c_int, [c_void_p, c_int]),
    "pp_batch_orth": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "pp_gmres_setup_double": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(SetupInfo)]),
    "pp_gmres_setup_checked": (c_int, [c_void_p, c_void_p, c_int, c_int, ctypes.POINTER(StchOpts), c_void_p,
                                       ctypes.POINTER(c_void_p), ctypes.POINTER(SetupInfo), P_double]),
    "pp_poly_from_roots": (c_int, [c_int, P_double, P_double, c_int, ctypes.POINTER(c_void_p)]),
    "pp_poly_roots": (c_int, [c_void_p, c_int, c_int, P_double, P_double, P_int, P_int, P_int]),
    "pp_poly_destroy": (None, [c_void_p]),
    "pp_apply": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "pp_apply_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "pp_chain_bytes": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, ctypes.POINTER(c_int64),
                               ctypes.POINTER(c_int64)]),
    "pp_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts), c_void_p,
                         ctypes.POINTER(SolveInfo)]),
    "pp_stability_check": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, P_double]),
    "pp_batch_create": (c_int, [c_int, ctypes.POINTER(c_int64), c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                ctypes.POINTER(c_void_p)]),
    "pp_batch_set_values": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pp_batch_set_format": (c_int, [c_void_p, c_int]),
    "pp_block_jacobi_nnz": (c_int, [c_void_p, c_int, c_void_p, ctypes.POINTER(c_int64)]),
    "pp_block_jacobi": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pp_matrix_right_blocks": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "pp_batch_format": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "pp_batch_tune": (c_int, [c_void_p, c_int, c_int, c_void_p]),
    "pp_batch_set_chain_config": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "pp_batch_chain_config": (c_int, [c_void_p, c_int, c_int, P_int, P_int, P_int, P_double]),
    "pp_batch_destroy": (None, [c_void_p]),
    "pp_batch_setup": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, ctypes.POINTER(c_void_p),
                               ctypes.POINTER(SetupInfo)]),
    "pp_batch_solve": (c_int, [c_void_p, ctypes.POINTER(c_void_p), c_int, c_void_p, c_void_p,
                               ctypes.POINTER(SolveOpts), c_void_p, ctypes.POINTER(SolveInfo)]),
    "pp_harmonic_ritz": (c_int, [c_int, P_double, c_int, P_double, P_double]),
    "pp_hessenberg_eig": (c_int, [c_int, P_double, c_int, P_double, P_double]),
    "pp_leja_order": (c_int, [c_int, P_double, P_double, P_int]),
    "pp_add_roots": (c_int, [c_int, P_double, P_double, c_int, c_int, P_double, P_double, P_int, P_int,
                             P_double, P_int]),
    "pp_last_error": (ctypes.c_char_p, []),
    "pp_version": (ctypes.c_char_p, []),
}


class PPError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.pp_last_error().decode(errors="replace") if _lib is not None else ""
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1911_07065_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
lib = _lib


def check(status, where):
    """Raise PPError on a negative (error) status; return warnings unchanged."""
    if status < 0:
        raise PPError(status, where)
    return status
