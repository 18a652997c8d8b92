"""ctypes declarations of the C ABI in include/itn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libitn.so")

# itn_status
ITN_OK = 0
STATUS_NAMES = {
    0: "ITN_OK", 1: "ITN_E_ARG", 2: "ITN_E_SHAPE", 3: "ITN_E_LABEL", 4: "ITN_E_ARROW",
    5: "ITN_E_FLUX", 6: "ITN_E_DTYPE", 7: "ITN_E_WORKSPACE", 8: "ITN_E_HIP",
    9: "ITN_E_NOT_CONVERGED", 10: "ITN_E_UNSUPPORTED", 11: "ITN_E_NODEVICE",
}
ITN_F64, ITN_F32, ITN_BF16 = 0, 1, 2
ITN_P_F64, ITN_P_F32, ITN_P_BF16 = 0, 1, 2
ITN_LEFT, ITN_RIGHT = 0, 1
ITN_OP_CONTRACT, ITN_OP_HEFF, ITN_OP_ENV_UPDATE = 0, 1, 2


class itn_space(C.Structure):
    _fields_ = [("nsec", C.c_int32), ("nq", C.c_int32), ("qn", C.POINTER(C.c_int32)),
                ("dim", C.POINTER(C.c_int32)), ("arrow", C.c_int8), ("mod", C.POINTER(C.c_int32))]


class itn_tensor(C.Structure):
    _fields_ = [("rank", C.c_int32), ("dims", C.POINTER(C.c_int64)),
                ("label", C.POINTER(C.c_int32)), ("space", C.POINTER(itn_space)),
                ("dtype", C.c_int), ("data", C.c_void_p), ("nblocks", C.c_int64),
                ("block_sec", C.POINTER(C.c_int32)), ("block_off", C.POINTER(C.c_int64)),
                ("flux", C.POINTER(C.c_int32))]


class itn_plan_info(C.Structure):
    _fields_ = [("out_nblocks", C.c_int64), ("out_elems", C.c_int64),
                ("n_pairs_stage1", C.c_int64), ("n_groups_stage1", C.c_int64),
                ("n_pairs_stage4", C.c_int64), ("n_tiles", C.c_int64), ("flops", C.c_double),
                ("x_elems", C.c_int64), ("z_elems", C.c_int64), ("flops_wstage", C.c_double),
                ("mode_stage1", C.c_int32), ("mode_stage4", C.c_int32), ("wstage_tile", C.c_int32),
                ("flops_stage1", C.c_double)]


class itn_sweep_params(C.Structure):
    _fields_ = [("nsweeps", C.c_int32), ("maxdim", C.POINTER(C.c_int32)),
                ("cutoff", C.POINTER(C.c_double)), ("mindim", C.c_int32),
                ("krylovdim", C.c_int32), ("maxiter", C.c_int32), ("eig_tol", C.c_double),
                ("prec", C.c_int), ("refine", C.c_int32), ("energy_tol", C.c_double),
                ("timing", C.c_int32), ("northo", C.c_int32), ("ortho", C.POINTER(C.c_void_p)),
                ("weight", C.c_double), ("block", C.c_int32)]


class itn_sweep_result(C.Structure):
    _fields_ = [("sweeps_done", C.c_int32), ("energy", C.POINTER(C.c_double)),
                ("max_trunc", C.POINTER(C.c_double)), ("max_bond", C.POINTER(C.c_int32)),
                ("seconds", C.POINTER(C.c_double)), ("matvecs", C.POINTER(C.c_int64)),
                ("residual", C.POINTER(C.c_double)), ("t_matvec", C.POINTER(C.c_double)),
                ("t_solver", C.POINTER(C.c_double)), ("t_split", C.POINTER(C.c_double)),
                ("t_env", C.POINTER(C.c_double)), ("matvecs_f64", C.POINTER(C.c_int64))]


P = C.c_void_p
T = C.POINTER(itn_tensor)
S = C.c_int  # itn_status

# name -> (restype, argtypes); every symbol declared in include/itn.h
SIGNATURES = {
    "itn_create": (S, [C.POINTER(P), C.c_int]),
    "itn_destroy": (S, [P]),
    "itn_last_error": (C.c_char_p, [P]),
    "itn_sync": (S, [P, P]),
    "itn_version": (C.c_char_p, []),
    "itn_profile_enable": (S, [P, C.c_int32]),
    "itn_profile_report": (S, [P, C.c_int32, C.c_char_p, C.POINTER(C.c_double),
                               C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "itn_cast": (S, [P, T, T, P]),
    "itn_contract": (S, [P, T, T, T, C.c_int, P]),
    "itn_heff_apply": (S, [P, T, T, T, T, T, C.c_int32, T, C.c_int, P]),
    "itn_heff_apply_sum": (S, [P, C.c_int32, P, P, P, P, T, C.c_int32, T, C.c_int, P]),
    "itn_heff_apply_noalloc": (S, [P, T, T, T, T, T, C.c_int32, T, C.c_int, P]),
    "itn_heff_noalloc_max_bytes": (S, [C.POINTER(C.c_size_t)]),
    "itn_workspace_size": (S, [P, C.c_int, C.c_int32, C.POINTER(T), C.c_int32, C.c_int32, C.c_int,
                               C.POINTER(C.c_size_t)]),
    "itn_set_workspace": (S, [P, P, C.c_size_t]),
    "itn_heff_workspace_size": (S, [P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int, C.POINTER(C.c_size_t)]),
    "itn_qn_heff_plan": (S, [P, T, T, T, T, T, C.c_int32, C.c_int, C.POINTER(P)]),
    "itn_plan_destroy": (S, [P]),
    "itn_qn_allowed_blocks": (S, [P, T, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "itn_plan_query": (S, [P, C.POINTER(itn_plan_info)]),
    "itn_plan_out_blocks": (S, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "itn_qn_heff_apply": (S, [P, P, T, T, T, T, P]),
    "itn_qn_prepare_env": (S, [P, P, T, T, P]),
    "itn_qn_heff_diag": (S, [P, T, T, T, T, T, P]),
    "itn_env_update": (S, [P, T, T, T, C.c_int, T, C.c_int, P]),
    "itn_mpo_create": (S, [P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                           C.POINTER(P)]),
    "itn_mpo_destroy": (S, [P]),
    "itn_mps_create": (S, [P, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                           C.POINTER(C.c_double), C.POINTER(P)]),
    "itn_mps_destroy": (S, [P]),
    "itn_mps_bonds": (S, [P, C.POINTER(C.c_int32)]),
    "itn_mps_get_site": (S, [P, P, C.c_int32, C.POINTER(C.c_double)]),
    "itn_dmrg_sweep": (S, [P, P, P, C.POINTER(itn_sweep_params), C.POINTER(itn_sweep_result)]),
    "itn_qn_mps_create": (S, [P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(P)]),
    "itn_qn_mps_destroy": (S, [P]),
    "itn_qn_mps_bonds": (S, [P, C.POINTER(C.c_int32)]),
    "itn_qn_mps_link": (S, [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                            C.POINTER(C.c_int32)]),
    "itn_qn_mps_get_site": (S, [P, P, C.c_int32, C.POINTER(C.c_double)]),
    "itn_qn_dmrg_sweep": (S, [P, P, P, C.POINTER(C.c_int32), C.POINTER(itn_sweep_params),
                              C.POINTER(itn_sweep_result)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libitn.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            "libitn.so not found at %s: build it with `python -m paper_2007_14822_amd.build` "
            "(there is no CPU fallback)" % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
