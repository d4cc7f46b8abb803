"""ctypes loader for libmrhs.so: argument types of every exported entry point.

The library is built in-tree by ``python -m paper_2211_13719_amd.build``.
Importing this module without the built library raises ImportError: there
is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmrhs.so")

F64, F32, BF16, F16 = 0, 1, 2, 3

STATUS = {
    0: "MRHS_OK",
    1: "MRHS_ERR_INVALID_ARG",
    2: "MRHS_ERR_SHAPE",
    3: "MRHS_ERR_UNSUPPORTED",
    4: "MRHS_ERR_STATE",
    5: "MRHS_ERR_OOM",
    6: "MRHS_ERR_HIP",
    7: "MRHS_ERR_NOT_CONVERGED",
}

_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_f64 = C.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "mrhs_create": (_i32, [C.POINTER(_vp), C.POINTER(_i32), _i32, _i32, _vp]),
    "mrhs_destroy": (None, [_vp]),
    "mrhs_last_error": (C.c_char_p, [_vp]),
    "mrhs_set_stream": (_i32, [_vp, _vp]),
    "mrhs_synchronize": (_i32, [_vp]),
    "mrhs_set_gauge": (_i32, [_vp, _vp, _i32, _i32]),
    "mrhs_build_clover": (_i32, [_vp, _f64, _f64]),
    "mrhs_set_clover": (_i32, [_vp, _vp, _i32, _i32, _f64]),
    "mrhs_get_clover": (_i32, [_vp, _vp, _i32, _i32]),
    "mrhs_dwc_apply": (_i32, [_vp, _vp, _vp, _i32, _i32]),
    "mrhs_hop_apply": (_i32, [_vp, _vp, _vp, _i32, _i32]),
    "mrhs_clover_apply": (_i32, [_vp, _vp, _vp, _i32, _i32]),
    "mrhs_hop_eo_apply": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32]),
    "mrhs_clover_eo_apply": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _i32]),
    "mrhs_schur_apply": (_i32, [_vp, _vp, _vp, _i32, _i32]),
    "mrhs_dot": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32]),
    "mrhs_norm2": (_i32, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32]),
    "mrhs_multi_dot": (_i32, [_vp, _vp, C.POINTER(_vp), _i32, _vp, _i64, _i32, _i32, _i32, _i32]),
    "mrhs_multi_dot_noalloc": (_i32, [_vp, _vp, C.POINTER(_vp), _i32, _vp, _i64, _i32, _i32, _i32, _i32]),
    "mrhs_read_probe": (_i32, [_vp, _vp, _i64, _i32, _i32, _i32, _vp]),
    "mrhs_set_eo_walk": (_i32, [_vp, _i32, _vp, _i32]),
    "mrhs_get_eo_walk": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mrhs_set_f64_walk": (_i32, [_vp, _i32, _vp, _i32]),
    "mrhs_get_f64_walk": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mrhs_axpy": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32]),
    "mrhs_mg_create": (_i32, [_vp, _vp, C.POINTER(_vp)]),
    "mrhs_mg_destroy": (None, [_vp]),
    "mrhs_mg_level_info": (_i32, [_vp, _i32, C.POINTER(_i32), C.POINTER(_i32)]),
    "mrhs_mg_set_basis": (_i32, [_vp, _i32, _vp, _i32, _i32]),
    "mrhs_mg_get_basis": (_i32, [_vp, _i32, _vp, _i32, _i32]),
    "mrhs_mg_block_orthonormalise": (_i32, [_vp, _i32]),
    "mrhs_restrict": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32]),
    "mrhs_prolong": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32]),
    "mrhs_block_normalise": (_i32, [_vp, _i32, _vp, _i32, _i32, _vp]),
    "mrhs_coarse_set_blocks": (_i32, [_vp, _i32, _vp, _i32, _i32]),
    "mrhs_coarse_get_blocks": (_i32, [_vp, _i32, _vp, _i32, _i32]),
    "mrhs_mg_build_coarse": (_i32, [_vp, _i32]),
    "mrhs_coarse_apply": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32]),
    "mrhs_mg_tune": (_i32, [_vp, _vp, _i32]),
    "mrhs_mg_get_tuning": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "mrhs_mg_set_lowp_cfg": (_i32, [_vp, _i32, _i32, _i32]),
    "mrhs_coarse_mr_solve": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32, _i32]),
    "mrhs_coarse_hop_eo_apply": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32, _i32]),
    "mrhs_coarse_self_eo_apply": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32, _i32, _i32]),
    "mrhs_mg_precondition": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "mrhs_mg_setup": (_i32, [_vp, _vp]),
    "mrhs_mg_solve": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "mrhs_tune": (_i32, [_vp, C.POINTER(_i32), _i32, C.c_char_p]),
    "mrhs_get_tuning": (_i32, [_vp, _i32, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32), C.POINTER(C.c_float)]),
}


class VcycleParams(C.Structure):
    _fields_ = [("nu_pre", _i32), ("nu_post", _i32), ("coarsest_iters", _i32), ("coarse_prec", _i32),
                ("fine_eo", _i32), ("coarse_eo", _i32), ("fine_sap", _i32), ("sap_iters", _i32)]


class SetupParams(C.Structure):
    _fields_ = [("setup_iters", _i32), ("smooth_steps", _i32), ("adapt_iters", _i32), ("vc", VcycleParams)]


class SolveParams(C.Structure):
    _fields_ = [("tol", _f64), ("restart", _i32), ("max_iters", _i32), ("precondition", _i32), ("use_graph", _i32),
                ("timers", _i32), ("vc", VcycleParams), ("reorth_eta", _f64), ("krylov_prec", _i32)]


class SolveStats(C.Structure):
    _fields_ = [("nrhs", _i32), ("iters", _i32), ("cycles", _i32), ("reorth", _i32), ("converged", _i32 * 64),
                ("rel_resid", _f64 * 64), ("seconds_total", _f64), ("seconds_precond", _f64),
                ("seconds_phase", _f64 * 4)]


class MgParams(C.Structure):
    _fields_ = [("nlevels", _i32), ("block", (_i32 * 4) * 2), ("n_v", _i32 * 2)]


class MrhsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing; build it with `python -m paper_2211_13719_amd.build` "
            "(the HIP library is required, there is no CPU fallback)"
        )
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so that the streams and device memory the binding passes in belong to
    # the runtime the library calls (loaded the other way round, the process
    # can hold two runtimes and the library's may see no device)
    import torch  # noqa: F401

    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()
