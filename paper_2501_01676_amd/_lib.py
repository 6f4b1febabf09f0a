"""ctypes binding of libabddc_hip.so (argument marshalling only).

The C ABI is declared in include/abddc.h; every structure below mirrors it
field by field.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabddc_hip.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, ESINGULAR, EEIG, EDEVICE, ESTATE = 0, 1, -1, -2, -3, -4, -5, -6

STAGE_SCHUR, STAGE_LOCAL_RHS, STAGE_FACE_EIG, STAGE_EDGE_EIG = 0, 1, 2, 3
STAGE_FACE_BASIS, STAGE_EDGE_BASIS, STAGE_COUNTS, STAGE_DELUXE = 4, 5, 6, 7
MLP_FEATURES, MLP_OUTPUTS, MLP_PARAMS = 133, 28, 37276


# abddc_device allocation hooks: void* alloc(size_t bytes, void* user),
# void free(void* p, void* user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Device(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("user", C.c_void_p)]


class Problem(C.Structure):
    _fields_ = [
        ("nsub", C.c_int32 * 3),
        ("width", C.POINTER(C.c_int32) * 3),
        ("length", C.c_double * 3),
        ("nu", C.POINTER(C.c_double)),
        ("beta0", C.c_double * 3),
        ("beta1", C.c_double * 9),
        ("c", C.c_double),
        ("f_nodal", C.POINTER(C.c_double)),
        ("f_const", C.c_double),
        ("tau", C.c_double),
        ("arrays_on_device", C.c_int32),
        ("element", C.c_int32),
        ("origin", C.c_double * 3),
        ("a_nodal", C.POINTER(C.c_double)),
        ("u_dirichlet", C.POINTER(C.c_double)),
        ("part", C.POINTER(C.c_int32)),
        ("n_parts", C.c_int32),
    ]


class Options(C.Structure):
    _fields_ = [
        ("theta_face", C.c_double),
        ("theta_edge", C.c_double),
        ("edge_variant", C.c_int32),
        ("edge_h_mode", C.c_int32),
        ("deluxe_source", C.c_int32),
        ("pinv_rtol", C.c_double),
        ("svd_rtol", C.c_double),
        ("tie_rtol", C.c_double),
        ("precision", C.c_int32),
        ("constraint_source", C.c_int32),
        ("mlp", C.c_void_p),
        ("judge_iters", C.c_int32),
        ("judge_ratio", C.c_double),
    ]


class Counts(C.Structure):
    _fields_ = [("n_vertex", C.c_int32), ("pnum_face", C.c_int32), ("pnum_edge", C.c_int32),
                ("n_primal", C.c_int32), ("n_near_ties", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("relres_true", C.c_double),
                ("t_setup_s", C.c_double), ("t_iter_s", C.c_double),
                ("resid_history", C.POINTER(C.c_double)), ("resid_cap", C.c_int32),
                ("redone", C.c_int32), ("first_iters", C.c_int32)]


_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_I32P = C.POINTER(C.c_int32)

SIGNATURES = {
    "abddc_assemble": (C.c_int, [C.POINTER(Problem), C.POINTER(Device), C.POINTER(_P)]),
    "abddc_setup_coarse_space": (C.c_int, [_P, C.POINTER(Options), C.POINTER(Counts)]),
    "abddc_apply_bddc": (C.c_int, [_P, _P, _P]),
    "abddc_apply_bddc_noalloc": (C.c_int, [_P, _P, _P]),
    "abddc_cache_stats": (C.c_int, [C.c_int32, _I64P, _I64P]),
    "abddc_apply_schur": (C.c_int, [_P, _P, _P]),
    "abddc_get_rhs": (C.c_int, [_P, _P]),
    "abddc_gmres_solve": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int32, _P, C.POINTER(SolveInfo)]),
    "abddc_query": (C.c_int, [_P, _I64P, _I64P, _I32P, _I32P, _I32P]),
    "abddc_get_stage": (C.c_int64, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int64]),
    "abddc_phase_times": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int32]),
    "abddc_kernel_stats": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_double), _I64P, C.POINTER(C.c_double)]),
    "abddc_set_kernel_stats": (C.c_uint32, [C.c_uint32]),
    "abddc_destroy": (None, [_P]),
    "abddc_last_error": (C.c_char_p, []),
    "abddc_mlp_create": (C.c_int, [C.POINTER(C.c_float), C.c_int32, C.POINTER(Device), C.POINTER(_P)]),
    "abddc_mlp_get_params": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int32]),
    "abddc_mlp_forward": (C.c_int, [_P, _P, C.c_int32, _P]),
    "abddc_mlp_loss_grad": (C.c_int, [_P, _P, _P, C.c_int32, _P, C.POINTER(C.c_float)]),
    "abddc_mlp_train_step": (C.c_int, [_P, _P, _P, C.c_int32, C.c_float, C.POINTER(C.c_float)]),
    "abddc_mlp_set_ranges": (C.c_int, [_P, _P, C.c_int32]),
    "abddc_mlp_destroy": (None, [_P]),
    "abddc_edge_features": (C.c_int, [_P, _P, _P]),
    "abddc_edge_projectors": (C.c_int, [_P, _P]),
    "abddc_learned_stats": (C.c_int, [_P, _I32P, _I32P]),
    "abddc_test_partial_lu": (C.c_int, [C.c_int32, _P, _I64P, _I32P, _I32P, _I32P, _I32P, C.c_int32, _P]),
    "abddc_test_gemm": (C.c_int, [C.c_int32, _P, _I64P, _I64P, _I64P, _I32P, _I32P, _I32P, _I32P, _I32P,
                                  _I32P, C.c_int32, C.c_int32, C.c_double, C.c_double, _P]),
    "abddc_test_sygv": (C.c_int, [C.c_int32, _P, _I64P, _I64P, _I64P, _I64P, _I32P, _P]),
    "abddc_test_sygv_select": (C.c_int, [C.c_int32, _P, _I64P, _I64P, _I64P, _I64P, _I32P, C.c_double, _P]),
    "abddc_test_schur_pinv": (C.c_int, [C.c_int32, _P, _I64P, _I32P, _I32P, C.c_double, _P]),
    "abddc_test_parallel_sum": (C.c_int, [C.c_int32, _P, _I64P, _I64P, _I64P, _I32P, C.c_double, _P]),
}

_lib = None


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run paper_2501_01676_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AbddcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"abddc error {code}: {msg}")
        self.code = code


def check(rc):
    if rc < 0:
        raise AbddcError(rc, load().abddc_last_error().decode())
    return rc


def i64(seq):
    return (C.c_int64 * len(seq))(*[int(v) for v in seq])


def i32(seq):
    return (C.c_int32 * len(seq))(*[int(v) for v in seq])
