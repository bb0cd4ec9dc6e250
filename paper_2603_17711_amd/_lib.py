"""ctypes binding of include/tenso.h (argument marshalling only)."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtenso.so")


class TensoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tenso error {code}: {msg}")
        self.code = code


class c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class PlanOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("method", C.c_int), ("max_rank", C.c_int)]


class VmfOpts(C.Structure):
    _fields_ = [("ode_rtol", C.c_double), ("ode_atol", C.c_double), ("vmf_atol", C.c_double),
                ("fixed_substeps", C.c_int), ("max_substeps", C.c_int)]


FP64, FP32, FP32_3M, BF16 = 0, 1, 2, 3
PS1, PS2, VMF = 0, 1, 2
DRIVE_FN = C.CFUNCTYPE(None, C.c_double, C.POINTER(C.c_double), C.c_void_p)
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENUMERIC", -5: "EUNSUPPORTED"}

_lib = None

P = C.c_void_p
I32P = C.POINTER(C.c_int32)
DP = C.POINTER(C.c_double)
C128P = C.POINTER(c128)
SIGS = {
    "tenso_last_error": (C.c_char_p, []),
    "tenso_build_tree": (C.c_int, [C.c_int, I32P, C.c_int, I32P, I32P, C.c_int, I32P, C.POINTER(P)]),
    "tenso_tree_train": (C.c_int, [C.c_int, C.c_int, I32P, C.c_int, C.POINTER(P)]),
    "tenso_tree_nary": (C.c_int, [C.c_int, C.c_int, I32P, C.c_int, C.c_int, C.POINTER(P)]),
    "tenso_tree_ranks": (C.c_int, [P, I32P]),
    "tenso_tree_n_nodes": (C.c_int, [P]),
    "tenso_tree_destroy": (None, [P]),
    "tenso_build_generator": (C.c_int, [P, C.c_int, C128P, I32P, I32P, I32P, C128P, C.POINTER(P)]),
    "tenso_gen_destroy": (None, [P]),
    "tenso_plan_create": (C.c_int, [P, P, C.POINTER(PlanOpts), C.POINTER(P)]),
    "tenso_plan_destroy": (None, [P]),
    "tenso_plan_set_graph": (C.c_int, [P, C.c_int]),
    "tenso_plan_set_tile_work": (C.c_int, [P, C.c_double]),
    "tenso_plan_sizes": (C.c_int, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "tenso_plan_shapes": (C.c_int, [P, I32P, I32P]),
    "tenso_state_init": (C.c_int, [P, C128P, P, P]),
    "tenso_state_import": (C.c_int, [P, C128P, P, P]),
    "tenso_state_export": (C.c_int, [P, P, C128P, I32P, P]),
    "tenso_apply_generator": (C.c_int, [P, P, C.c_int, DP, P, P, P]),
    "tenso_apply_generator_noalloc": (C.c_int, [P, P, C.c_int, DP, P, P]),
    "tenso_plan_query": (C.c_int, [P, P, C.POINTER(PlanOpts), C.POINTER(C.c_size_t),
                                   C.POINTER(C.c_size_t), C.POINTER(C.c_int64), DP]),
    "tenso_step_fixed": (C.c_int, [P, P, C.c_double, C.c_double, C.c_int, P, P, P]),
    "tenso_step_adaptive": (C.c_int, [P, P, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int,
                                      P, P, P]),
    "tenso_step_vmf": (C.c_int, [P, P, C.c_double, C.c_double, C.c_int, C.POINTER(VmfOpts),
                                 DRIVE_FN, P, P, P]),
    "tenso_vmf_derivative": (C.c_int, [P, P, C.c_double, DP, P, P, P]),
    "tenso_vmf_stats": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), DP]),
    "tenso_plan_set_ps2_truncation": (C.c_int, [P, C.c_double, C.c_double]),
    "tenso_step_mix": (C.c_int, [P, P, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int,
                                 C.POINTER(VmfOpts), DRIVE_FN, P, P, P, I32P]),
    "tenso_reduced_rho": (C.c_int, [P, P, C128P, DP, P, P]),
    "tenso_reduced_rho_pure": (C.c_int, [P, P, C128P, DP, P, P]),
    "tenso_rank_trajectory": (C.c_int, [P, I32P, C.c_int]),
    "tenso_svd_truncate": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, DP, P, I32P,
                                     DP, P]),
    "tenso_profile": (C.c_int, [C.c_int]),
    "tenso_profile_stats": (C.c_int, [DP, C.POINTER(C.c_int64), DP, DP]),
    "tenso_profile_records": (C.c_int, [C.c_int64, DP, DP, DP, C.POINTER(C.c_int64)]),
    "tenso_batch_create": (C.c_int, [C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(P)]),
    "tenso_batch_step": (C.c_int, [P, DP, DP, C.c_int, C.POINTER(P), P]),
    "tenso_batch_reduced_rho": (C.c_int, [P, C.POINTER(C128P), P]),
    "tenso_batch_destroy": (None, [P]),
    "tenso_batch_set_graph": (C.c_int, [P, C.c_int]),
    "tenso_batch_set_parts": (C.c_int, [P, C.c_int]),
    "tenso_batch_status": (C.c_int, [P, C.POINTER(C.c_int32)]),
    "tenso_batch_state_bytes": (C.c_int, [P, C.POINTER(C.c_size_t)]),
    "tenso_batch_autotune": (C.c_int, [P, DP, C.c_int, C.POINTER(P), P, C.c_size_t, DP, P]),
    "tenso_batch_step_record": (C.c_int, [P, DP, DP, C.c_int, C.c_int, C.POINTER(P), P, P]),
    "tenso_batch_record_bytes": (C.c_int, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "tenso_mlp_gemm": (C.c_int, [C.c_int, C.c_int, C.c_int, P, C.c_long, C.c_long, P, C.c_long,
                                 C.c_long, P, C.c_long, C.c_float, P, C.c_int, P, P]),
    "tenso_mlp_silu_bwd": (C.c_int, [P, P, P, C.c_long, P]),
    "tenso_mlp_col_sum": (C.c_int, [P, C.c_int, C.c_int, P, P]),
    "tenso_mlp_mse": (C.c_int, [P, P, C.c_long, P, P, P]),
    "tenso_mlp_adam": (C.c_int, [P, P, P, P, C.c_long, C.c_float, C.c_float, C.c_float, C.c_float,
                                 C.c_int, P]),
}


def lib():
    """Load libtenso.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        # The library must share torch's HIP runtime (same SONAME): load torch's
        # runtime into the process first so the dynamic linker reuses it.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code is not None and code < 0:
        msg = lib().tenso_last_error().decode()
        raise TensoError(f"{ERRORS.get(code, code)}", msg)
    return code
