"""ctypes declarations of the C-ABI in include/ckkt.h.

Loading fails loudly when libckkt.so has not been built: there is no
fallback implementation of any entry point.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libckkt.so")

CKKT_OK = 0
MLP_F, MLP_H = 8, 64
MLP_NPARAM = MLP_H * MLP_F + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1
MLP_NOALLOC_MAX_ROWS = 32768
MAX_DEVICE_REFINE = 8
STATUS_NAMES = {0: "OK", -1: "ERR_ARG", -2: "ERR_PATTERN", -3: "ERR_NOT_SPD", -4: "ERR_NO_CONVERGENCE",
                -5: "ERR_BREAKDOWN", -6: "ERR_STATE", -7: "ERR_HIP", -8: "ERR_WORKSPACE", -9: "ERR_NONFINITE",
                -10: "ERR_TIMEOUT", -11: "ERR_HOST_MEMORY"}
LIFTED, HYKKT = 0, 1
FP64, FP32_IR = 0, 1
ORDER_AMD, ORDER_NATURAL = 0, 1

P_i32 = POINTER(c_int32)
P_f64 = POINTER(c_double)


class Pattern(ctypes.Structure):
    _fields_ = [("n", c_int64), ("m_eq", c_int64), ("m_ineq", c_int64),
                ("w_ptr", P_i32), ("w_idx", P_i32), ("g_ptr", P_i32), ("g_idx", P_i32),
                ("h_ptr", P_i32), ("h_idx", P_i32), ("formulation", c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("ordering", c_int32), ("tol", c_double), ("ir_maxit", c_int32),
                ("cg_tol", c_double), ("cg_maxit", c_int32), ("relax", c_int32), ("lds_front_max", c_int32),
                ("learned", c_int32), ("dense_row_min", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n", c_int64), ("m_eq", c_int64), ("m_ineq", c_int64), ("nnz_k", c_int64),
                ("nnz_l", c_int64), ("nnz_l_stored", c_int64), ("factor_flops", c_double),
                ("assembly_products", c_double), ("n_supernodes", c_int32), ("n_levels", c_int32),
                ("max_front", c_int32), ("n_big_fronts", c_int32), ("workspace_bytes", c_int64),
                ("analyze_seconds", c_double), ("failed_column", c_int32), ("n_dense_rows", c_int32),
                ("n_instances", c_int32), ("pad", c_int32), ("order_seconds", c_double),
                ("symbolic_seconds", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", c_int32), ("refine_steps", c_int32), ("cg_iters", c_int32), ("pcg_iters", c_int32),
                ("fallback", c_int32), ("pad", c_int32), ("omega", c_double), ("rho", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Inertia(ctypes.Structure):
    _fields_ = [("delta_w_min", c_double), ("delta_w_0", c_double), ("delta_w_max", c_double),
                ("kappa_minus", c_double), ("kappa_plus", c_double), ("kappa_plus_bar", c_double),
                ("delta_w_last", c_double), ("delta_w", c_double), ("attempts", c_int32), ("pad", c_int32)]


# (name, restype, argtypes): every entry point declared in include/ckkt.h
SIGNATURES = [
    ("ckkt_default_options", None, [POINTER(Options)]),
    ("ckkt_analyze", c_int32, [POINTER(Pattern), POINTER(Options), POINTER(c_void_p), POINTER(c_size_t)]),
    ("ckkt_batch_analyze", c_int32, [c_int32, POINTER(Pattern), POINTER(Options), POINTER(c_void_p),
                                     POINTER(c_size_t)]),
    ("ckkt_analyze_device", c_int32, [POINTER(Pattern), POINTER(Options), c_void_p, POINTER(c_void_p),
                                      POINTER(c_size_t)]),
    ("ckkt_batch_analyze_device", c_int32, [c_int32, POINTER(Pattern), POINTER(Options), c_void_p,
                                            POINTER(c_void_p), POINTER(c_size_t)]),
    ("ckkt_plan_size", c_int32, [c_void_p, POINTER(c_size_t)]),
    ("ckkt_plan_save", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("ckkt_plan_load", c_int32, [c_void_p, c_size_t, POINTER(Options), POINTER(c_void_p), POINTER(c_size_t)]),
    ("ckkt_bind_workspace", c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    ("ckkt_factorize", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p]),
    ("ckkt_factor_status", c_int32, [c_void_p, c_void_p]),
    ("ckkt_factorize_dual_reg", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                          c_void_p]),
    ("ckkt_default_inertia", None, [POINTER(Inertia)]),
    ("ckkt_factorize_inertia", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                         POINTER(Inertia), c_void_p]),
    ("ckkt_solve", c_int32, [c_void_p, c_void_p, c_void_p, POINTER(SolveInfo), c_void_p]),
    ("ckkt_batch_factorize_solve", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                             c_void_p, c_int32, P_f64, POINTER(SolveInfo), c_void_p]),
    ("ckkt_solve_augmented", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_void_p, POINTER(SolveInfo), c_void_p]),
    ("ckkt_recover_bound_dual", c_int32, [c_int64, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    ("ckkt_apply_inverse", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("ckkt_export_k", c_int32, [c_void_p, P_i32, P_i32, c_void_p, c_void_p]),
    ("ckkt_host_factor_solve", c_int32, [c_void_p, P_f64, P_f64, P_f64, P_f64, P_f64, c_double, P_f64, P_f64,
                                         P_i32]),
    ("ckkt_host_factor_solve_inertia", c_int32, [c_void_p, P_f64, P_f64, P_f64, P_f64, P_f64, c_double,
                                                 POINTER(Inertia), P_f64, P_f64]),
    ("ckkt_features", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                c_void_p]),
    ("ckkt_mlp_forward", c_int32, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("ckkt_mlp_workspace", c_size_t, [c_int64]),
    ("ckkt_mlp_backward", c_int32, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("ckkt_mlp_backward_noalloc", c_int32, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("ckkt_adam", c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_float, c_void_p]),
    ("ckkt_mlp_train_step", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_float,
                                      POINTER(c_double), c_void_p]),
    ("ckkt_pcg_solve", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                 c_void_p, c_void_p, c_int32, c_double, c_int32, POINTER(SolveInfo), c_void_p]),
    ("ckkt_autotune", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                P_i32, POINTER(c_double), c_void_p]),
    ("ckkt_get_info", c_int32, [c_void_p, POINTER(Info)]),
    ("ckkt_status_string", c_char_p, [c_int32]),
    ("ckkt_destroy", None, [c_void_p]),
    ("ckkt_set_timing", c_int32, [c_void_p, c_int32]),
    ("ckkt_get_timing", c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
]

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_14236_amd.build_lib` "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class CkktError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {name}" if where else name)


def check(status, where=""):
    if status != CKKT_OK:
        raise CkktError(status, where)
