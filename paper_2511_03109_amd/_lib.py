"""ctypes declarations of the C ABI in include/ph.h (argument marshalling only)."""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libph.so")

PH_OK, PH_EINVAL, PH_EDOMAIN, PH_ENOMEM, PH_EHIP, PH_ESTATE, PH_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
KERNELS = {"gaussian": 0, "matern32": 1, "matern12": 2, "aniso_gaussian": 3, "poly_test": 4,
           "poly2_test": 5, "matern": 6}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2}
NEAR_MODES = {"auto": 0, "blocks": 1, "factored": 2}
FORMATS = {"h2": 0, "h": 1, "h2_implicit": 2}
COUPLINGS = {"materialized": 0, "implicit": 1}


class TreeOpts(C.Structure):
    _fields_ = [("d", C.c_int), ("lo", C.c_double), ("hi", C.c_double), ("leaf_size", C.c_int),
                ("l_max", C.c_int), ("eta2_num", C.c_int), ("eta2_den", C.c_int)]


class TreeInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int), ("l_max", C.c_int), ("n_nodes", C.c_int64),
                ("n_leaves", C.c_int64), ("n_near", C.c_int64), ("n_far", C.c_int64),
                ("n_classes", C.c_int64), ("near_entries", C.c_int64), ("min_far_level", C.c_int)]


class OfflineOpts(C.Structure):
    _fields_ = [("kernel", C.c_int), ("d_theta", C.c_int), ("theta_lo", C.c_double * 2),
                ("theta_hi", C.c_double * 2), ("p_s", C.c_int), ("p_theta", C.c_int),
                ("tol", C.c_double), ("num_threads", C.c_int)]


class CgStats(C.Structure):
    _fields_ = [("outer_steps", C.c_int), ("inner_iterations", C.c_int), ("rel_residual", C.c_double),
                ("converged", C.c_int)]


class TuneInfo(C.Structure):
    _fields_ = [("chunks", C.c_int), ("prefetch", C.c_int), ("overlap", C.c_int), ("ms", C.c_double),
                ("fused_tcb", C.c_int), ("fused_rt", C.c_int)]


class ModelInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_near_stored", C.c_int64), ("n_classes_stored", C.c_int64),
                ("near_entries", C.c_int64), ("near_factor_entries", C.c_int64),
                ("near_rank_mean", C.c_double), ("near_rank_max", C.c_int),
                ("far_rank_mean", C.c_double), ("far_rank_max", C.c_int),
                ("device_bytes", C.c_int64), ("kernel_evals", C.c_int64), ("P", C.c_int),
                ("p_theta", C.c_int), ("d_theta", C.c_int), ("svd_sweeps_max", C.c_int)]


class TraceStats(C.Structure):
    _fields_ = [("ms", C.c_double * 16), ("count", C.c_int64 * 16)]


STAGES = ["theta", "far_inst", "near_inst", "perm_in", "leaf_up", "transfer_up", "coupling",
          "transfer_down", "near_mvm", "perm_out", "coupling_reduce", "leaf_down", "bilinear",
          "solve", "near_gather"]

_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

SIGNATURES = {
    "ph_last_error": ([], C.c_char_p),
    "ph_version": ([], C.c_char_p),
    "ph_build_tree": ([_DP, C.c_int64, C.POINTER(TreeOpts), C.POINTER(_P)], C.c_int),
    "ph_tree_info_get": ([_P, C.POINTER(TreeInfo)], C.c_int),
    "ph_tree_perm": ([_P, _I64P], C.c_int),
    "ph_tree_nodes": ([_P, _I32P, _I32P, _I64P, _I64P, _I32P], C.c_int),
    "ph_tree_blocks": ([_P, _I32P, _I32P, _I32P], C.c_int),
    "ph_tree_classes": ([_P, _I32P, _I32P], C.c_int),
    "ph_tree_free": ([_P], None),
    "ph_kernel_eval": ([C.c_int, C.c_int, _DP, _DP, C.c_int64, _DP, _DP], C.c_int),
    "ph_offline_compress": ([_P, C.POINTER(OfflineOpts), _P, C.POINTER(_P)], C.c_int),
    "ph_offline_compress_h": ([_P, C.POINTER(OfflineOpts), _P, C.POINTER(_P)], C.c_int),
    "ph_offline_compress_gpu": ([_P, C.POINTER(OfflineOpts), _P, C.POINTER(_P)], C.c_int),
    "ph_offline_compress_tt": ([_P, C.POINTER(OfflineOpts), C.c_int, _P, C.POINTER(_P)], C.c_int),
    "ph_tt_far_ranks": ([_P, C.POINTER(OfflineOpts), C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
    "ph_model_format": ([_P, C.POINTER(C.c_int)], C.c_int),
    "ph_model_info_get": ([_P, C.POINTER(ModelInfo)], C.c_int),
    "ph_model_near_ranks": ([_P, _I32P], C.c_int),
    "ph_model_class_ranks": ([_P, _I32P], C.c_int),
    "ph_model_free": ([_P], None),
    "ph_instantiate": ([_P, _DP, C.c_int, C.c_int, _P, C.POINTER(_P)], C.c_int),
    "ph_instantiate_grad": ([_P, _DP, C.c_int, C.c_int, C.c_int, _P, C.POINTER(_P)], C.c_int),
    "ph_instantiate_ex": ([_P, _DP, C.c_int, C.c_int, C.c_int, C.c_int, _P, C.POINTER(_P)], C.c_int),
    "ph_inst_near_mode": ([_P, C.POINTER(C.c_int)], C.c_int),
    "ph_matvec": ([_P, _P, _P, C.c_int64, C.c_double, C.c_double, C.c_double, _P], C.c_int),
    "ph_matvec_noalloc": ([_P, _P, _P, C.c_int64, C.c_double, C.c_double, C.c_double, _P], C.c_int),
    "ph_bilinear": ([_P, _P, _P, C.c_int64, _P, _P], C.c_int),
    "ph_cg_solve": ([_P, _P, _P, _P, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                     C.POINTER(CgStats), _P], C.c_int),
    "ph_cg_solve_batch": ([_P, _P, _P, _P, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                           C.POINTER(CgStats), _P], C.c_int),
    "ph_autotune": ([_P, _P, _P, C.c_int64, _P, C.POINTER(TuneInfo)], C.c_int),
    "ph_graph_create": ([_P, _P, _P, C.c_int64, C.c_double, _P, C.POINTER(_P)], C.c_int),
    "ph_graph_launch": ([_P, _DP, _P], C.c_int),
    "ph_graph_free": ([_P], None),
    "ph_inst_near_block": ([_P, C.c_int, C.c_int64, _DP], C.c_int),
    "ph_inst_coupling": ([_P, C.c_int, C.c_int64, _DP], C.c_int),
    "ph_inst_free": ([_P], None),
    "ph_trace_enable": ([C.c_int], C.c_int),
    "ph_trace_read": ([C.POINTER(TraceStats), C.c_int], C.c_int),
}

_lib = None


def lib():
    """Load libph.so (built in-tree); raise loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2511_03109_amd.build` (there is no fallback)")
        h = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(h, name)
            f.argtypes = args
            f.restype = res
        _lib = h
    return _lib


class PHError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().ph_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def check(code, where):
    if code != PH_OK:
        raise PHError(code, where)
