"""ctypes mirror of include/pdd.h (structures, enums, function prototypes)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PDD_LIBRARY selects another build of the library (e.g. a host-sanitizer build)
LIB_PATH = os.environ.get("PDD_LIBRARY") or os.path.join(HERE, "libpdd.so")

PDD_OK, PDD_WARN_CENSORED, PDD_WARN_REDRAWN = 0, 1, 2
PDD_ERR_INVALID_ARG, PDD_ERR_UNSUPPORTED, PDD_ERR_NOT_ADMISSIBLE, PDD_ERR_HIP, PDD_ERR_NO_MEMORY = -1, -2, -3, -4, -5

PDD_DOM_BOX, PDD_DOM_BALL, PDD_DOM_FREE = 0, 1, 2
PDD_FP64_PLAIN, PDD_FP64, PDD_FP32_STEP = 0, 1, 2
PDD_RNG_PAIR52, PDD_RNG_QUAD24 = 0, 1
PDD_SCHED_AUTO, PDD_SCHED_PERSISTENT, PDD_SCHED_PERSISTENT_GRAPH = 0, 1, 2
(PDD_KERNEL_WALK, PDD_KERNEL_WALK_ADJOINT, PDD_KERNEL_WOS, PDD_KERNEL_WALK_BATCH, PDD_KERNEL_WOS_BATCH,
 PDD_KERNEL_BRANCH, PDD_KERNEL_BRANCH_BVP) = range(7)

EXPORTED = ["pdd_mc_interface", "pdd_mc_interface_noalloc", "pdd_mc_interface_batch", "pdd_wos_interface_batch",
            "pdd_wos_interface", "pdd_branching_eval", "pdd_branching_bvp", "pdd_mc_adjoint",
            "pdd_mc_value_jacobian", "pdd_item_count", "pdd_set_schedule", "pdd_get_schedule",
            "pdd_save_schedules", "pdd_load_schedules",
            "pdd_param_count", "pdd_jacobian_apply", "pdd_misfit_gradient", "pdd_node_moments", "pdd_merge_estimates",
            "pdd_query_warnings", "pdd_release_workspace", "pdd_cached_plan_count", "pdd_status_string",
            "pdd_last_error", "pdd_version"]


class pdd_domain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("center", C.c_double * 3), ("radius", C.c_double)]


class pdd_factor(C.Structure):
    _fields_ = [("fn", C.c_int32), ("dim", C.c_int32), ("power", C.c_int32), ("pad", C.c_int32),
                ("a", C.c_double), ("b", C.c_double)]


class pdd_fun(C.Structure):
    _fields_ = [("n_terms", C.c_int32), ("n_factors", C.c_int32), ("factors", C.POINTER(pdd_factor)),
                ("coef", C.c_void_p), ("poly_degree", C.c_int32), ("pad", C.c_int32), ("poly", C.c_void_p)]


class pdd_linear_problem(C.Structure):
    _fields_ = [("domain", pdd_domain), ("sigma", C.c_double), ("b", pdd_fun * 3), ("c", pdd_fun),
                ("f", pdd_fun), ("g", pdd_fun)]


class pdd_branching_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("max_segments", C.c_int32), ("sigma", C.c_double), ("beta", C.c_double),
                ("T", C.c_double), ("alpha", C.c_double * 5), ("q", C.c_double * 5), ("psi_sup", C.c_double),
                ("psi", pdd_fun)]


class pdd_branching_boundary(C.Structure):
    _fields_ = [("domain", pdd_domain), ("g", pdd_fun), ("g_sup", C.c_double), ("dt", C.c_double),
                ("n_times", C.c_int32), ("pad", C.c_int32), ("times", C.POINTER(C.c_double))]


class pdd_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rng_layout", C.c_int32), ("max_steps", C.c_int64),
                ("dump_phi", C.c_void_p), ("dump_steps", C.c_void_p), ("schedule", C.c_int32),
                ("chunk_paths", C.c_int32), ("blocks_per_cu", C.c_int32), ("refill_groups", C.c_int32),
                ("boundary_correction", C.c_int32), ("specialize", C.c_int32),
                ("skip_items", C.c_void_p), ("partials", C.c_void_p)]


class pdd_item_stat(C.Structure):
    _fields_ = [("mean", C.c_double), ("m2", C.c_double), ("n", C.c_int64), ("steps", C.c_int64),
                ("censored", C.c_int64), ("redrawn", C.c_int64)]


class pdd_node_stat(C.Structure):
    _fields_ = [("mean", C.c_double), ("m2", C.c_double), ("n", C.c_int64), ("steps", C.c_int64),
                ("censored", C.c_int64)]


class pdd_launch_schedule(C.Structure):
    _fields_ = [("chunk_paths", C.c_int32), ("blocks_per_cu", C.c_int32), ("refill_groups", C.c_int32),
                ("pad", C.c_int32)]


class pdd_fun_grad(C.Structure):
    _fields_ = [("dcoef", C.c_void_p), ("dpoly", C.c_void_p)]


def load(path: str = LIB_PATH) -> C.CDLL:
    L = C.CDLL(path)
    L.pdd_mc_interface.argtypes = [C.POINTER(pdd_linear_problem), C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                   C.c_double, C.c_uint64, C.POINTER(pdd_options), C.c_void_p, C.c_void_p]
    L.pdd_mc_interface.restype = C.c_int
    L.pdd_mc_interface_noalloc.argtypes = L.pdd_mc_interface.argtypes
    L.pdd_mc_interface_noalloc.restype = C.c_int
    L.pdd_mc_interface_batch.argtypes = [C.POINTER(pdd_linear_problem), C.c_int32, C.POINTER(C.c_int32), C.c_void_p,
                                         C.c_int64, C.POINTER(C.c_int64), C.c_double, C.c_uint64,
                                         C.POINTER(pdd_options), C.c_void_p, C.c_void_p]
    L.pdd_mc_interface_batch.restype = C.c_int
    L.pdd_wos_interface_batch.argtypes = L.pdd_mc_interface_batch.argtypes
    L.pdd_wos_interface_batch.restype = C.c_int
    L.pdd_wos_interface.argtypes = L.pdd_mc_interface.argtypes
    L.pdd_wos_interface.restype = C.c_int
    L.pdd_branching_eval.argtypes = [C.POINTER(pdd_branching_problem), C.c_void_p, C.c_int64, C.c_int64, C.c_uint64,
                                     C.POINTER(pdd_options), C.c_void_p, C.c_void_p]
    L.pdd_branching_eval.restype = C.c_int
    L.pdd_branching_bvp.argtypes = [C.POINTER(pdd_branching_problem), C.POINTER(pdd_branching_boundary), C.c_void_p,
                                    C.c_int64, C.c_int64, C.c_uint64, C.POINTER(pdd_options), C.c_void_p,
                                    C.c_void_p]
    L.pdd_branching_bvp.restype = C.c_int
    L.pdd_mc_adjoint.argtypes = [C.POINTER(pdd_linear_problem), C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                 C.c_double, C.c_uint64, C.POINTER(pdd_options), C.c_void_p,
                                 C.POINTER(pdd_fun_grad), C.c_void_p, C.c_void_p]
    L.pdd_mc_adjoint.restype = C.c_int
    L.pdd_mc_value_jacobian.argtypes = [C.POINTER(pdd_linear_problem), C.c_void_p, C.c_int64,
                                        C.POINTER(C.c_int64), C.c_double, C.c_uint64, C.POINTER(pdd_options),
                                        C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    L.pdd_mc_value_jacobian.restype = C.c_int
    L.pdd_item_count.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_int64), C.POINTER(pdd_options)]
    L.pdd_item_count.restype = C.c_int64
    L.pdd_set_schedule.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(pdd_launch_schedule)]
    L.pdd_set_schedule.restype = C.c_int
    L.pdd_get_schedule.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(pdd_launch_schedule),
                                   C.POINTER(C.c_int32)]
    L.pdd_get_schedule.restype = C.c_int
    L.pdd_save_schedules.argtypes = [C.c_char_p]
    L.pdd_save_schedules.restype = C.c_int
    L.pdd_load_schedules.argtypes = [C.c_char_p]
    L.pdd_load_schedules.restype = C.c_int
    L.pdd_param_count.argtypes = [C.POINTER(pdd_linear_problem)]
    L.pdd_param_count.restype = C.c_int64
    L.pdd_jacobian_apply.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
    L.pdd_jacobian_apply.restype = C.c_int
    L.pdd_misfit_gradient.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
    L.pdd_misfit_gradient.restype = C.c_int
    L.pdd_merge_estimates.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
    L.pdd_merge_estimates.restype = C.c_int
    L.pdd_node_moments.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    L.pdd_node_moments.restype = C.c_int
    L.pdd_cached_plan_count.argtypes = []
    L.pdd_cached_plan_count.restype = C.c_int64
    L.pdd_query_warnings.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.pdd_query_warnings.restype = C.c_int
    L.pdd_release_workspace.argtypes = []
    L.pdd_release_workspace.restype = C.c_int
    L.pdd_status_string.argtypes = [C.c_int]
    L.pdd_status_string.restype = C.c_char_p
    L.pdd_last_error.argtypes = []
    L.pdd_last_error.restype = C.c_char_p
    L.pdd_version.argtypes = []
    L.pdd_version.restype = C.c_int
    return L
