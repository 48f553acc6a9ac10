"""ctypes declarations of libnpfem.so (the C ABI of include/npfem.h).

Loading fails loudly when the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint32, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnpfem.so")


class Material(ctypes.Structure):
    _fields_ = [(k, c_double) for k in ("B", "C", "D", "k_bend", "k_volume", "beta", "kappa",
                                        "density", "k_mat", "k_area_global")]


class SolverParams(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("lbfgs_m", c_int32), ("max_iter", c_int32),
                ("max_halvings", c_int32), ("tol", c_double), ("c1", c_double),
                ("noise_factor", c_double), ("cells_per_tile", c_int32), ("grid_blocks", c_int32),
                ("inverse_bf16", c_int32), ("volume_normaliser", c_int32)]


class NetConfig(ctypes.Structure):
    _fields_ = [("hidden", c_int32), ("layers", c_int32), ("force_floor", c_double), ("shape_scale", c_double)]


CELL_STATS_DTYPE = np.dtype([("iterations", np.int32), ("evaluations", np.int32),
                             ("status", np.uint32), ("halvings", np.int32), ("residual", np.float64),
                             ("objective", np.float64), ("volume", np.float64), ("area", np.float64)])

STATS_TOTAL_DTYPE = np.dtype([("cell_steps", np.int64), ("iterations", np.int64), ("evaluations", np.int64),
                              ("halvings", np.int64), ("not_converged", np.int64), ("status_count", np.int64, (4,)),
                              ("max_iterations", np.int32), ("start_fallback", np.int32), ("max_residual", np.float64)])

FP32, FP64 = 0, 1
CONVERGED, MAXITER, LS_FAIL, NONFINITE, DEGENERATE_TRI, START_FALLBACK = 1, 2, 4, 8, 16, 32
N_TERMS = 11
VOLUME_STEP_FROZEN, VOLUME_PAPER_LITERAL = 0, 1

_P = c_void_p
_SIGNATURES = {
    "npfem_status_string": (c_char_p, [c_int32]),
    "npfem_last_error": (c_char_p, []),
    "npfem_material_default": (None, [POINTER(Material)]),
    "npfem_solver_params_default": (None, [POINTER(SolverParams)]),
    "npfem_mesh_create": (c_int32, [c_int32, _P, c_int32, _P, POINTER(c_void_p)]),
    "npfem_mesh_destroy": (None, [c_void_p]),
    "npfem_mesh_query": (c_int32, [c_void_p, _P, _P, _P, _P, _P]),
    "npfem_mesh_rest_data": (c_int32, [c_void_p, _P, _P, _P, _P]),
    "npfem_plan_create": (c_int32, [c_int32, _P, c_int32, POINTER(Material), c_double,
                                    POINTER(SolverParams), POINTER(c_void_p)]),
    "npfem_plan_destroy": (None, [c_void_p]),
    "npfem_plan_masses": (c_int32, [c_void_p, c_int32, _P]),
    "npfem_batch_create": (c_int32, [c_void_p, c_int64, _P, POINTER(c_void_p), POINTER(c_int64)]),
    "npfem_batch_destroy": (None, [c_void_p]),
    "npfem_batch_schedule": (c_int32, [c_void_p, c_int32, c_int32]),
    "npfem_batch_get_schedule": (c_int32, [c_void_p, _P, _P, _P, _P]),
    "npfem_batch_autotune": (c_int32, [c_void_p, _P, _P, _P, _P, _P, c_int32, _P, _P]),
    "npfem_batch_set_graph": (c_int32, [c_void_p, c_int32]),
    "npfem_batch_graph_counts": (c_int32, [c_void_p, _P, _P]),
    "npfem_step": (c_int32, [c_void_p, _P, _P, _P, _P, _P, _P, _P, _P]),
    "npfem_step_noalloc": (c_int32, [c_void_p, _P, _P, _P, _P, _P, _P, _P, _P]),
    "npfem_collisions_detect": (c_int32, [c_void_p, _P, _P, c_double, _P, _P, _P, _P]),
    "npfem_step_contacts": (c_int32, [c_void_p, _P, _P, _P, _P, _P, c_double, _P, _P, _P, _P]),
    "npfem_eval": (c_int32, [c_void_p, _P, _P, _P, _P, _P, _P, _P]),
    "npfem_stats_accumulate": (c_int32, [_P, c_int64, _P, _P]),
    "npfem_stats_reset": (c_int32, [_P, _P]),
    "npfem_apply_inverse": (c_int32, [c_void_p, c_int32, c_int32, _P, _P, c_int32, _P, _P]),
    "npfem_solve_factor_workspace": (c_int64, [c_void_p, c_int32, c_int32]),
    "npfem_solve_factor": (c_int32, [c_void_p, c_int32, c_int32, _P, _P, c_int32, _P, c_int64, _P, _P]),
    "npfem_drag_forces": (c_int32, [c_void_p, _P, _P, _P, _P, _P, c_double, c_double, c_double,
                                    c_double, _P, _P]),
    "npfem_first_guess": (c_int32, [c_void_p, _P, _P, _P, _P, _P]),
    "npfem_net_config_default": (None, [POINTER(NetConfig)]),
    "npfem_net_param_count": (c_int64, [POINTER(NetConfig)]),
    "npfem_net_create": (c_int32, [c_void_p, POINTER(NetConfig), _P, POINTER(c_void_p)]),
    "npfem_net_destroy": (None, [c_void_p]),
    "npfem_net_set_params": (c_int32, [c_void_p, _P]),
    "npfem_net_get_params": (c_int32, [c_void_p, _P]),
    "npfem_net_infer": (c_int32, [c_void_p, c_void_p, _P, _P, _P, _P, _P]),
    "npfem_step_learned": (c_int32, [c_void_p, c_void_p, _P, _P, _P, _P, _P, _P, _P]),
    "npfem_net_loss_grad": (c_int32, [c_void_p, c_void_p, _P, c_int32, _P, _P, _P, _P, _P, POINTER(c_double),
                                      _P, _P]),
    "npfem_net_adam_step": (c_int32, [c_void_p, _P, c_double, c_double, c_double, c_double, _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1903_06479_amd.build.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class NpfemError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.npfem_last_error().decode()
        super().__init__(f"{where}: {L.npfem_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != 0:
        raise NpfemError(status, where)
