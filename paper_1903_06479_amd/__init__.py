"""MI355X-native batched npFEM red-blood-cell step (Kotsalos, Latt & Chopard,
arXiv:1903.06479), behind the C ABI of include/npfem.h.

    from paper_1903_06479_amd import Mesh, Plan, Batch, default_material, default_params
"""
from .solver import Batch, Mesh, Net, Plan, StatsTotal, default_material, default_net_config, default_params  # noqa: F401
from ._native import (CELL_STATS_DTYPE, CONVERGED, DEGENERATE_TRI, FP32, FP64, LS_FAIL, MAXITER, START_FALLBACK,  # noqa: F401
                      NONFINITE)
