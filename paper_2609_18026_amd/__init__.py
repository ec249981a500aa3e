"""MI355X (gfx950) mapped associated-Legendre / Fourier spectral transforms and RHS.

Python binding of the C ABI declared in include/mlg.h (libmlg.so, built in-tree by
``python -m paper_2609_18026_amd.build``).  The binding only marshals arguments:
every step of the computation runs in the library's HIP kernels.  There is no CPU
fallback; if the library is missing or fails to load, every entry point raises.
"""
from .binding import (Batch, Closure, MLG_FP32, MLG_FP64, MLG_LOG_PRESCRIBE, MLG_LOG_SOLVE, MLG_RHS_KPP, MLG_RHS_U2,
                      MLG_SPLIT_BF16, MlgError, Plan,
                      lib, mlg_backward, mlg_forward, mlg_grid, mlg_last_error, mlg_layout,
                      mlg_plan_create, mlg_plan_destroy, mlg_plan_nodes, mlg_plan_query, mlg_rhs_scalar,
                      mlg_rhs_tp, mlg_synthesize, mlg_tp_energy, mlg_timing_enable, mlg_timing_read)

__all__ = [
    "Batch", "Closure", "MLG_FP32", "MLG_FP64", "MLG_LOG_PRESCRIBE", "MLG_LOG_SOLVE", "MLG_RHS_KPP", "MLG_RHS_U2",
    "MLG_SPLIT_BF16", "MlgError", "Plan", "lib",
    "mlg_backward", "mlg_forward", "mlg_grid", "mlg_last_error", "mlg_layout", "mlg_plan_create",
    "mlg_plan_destroy", "mlg_plan_nodes", "mlg_plan_query", "mlg_rhs_scalar", "mlg_rhs_tp",
    "mlg_synthesize", "mlg_tp_energy", "mlg_timing_enable", "mlg_timing_read",
]
