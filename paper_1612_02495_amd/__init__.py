"""Swept time-space decomposition for explicit 1-D periodic stencils on MI355X.

The computation lives in libswept.so (HIP kernels for gfx950 behind the C ABI
of include/swept.h); this package is its Python binding.  Importing it does
not load the library; the first call does.
"""
from .swept import (Plan, SweptError, naive_run, swept_last_error, swept_plan_create,
                    swept_plan_destroy, swept_plan_info, swept_plan_set_engine, swept_plan_set_checks, swept_run,
                    swept_run_noalloc, swept_batch_set_checks,
                    swept_schedule, swept_tile_geometry, swept_autotune, swept_autotune_lookup,
                    swept_autotune_forget, Batch, swept_batch_create, swept_batch_run, swept_batch_set_engine,
                    swept_batch_info,
                    swept_batch_destroy, AdjointPlan, swept_heat, swept_adjoint_create, swept_forward_ckpt,
                    swept_adjoint_run, swept_adjoint_info, swept_adjoint_destroy, KsAdjointPlan, swept_ks,
                    swept_ks_adjoint_create, swept_ks_forward_ckpt, swept_ks_adjoint_run, swept_ks_adjoint_info,
                    swept_ks_adjoint_destroy, release_cached_plans)

__all__ = ["Plan", "SweptError", "swept_plan_create", "swept_run", "swept_run_noalloc", "naive_run",
           "swept_plan_info", "swept_plan_set_engine", "swept_plan_set_checks", "swept_batch_set_checks",
           "swept_plan_destroy", "swept_last_error", "swept_schedule",
           "swept_tile_geometry", "swept_autotune", "swept_autotune_lookup", "swept_autotune_forget",
           "Batch", "swept_batch_create", "swept_batch_run", "swept_batch_set_engine", "swept_batch_info",
           "swept_batch_destroy",
           "AdjointPlan", "swept_heat", "swept_adjoint_create", "swept_forward_ckpt", "swept_adjoint_run",
           "swept_adjoint_info", "swept_adjoint_destroy", "KsAdjointPlan", "swept_ks",
           "swept_ks_adjoint_create", "swept_ks_forward_ckpt", "swept_ks_adjoint_run", "swept_ks_adjoint_info",
           "swept_ks_adjoint_destroy", "release_cached_plans"]
