"""Python binding of the swept library: the C-ABI entry points under their own
names, plus a small ``Plan`` convenience class.  PyTorch only supplies device
memory (``Tensor.data_ptr()``) and the HIP stream; all arithmetic runs in the
HIP kernels of libswept.so.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (SWEPT_ENGINE_AUTO, SWEPT_ENGINE_COMPACT, SWEPT_ENGINE_LDS, SWEPT_ENGINE_RESIDENT,
                   SWEPT_ENGINE_WAVE, SWEPT_F32, SWEPT_F64, SWEPT_HEAT_FTCS, SWEPT_HEAT_INSULATED,
                   SWEPT_KS_RK2, SweptError, check)

KINDS = {"heat": SWEPT_HEAT_FTCS, "ks": SWEPT_KS_RK2, "heat_insulated": SWEPT_HEAT_INSULATED}
ENGINES = {"auto": SWEPT_ENGINE_AUTO, "lds": SWEPT_ENGINE_LDS, "wave": SWEPT_ENGINE_WAVE,
           "compact": SWEPT_ENGINE_COMPACT, "resident": SWEPT_ENGINE_RESIDENT}


def _kind(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def _dtype_code(dtype) -> int:
    import torch
    if dtype in (torch.float64, np.float64, "f64", "float64", SWEPT_F64):
        return SWEPT_F64
    if dtype in (torch.float32, np.float32, "f32", "float32", SWEPT_F32):
        return SWEPT_F32
    raise ValueError(f"unsupported dtype {dtype!r}")


def _stream_ptr(tensor, stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(tensor.device)
    return ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


# --------------------------------------------------------- C-ABI names --

def swept_plan_create(n: int, kind, dtype, dt: float, dx: float, alpha: float = 0.0,
                      tile_width: int = 0, steps_per_cycle: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(_lib.lib().swept_plan_create(ctypes.byref(h), int(n), _kind(kind), _dtype_code(dtype),
                                       float(dt), float(dx), float(alpha), int(tile_width),
                                       int(steps_per_cycle)))
    return h


def swept_run(plan, u, steps: int, stream=None) -> None:
    check(_lib.lib().swept_run(plan, ctypes.c_void_p(u.data_ptr()), int(steps), _stream_ptr(u, stream)))


def swept_run_noalloc(n: int, kind, dtype, dt: float, dx: float, alpha: float, tile_width: int,
                      steps_per_cycle: int, u, steps: int, stream=None) -> None:
    """swept_run without a plan: the edge slots live in the library's static
    per-device array, so the call allocates no device memory."""
    check(_lib.lib().swept_run_noalloc(int(n), _kind(kind), _dtype_code(dtype), float(dt), float(dx), float(alpha),
                                       int(tile_width), int(steps_per_cycle), ctypes.c_void_p(u.data_ptr()),
                                       int(steps), _stream_ptr(u, stream)))


def naive_run(plan, u, steps: int, stream=None) -> None:
    check(_lib.lib().naive_run(plan, ctypes.c_void_p(u.data_ptr()), int(steps), _stream_ptr(u, stream)))


def swept_plan_info(plan) -> dict:
    w, spc, ws = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    check(_lib.lib().swept_plan_info(plan, ctypes.byref(w), ctypes.byref(spc), ctypes.byref(ws)))
    return {"tile_width": w.value, "steps_per_cycle": spc.value, "workspace_bytes": ws.value}


def swept_plan_set_engine(plan, engine) -> None:
    e = ENGINES[engine] if isinstance(engine, str) else int(engine)
    check(_lib.lib().swept_plan_set_engine(plan, e))


def swept_plan_set_checks(plan, flags: int) -> None:
    check(_lib.lib().swept_plan_set_checks(plan, int(flags)))


def swept_plan_destroy(plan) -> None:
    if plan:
        _lib.lib().swept_plan_destroy(plan)


def swept_last_error() -> str:
    return _lib.last_error()


def swept_schedule(kind, tile_width: int, steps_per_cycle: int, steps: int) -> list[int]:
    count = ctypes.c_int64()
    check(_lib.lib().swept_schedule(_kind(kind), int(tile_width), int(steps_per_cycle), int(steps),
                                    None, 0, ctypes.byref(count)))
    buf = (ctypes.c_int32 * max(count.value, 1))()
    check(_lib.lib().swept_schedule(_kind(kind), int(tile_width), int(steps_per_cycle), int(steps),
                                    buf, count.value, ctypes.byref(count)))
    return list(buf[: count.value])


def swept_tile_geometry(kind, tile_width: int) -> dict:
    t, r, e = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(_lib.lib().swept_tile_geometry(_kind(kind), int(tile_width), ctypes.byref(t),
                                         ctypes.byref(r), ctypes.byref(e)))
    return {"full_tiers": t.value, "row_values": r.value, "edge_slot_values": e.value}


ENGINE_NAMES = {v: k for k, v in ENGINES.items()}


def swept_autotune(n: int, kind, dtype, dt: float, dx: float, alpha: float = 0.0, steps: int = 0,
                   max_results: int = 64) -> dict:
    """Time the candidate configurations (device work, synchronous); returns the
    winner and every timed candidate."""
    res = (_lib.TuneResult * max_results)()
    cnt, w, spc, eng = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(_lib.lib().swept_autotune(int(n), _kind(kind), _dtype_code(dtype), float(dt), float(dx),
                                    float(alpha), int(steps), res, max_results, ctypes.byref(cnt),
                                    ctypes.byref(w), ctypes.byref(spc), ctypes.byref(eng)))
    cands = [{"tile_width": r.tile_width, "steps_per_cycle": r.steps_per_cycle,
              "engine": ENGINE_NAMES[r.engine], "ns_per_cell_update": r.ns_per_cell_update}
             for r in res[: min(cnt.value, max_results)]]
    return {"tile_width": w.value, "steps_per_cycle": spc.value, "engine": ENGINE_NAMES[eng.value],
            "candidates": cands}


def swept_autotune_lookup(n: int, kind, dtype):
    """Remembered configuration for (kind, dtype, n), or None."""
    w, spc, eng, ns = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    rc = _lib.lib().swept_autotune_lookup(int(n), _kind(kind), _dtype_code(dtype), ctypes.byref(w),
                                          ctypes.byref(spc), ctypes.byref(eng), ctypes.byref(ns))
    if rc == _lib.SWEPT_EUNSUPPORTED:
        return None
    check(rc)
    return {"tile_width": w.value, "steps_per_cycle": spc.value, "engine": ENGINE_NAMES[eng.value],
            "ns_per_cell_update": ns.value}


def swept_autotune_forget() -> None:
    _lib.lib().swept_autotune_forget()


# ------------------------------------------------------------ wrapper --

# ------------------------------------------------------------- batched --

def swept_batch_create(n, kind, dtype, dt, dx, alpha, steps: int) -> ctypes.c_void_p:
    n = np.ascontiguousarray(n, dtype=np.int64)
    m = n.size
    dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (m,)))
    dx = np.ascontiguousarray(np.broadcast_to(np.asarray(dx, dtype=np.float64), (m,)))
    alpha = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, dtype=np.float64), (m,)))
    pd = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    check(_lib.lib().swept_batch_create(ctypes.byref(h), m, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        _kind(kind), _dtype_code(dtype), dt.ctypes.data_as(pd),
                                        dx.ctypes.data_as(pd), alpha.ctypes.data_as(pd), int(steps)))
    return h


def swept_batch_run(batch, u, use_graph: bool = True, stream=None) -> None:
    check(_lib.lib().swept_batch_run(batch, ctypes.c_void_p(u.data_ptr()), int(bool(use_graph)),
                                     _stream_ptr(u, stream)))


def swept_batch_set_engine(batch, engine) -> None:
    e = ENGINES[engine] if isinstance(engine, str) else int(engine)
    check(_lib.lib().swept_batch_set_engine(batch, e))


def swept_batch_set_checks(batch, flags: int) -> None:
    check(_lib.lib().swept_batch_set_checks(batch, int(flags)))


def swept_batch_info(batch, nprob: int) -> dict:
    tot, ws, grid = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_int()
    offs = np.zeros(nprob, dtype=np.int64)
    check(_lib.lib().swept_batch_info(batch, ctypes.byref(tot), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      ctypes.byref(ws), ctypes.byref(grid)))
    return {"total_points": tot.value, "offsets": offs, "workspace_bytes": ws.value, "grid": grid.value}


def swept_batch_destroy(batch) -> None:
    if batch:
        _lib.lib().swept_batch_destroy(batch)


class Batch:
    """Owns a batched plan: independent periodic grids stored back to back."""

    def __init__(self, n, kind, dtype, dt, dx, alpha, steps: int):
        import torch
        self.n = np.asarray(n, dtype=np.int64).copy()
        self.kind = _kind(kind)
        self.dtype = torch.float64 if _dtype_code(dtype) == SWEPT_F64 else torch.float32
        self.steps = int(steps)
        self._h = swept_batch_create(self.n, kind, dtype, dt, dx, alpha, steps)
        inf = swept_batch_info(self._h, self.n.size)
        self.offsets = inf["offsets"]
        self.total_points = inf["total_points"]
        self.grid = inf["grid"]
        self.workspace_bytes = inf["workspace_bytes"]

    def set_engine(self, engine):
        """'resident' (grids of up to 16384 points whole in one workgroup's
        registers, the rest as compacted swept tiles), 'compact' (compacted swept
        tiles for every grid), 'wave' (register-engine swept tiles for every
        grid) or 'auto' (the default, the same as 'resident')."""
        swept_batch_set_engine(self._h, engine)
        self.grid = swept_batch_info(self._h, self.n.size)["grid"]
        return self

    def set_checks(self, nonfinite: bool = True):
        """Opt-in check of every grid for NaN or Inf after each run."""
        swept_batch_set_checks(self._h, _lib.SWEPT_CHECK_NONFINITE if nonfinite else 0)
        return self

    def run(self, u, use_graph: bool = True, stream=None):
        if not u.is_cuda or u.dtype != self.dtype or u.numel() != self.total_points or not u.is_contiguous():
            raise ValueError(f"u must be a contiguous device {self.dtype} tensor of {self.total_points} elements")
        swept_batch_run(self._h, u, use_graph, stream)
        return u

    def split(self, u):
        return [u[o:o + m] for o, m in zip(self.offsets, self.n)]

    def close(self):
        if self._h:
            swept_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- adjoint --

def swept_adjoint_create(batch: int, n: int, dtype, dt: float, dx: float, steps: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(_lib.lib().swept_adjoint_create(ctypes.byref(h), int(batch), int(n), _dtype_code(dtype), float(dt),
                                          float(dx), int(steps)))
    return h


def swept_adjoint_create_segmented(batch: int, n: int, dtype, dt: float, dx: float, steps: int,
                                   segment: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(_lib.lib().swept_adjoint_create_segmented(ctypes.byref(h), int(batch), int(n), _dtype_code(dtype),
                                                    float(dt), float(dx), int(steps), int(segment)))
    return h


def swept_forward_ckpt(adj, u0, alpha, uT, stream=None) -> None:
    check(_lib.lib().swept_forward_ckpt(adj, ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(alpha.data_ptr()),
                                        ctypes.c_void_p(uT.data_ptr()), _stream_ptr(u0, stream)))


def swept_adjoint_run(adj, g_uT, g_u0, g_alpha, stream=None) -> None:
    check(_lib.lib().swept_adjoint_run(adj, ctypes.c_void_p(g_uT.data_ptr()), ctypes.c_void_p(g_u0.data_ptr()),
                                       ctypes.c_void_p(g_alpha.data_ptr()), _stream_ptr(g_uT, stream)))


def swept_adjoint_info(adj) -> dict:
    cb, w, spc, r = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    check(_lib.lib().swept_adjoint_info(adj, ctypes.byref(cb), ctypes.byref(w), ctypes.byref(spc), ctypes.byref(r)))
    return {"checkpoint_bytes": cb.value, "tile_width": w.value, "steps_per_cycle": spc.value,
            "leading_classic_steps": r.value}


def swept_adjoint_destroy(adj) -> None:
    if adj:
        _lib.lib().swept_adjoint_destroy(adj)


class AdjointPlan:
    """Checkpointed swept forward and reverse sweep for a batch of heat grids."""

    def __init__(self, batch: int, n: int, dt: float, dx: float, steps: int, segment: int = 1):
        """segment: phases per checkpoint segment (1 keeps every phase's edge
        state; 0 picks about sqrt(phases), two-level checkpointing)."""
        self.batch, self.n, self.steps = int(batch), int(n), int(steps)
        self._h = (swept_adjoint_create(batch, n, "f64", dt, dx, steps) if segment == 1
                   else swept_adjoint_create_segmented(batch, n, "f64", dt, dx, steps, segment))
        self.info = swept_adjoint_info(self._h)
        self.generation = 0  # forward passes run so far (each rewrites the checkpoints)

    def _check(self, t, shape):
        import torch
        if not t.is_cuda or t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")

    def forward(self, u0, alpha, uT, stream=None):
        self._check(u0, (self.batch, self.n))
        self._check(alpha, (self.batch,))
        self._check(uT, (self.batch, self.n))
        swept_forward_ckpt(self._h, u0, alpha, uT, stream)
        self.generation += 1
        return uT

    def adjoint(self, g_uT, g_u0, g_alpha, stream=None):
        self._check(g_uT, (self.batch, self.n))
        self._check(g_u0, (self.batch, self.n))
        self._check(g_alpha, (self.batch,))
        swept_adjoint_run(self._h, g_uT, g_u0, g_alpha, stream)
        return g_u0, g_alpha

    def close(self):
        if self._h:
            swept_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Adjoint plans kept between autograd calls.  A plan's checkpoints are large
# (2.06 n x 8 bytes per grid per 32-step phase for heat, unless segmented),
# so a training loop must not allocate them anew at every step.  The pool
# holds plans whose checkpoints no pending backward needs: a forward takes a
# free plan of its configuration (or makes one) and its backward puts it back.
# Every forward bumps the plan's generation; a later backward of the same
# graph (retain_graph, gradcheck) whose plan has since run another forward
# recomputes its own forward, into a free plan, from the saved inputs.
_FREE_PLANS: dict = {}
_POOL_LIMIT = 1  # free plans kept per configuration


def _take_plan(key, make):
    free = _FREE_PLANS.get(key)
    if free:
        return free.pop()
    return make()


def _return_plan(key, plan):
    free = _FREE_PLANS.setdefault(key, [])
    if plan not in free and len(free) < _POOL_LIMIT:
        free.append(plan)


def release_cached_plans() -> None:
    """Drop the adjoint plans kept for reuse by swept_heat and swept_ks (their
    device memory is freed once no autograd graph refers to them)."""
    _FREE_PLANS.clear()


def _plan_for_backward(ctx, make, forward):
    """The plan holding ctx's checkpoints, recomputing them when needed."""
    plan = ctx.plan
    if plan.generation != ctx.generation:
        plan = _take_plan(ctx.key, make)
        forward(plan)
        ctx.plan, ctx.generation = plan, plan.generation
    return plan


def _swept_heat_fn():
    import torch

    class SweptHeatFn(torch.autograd.Function):
        """u_T = A(alpha)^steps u_0 for a batch of periodic heat grids (swept forward,
        checkpointed); backward is the hand-written swept adjoint, returning
        dJ/du_0 and dJ/dalpha."""

        @staticmethod
        def forward(ctx, u0, alpha, steps, dt, dx, segment):
            u0 = u0.contiguous()
            alpha = alpha.contiguous()
            key = ("heat", u0.device.index, u0.shape[0], u0.shape[1], float(dt), float(dx), int(steps), segment)
            ctx.make = lambda: AdjointPlan(u0.shape[0], u0.shape[1], dt, dx, steps, segment)
            plan = _take_plan(key, ctx.make)
            uT = torch.empty_like(u0)
            plan.forward(u0, alpha, uT)
            ctx.plan, ctx.key, ctx.generation = plan, key, plan.generation
            ctx.save_for_backward(u0, alpha)
            return uT

        @staticmethod
        def backward(ctx, g_uT):
            u0, alpha = ctx.saved_tensors
            plan = _plan_for_backward(ctx, ctx.make, lambda p: p.forward(u0, alpha, torch.empty_like(u0)))
            g_u0 = torch.empty((plan.batch, plan.n), dtype=torch.float64, device=g_uT.device)
            g_alpha = torch.empty((plan.batch,), dtype=torch.float64, device=g_uT.device)
            plan.adjoint(g_uT.contiguous(), g_u0, g_alpha)
            # a later forward may overwrite the checkpoints only after this
            # reverse sweep has read them: it runs on the same stream
            _return_plan(ctx.key, plan)
            return g_u0, g_alpha, None, None, None, None

    return SweptHeatFn


_SWEPT_HEAT_FN = None


def swept_heat(u0, alpha, steps: int, dt: float, dx: float, checkpoint_segment: int = 1):
    """Differentiable swept heat run: u0 [batch, n] float64, alpha [batch] float64.
    checkpoint_segment: 1 keeps every phase's edge state for the backward;
    0 (two-level, about sqrt(phases) per segment) or k > 1 keep every k-th and
    recompute the rest during the backward (less memory, one more forward)."""
    global _SWEPT_HEAT_FN
    if _SWEPT_HEAT_FN is None:
        _SWEPT_HEAT_FN = _swept_heat_fn()
    return _SWEPT_HEAT_FN.apply(u0, alpha, int(steps), float(dt), float(dx), int(checkpoint_segment))


def swept_ks_adjoint_create(batch: int, n: int, dtype, dt: float, dx: float, steps: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(_lib.lib().swept_ks_adjoint_create(ctypes.byref(h), int(batch), int(n), _dtype_code(dtype), float(dt),
                                             float(dx), int(steps)))
    return h


def swept_ks_forward_ckpt(adj, u0, uT, stream=None) -> None:
    check(_lib.lib().swept_ks_forward_ckpt(adj, ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(uT.data_ptr()),
                                           _stream_ptr(u0, stream)))


def swept_ks_adjoint_run(adj, g_uT, g_u0, stream=None) -> None:
    check(_lib.lib().swept_ks_adjoint_run(adj, ctypes.c_void_p(g_uT.data_ptr()), ctypes.c_void_p(g_u0.data_ptr()),
                                          _stream_ptr(g_uT, stream)))


def swept_ks_adjoint_info(adj) -> dict:
    cb, w, spc, r = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    check(_lib.lib().swept_ks_adjoint_info(adj, ctypes.byref(cb), ctypes.byref(w), ctypes.byref(spc),
                                           ctypes.byref(r)))
    return {"checkpoint_bytes": cb.value, "tile_width": w.value, "steps_per_cycle": spc.value,
            "leading_classic_steps": r.value}


def swept_ks_adjoint_destroy(adj) -> None:
    if adj:
        _lib.lib().swept_ks_adjoint_destroy(adj)


class KsAdjointPlan:
    """Checkpointed swept forward and reverse sweep for a batch of KS grids."""

    def __init__(self, batch: int, n: int, dt: float, dx: float, steps: int):
        self.batch, self.n, self.steps = int(batch), int(n), int(steps)
        self._h = swept_ks_adjoint_create(batch, n, "f64", dt, dx, steps)
        self.info = swept_ks_adjoint_info(self._h)
        self.generation = 0  # forward passes run so far (each rewrites the checkpoints)

    def _check(self, t, shape):
        import torch
        if not t.is_cuda or t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")

    def forward(self, u0, uT, stream=None):
        self._check(u0, (self.batch, self.n))
        self._check(uT, (self.batch, self.n))
        if u0.data_ptr() == uT.data_ptr():
            raise ValueError("u0 and uT may not alias")
        swept_ks_forward_ckpt(self._h, u0, uT, stream)
        self.generation += 1
        return uT

    def adjoint(self, g_uT, g_u0, stream=None):
        self._check(g_uT, (self.batch, self.n))
        self._check(g_u0, (self.batch, self.n))
        if g_uT.data_ptr() == g_u0.data_ptr():
            raise ValueError("g_uT and g_u0 may not alias")
        swept_ks_adjoint_run(self._h, g_uT, g_u0, stream)
        return g_u0

    def close(self):
        if self._h:
            swept_ks_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _swept_ks_fn():
    import torch

    class SweptKsFn(torch.autograd.Function):
        """u_T of a batch of periodic KS grids (swept forward, checkpointed);
        backward is the hand-written swept adjoint, returning dJ/du_0."""

        @staticmethod
        def forward(ctx, u0, steps, dt, dx):
            u0 = u0.contiguous()
            key = ("ks", u0.device.index, u0.shape[0], u0.shape[1], float(dt), float(dx), int(steps))
            ctx.make = lambda: KsAdjointPlan(u0.shape[0], u0.shape[1], dt, dx, steps)
            plan = _take_plan(key, ctx.make)
            uT = torch.empty_like(u0)
            plan.forward(u0, uT)
            ctx.plan, ctx.key, ctx.generation = plan, key, plan.generation
            ctx.save_for_backward(u0)
            return uT

        @staticmethod
        def backward(ctx, g_uT):
            (u0,) = ctx.saved_tensors
            plan = _plan_for_backward(ctx, ctx.make, lambda p: p.forward(u0, torch.empty_like(u0)))
            g_u0 = torch.empty((plan.batch, plan.n), dtype=torch.float64, device=g_uT.device)
            plan.adjoint(g_uT.contiguous(), g_u0)
            _return_plan(ctx.key, plan)
            return g_u0, None, None, None

    return SweptKsFn


_SWEPT_KS_FN = None


def swept_ks(u0, steps: int, dt: float, dx: float):
    """Differentiable swept KS run: u0 [batch, n] float64."""
    global _SWEPT_KS_FN
    if _SWEPT_KS_FN is None:
        _SWEPT_KS_FN = _swept_ks_fn()
    return _SWEPT_KS_FN.apply(u0, int(steps), float(dt), float(dx))


class Plan:
    """Owns a swept plan; validates tensors before handing them to the C ABI."""

    def __init__(self, n: int, kind, dtype, dt: float, dx: float, alpha: float = 0.0,
                 tile_width: int = 0, steps_per_cycle: int = 0, engine=None):
        import torch
        self.n = int(n)
        self.kind = _kind(kind)
        self.dtype = torch.float64 if _dtype_code(dtype) == SWEPT_F64 else torch.float32
        self._h = swept_plan_create(n, kind, dtype, dt, dx, alpha, tile_width, steps_per_cycle)
        if engine is not None:
            swept_plan_set_engine(self._h, engine)

    def _check_tensor(self, u):
        if not u.is_cuda:
            raise ValueError("u must be a device tensor")
        if u.dtype != self.dtype or u.numel() != self.n or not u.is_contiguous():
            raise ValueError(f"u must be a contiguous {self.dtype} tensor of {self.n} elements")

    def run(self, u, steps: int, stream=None):
        self._check_tensor(u)
        swept_run(self._h, u, steps, stream)
        return u

    def naive(self, u, steps: int, stream=None):
        self._check_tensor(u)
        naive_run(self._h, u, steps, stream)
        return u

    def set_engine(self, engine):
        swept_plan_set_engine(self._h, engine)

    def set_checks(self, nonfinite: bool = True):
        """Opt-in check: runs then wait for their stream and raise SweptError
        (code SWEPT_ENONFINITE) when the grid holds NaN or Inf."""
        swept_plan_set_checks(self._h, _lib.SWEPT_CHECK_NONFINITE if nonfinite else 0)
        return self

    def info(self) -> dict:
        return swept_plan_info(self._h)

    def close(self):
        if self._h:
            swept_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


__all__ = ["Plan", "SweptError", "swept_plan_create", "swept_run", "swept_run_noalloc", "naive_run", "swept_plan_info",
           "swept_plan_set_engine", "swept_plan_set_checks", "swept_batch_set_checks", "swept_plan_destroy", "swept_last_error", "swept_schedule",
           "swept_tile_geometry", "swept_autotune", "swept_autotune_lookup", "swept_autotune_forget",
           "Batch", "swept_batch_create", "swept_batch_run", "swept_batch_set_engine", "swept_batch_info",
           "swept_batch_destroy",
           "AdjointPlan", "swept_heat", "swept_adjoint_create", "swept_adjoint_create_segmented", "swept_forward_ckpt", "swept_adjoint_run",
           "swept_adjoint_info", "swept_adjoint_destroy", "release_cached_plans"]
