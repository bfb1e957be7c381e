"""CPU oracle (test infrastructure only).

Plain FP64 (and FP32) timesteppers for the periodic heat FTCS and
Kuramoto-Sivashinsky RK2 schemes of Magee & Niemeyer (arXiv 1612.02495,
Sec. 4.1 Eq. HeatDisc and Eq. KSDisc, Appendix), plus an FP64 reverse sweep
for the heat adjoint.  The arithmetic lives in ``oracle.c`` (plain C, built
with ``-O2 -ffp-contract=off``); this module only builds and calls it.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and this package never
imports the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, dbl = ctypes.c_int64, ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        pf = ctypes.POINTER(ctypes.c_float)
        lib.oracle_heat_f64.argtypes = [pd, i64, dbl, dbl, dbl, i64]
        lib.oracle_heat_f32.argtypes = [pf, i64, dbl, dbl, dbl, i64]
        lib.oracle_heat_insulated_f64.argtypes = [pd, i64, dbl, dbl, dbl, i64]
        lib.oracle_heat_insulated_f32.argtypes = [pf, i64, dbl, dbl, dbl, i64]
        lib.oracle_ks_f64.argtypes = [pd, i64, dbl, dbl, i64]
        lib.oracle_ks_f32.argtypes = [pf, i64, dbl, dbl, i64]
        lib.oracle_heat_adjoint_f64.argtypes = [pd, pd, i64, dbl, dbl, dbl, i64, i64, pd, pd, pd]
        pi = ctypes.POINTER(ctypes.c_int)
        lib.oracle_heat_f64_mt.argtypes = [pd, i64, dbl, dbl, dbl, i64, ctypes.c_int, pi]
        lib.oracle_ks_f64_mt.argtypes = [pd, i64, dbl, dbl, i64, ctypes.c_int, pi]
        lib.oracle_ks_adjoint_f64.argtypes = [pd, pd, i64, dbl, dbl, i64, i64, pd, pd]
        for f in (lib.oracle_heat_f64, lib.oracle_heat_f32, lib.oracle_heat_insulated_f64,
                  lib.oracle_heat_insulated_f32, lib.oracle_ks_f64, lib.oracle_ks_f32,
                  lib.oracle_heat_adjoint_f64, lib.oracle_ks_adjoint_f64, lib.oracle_heat_f64_mt,
                  lib.oracle_ks_f64_mt):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(u, dtype):
    a = np.array(u, dtype=dtype, copy=True, order="C")
    if a.ndim != 1:
        raise ValueError("oracle takes a 1-D grid")
    return a


def _ptr(a):
    ct = ctypes.c_double if a.dtype == np.float64 else ctypes.c_float
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


def heat(u0, alpha: float, dt: float, dx: float, steps: int, dtype=np.float64) -> np.ndarray:
    """Periodic heat FTCS (Eq. HeatDisc), `steps` full timesteps; returns a new array."""
    lib = _load()
    a = _arr(u0, dtype)
    f = lib.oracle_heat_f64 if a.dtype == np.float64 else lib.oracle_heat_f32
    _check(f(_ptr(a), a.size, float(alpha), float(dt), float(dx), int(steps)), "oracle_heat")
    return a


def heat_insulated(u0, alpha: float, dt: float, dx: float, steps: int, dtype=np.float64) -> np.ndarray:
    """Heat FTCS on a rod with insulated ends (Sec. 4.1): mirror ghosts about
    the end nodes, u[-1] = u[1] and u[n] = u[n-2]; `steps` full timesteps."""
    lib = _load()
    a = _arr(u0, dtype)
    f = lib.oracle_heat_insulated_f64 if a.dtype == np.float64 else lib.oracle_heat_insulated_f32
    _check(f(_ptr(a), a.size, float(alpha), float(dt), float(dx), int(steps)), "oracle_heat_insulated")
    return a


def ks(u0, dt: float, dx: float, steps: int, dtype=np.float64) -> np.ndarray:
    """Periodic Kuramoto-Sivashinsky, 5-point central differences, RK2 midpoint."""
    lib = _load()
    a = _arr(u0, dtype)
    f = lib.oracle_ks_f64 if a.dtype == np.float64 else lib.oracle_ks_f32
    _check(f(_ptr(a), a.size, float(dt), float(dx), int(steps)), "oracle_ks")
    return a


def heat_mt(u0, alpha: float, dt: float, dx: float, steps: int, threads: int = 0):
    """heat() in FP64 with each step's points split over host threads (OpenMP);
    the same bits as heat().  Returns (array, threads used)."""
    lib = _load()
    a = _arr(u0, np.float64)
    used = ctypes.c_int(0)
    _check(lib.oracle_heat_f64_mt(_ptr(a), a.size, float(alpha), float(dt), float(dx), int(steps), int(threads),
                                  ctypes.byref(used)), "oracle_heat_f64_mt")
    return a, used.value


def ks_mt(u0, dt: float, dx: float, steps: int, threads: int = 0):
    """ks() in FP64 with each sub-step's points split over host threads
    (OpenMP); the same bits as ks().  Returns (array, threads used)."""
    lib = _load()
    a = _arr(u0, np.float64)
    used = ctypes.c_int(0)
    _check(lib.oracle_ks_f64_mt(_ptr(a), a.size, float(dt), float(dx), int(steps), int(threads),
                                ctypes.byref(used)), "oracle_ks_f64_mt")
    return a, used.value


def heat_adjoint(u0, y, alpha: float, dt: float, dx: float, steps: int, ckpt: int = 0):
    """Returns (J, dJ/du0, dJ/dalpha) for J = 1/2 ||u_T - y||^2, heat FTCS, FP64."""
    lib = _load()
    a = _arr(u0, np.float64)
    yy = _arr(y, np.float64)
    if yy.size != a.size:
        raise ValueError("u0 and y differ in size")
    g = np.zeros_like(a)
    ga = ctypes.c_double(0.0)
    jj = ctypes.c_double(0.0)
    _check(lib.oracle_heat_adjoint_f64(_ptr(a), _ptr(yy), a.size, float(alpha), float(dt), float(dx),
                                       int(steps), int(ckpt), _ptr(g), ctypes.byref(ga),
                                       ctypes.byref(jj)), "oracle_heat_adjoint")
    return jj.value, g, ga.value


def ks_adjoint(u0, y, dt: float, dx: float, steps: int, ckpt: int = 0):
    """Returns (J, dJ/du0) for J = 1/2 ||u_T - y||^2, periodic KS RK2, FP64."""
    lib = _load()
    a = _arr(u0, np.float64)
    yy = _arr(y, np.float64)
    if yy.size != a.size:
        raise ValueError("u0 and y differ in size")
    g = np.zeros_like(a)
    J = ctypes.c_double()
    _check(lib.oracle_ks_adjoint_f64(_ptr(a), _ptr(yy), a.size, float(dt), float(dx), int(steps), int(ckpt),
                                     _ptr(g), ctypes.byref(J)), "oracle_ks_adjoint")
    return J.value, g
