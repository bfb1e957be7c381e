"""Seeded synthetic inputs for the swept heat / Kuramoto-Sivashinsky workloads.

This module holds no arithmetic of the method: it only draws random numbers
and evaluates initial conditions on the host in NumPy FP64.  Both the CPU
oracle (through the tests) and the HIP path consume what it returns, so the
two are compared on identical inputs.  Importing it never loads the HIP
library.

Workloads (the paper's grids are powers of two from 2^11 to 2^20, Sec. 5;
its heat problem is a 1-D rod and its KS problem a periodic chaotic field,
Sec. 4.1):

* ``heat_small``   N=1024, dx=2^-10, alpha=1, dt=dx^2/4 (Fo=1/4 exactly),
                   u0 = sin(2 pi x) + 0.01 N(0,1), 1000 steps, tile width 64.
* ``heat_large``   N=2^20, dx=2^-20, dt=2^-42, alpha=1 (Fo=1/4 exactly),
                   u0 = sum of 8 Fourier modes with amplitudes U(-1,1).
* ``ks``           dx=0.5, dt=0.005, x_i=0.5 i,
                   u0 = cos(x/16)(1+sin(x/16)) + 1e-3 N(0,1).
* ``heat_batch``   independent periodic heat problems with N log-uniform in
                   [2^8, 2^16], Fo ~ U(0.05, 0.45), mode-sum initial states.
* ``heat_rod``     the rod with insulated ends of Sec. 4.1: n nodes on [0, 1]
                   (dx = 1/(n-1)), alpha=1, dt=dx^2/4 (Fo=1/4 exactly), an
                   initial temperature gradient u0 = x plus 8 cosine modes
                   with amplitudes 0.1 U(-1,1).
* ``heat_adjoint`` batch of N=2^18 heat problems, dt=dx^2 so Fo = alpha,
                   alpha ~ U(0.05, 0.45), mode-sum u0, target from a
                   perturbed forward run.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(seed))


def mode_sum(n: int, rng: np.random.Generator, nmodes: int = 8):
    """u0_i = sum_j a_j sin(2 pi k_j i / n), a_j ~ U(-1,1), k_j distinct integers
    floor(2^U(0, log2(n) - 3)) (slowly and quickly decaying modes)."""
    hi = max(np.log2(n) - 3.0, 1.0)
    ks: list[int] = []
    guard = 0
    while len(ks) < nmodes and guard < 10000:
        k = int(np.floor(2.0 ** rng.uniform(0.0, hi)))
        k = max(1, min(k, n // 2 - 1 if n > 3 else 1))
        if k not in ks:
            ks.append(k)
        guard += 1
    amps = rng.uniform(-1.0, 1.0, size=len(ks))
    i = np.arange(n, dtype=np.float64)
    u = np.zeros(n, dtype=np.float64)
    for a, k in zip(amps, ks):
        u += a * np.sin(2.0 * np.pi * k * i / n)
    return u, np.array(ks, dtype=np.int64), amps


@dataclass
class Problem:
    kind: str  # "heat" or "ks"
    n: int
    dt: float
    dx: float
    alpha: float
    steps: int
    u0: np.ndarray
    tile_width: int = 0
    modes: np.ndarray | None = None
    amps: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def heat_small(seed: int = 0, steps: int = 1000) -> Problem:
    n = 1024
    dx = 2.0 ** -10
    dt = dx * dx / 4.0
    rng = _rng(seed)
    x = np.arange(n, dtype=np.float64) * dx
    u0 = np.sin(2.0 * np.pi * x) + 0.01 * rng.standard_normal(n)
    return Problem("heat", n, dt, dx, 1.0, steps, u0, tile_width=64)


def heat_large(seed: int = 1, n: int = 2 ** 20, steps: int = 100000) -> Problem:
    dx = 1.0 / n
    dt = dx * dx / 4.0
    rng = _rng(seed)
    u0, ks_, amps = mode_sum(n, rng)
    return Problem("heat", n, dt, dx, 1.0, steps, u0, modes=ks_, amps=amps)


def heat_rod(n: int = 2 ** 20, seed: int = 8, steps: int = 100000) -> Problem:
    """Insulated rod (Sec. 4.1): a temperature gradient plus cosine modes,
    which are the rod's own eigenmodes (cos(pi k i/(n-1)))."""
    dx = 1.0 / (n - 1)
    dt = dx * dx / 4.0
    rng = _rng(seed)
    i = np.arange(n, dtype=np.float64)
    ks_ = rng.choice(np.arange(1, max(2, n // 8)), size=min(8, max(1, n // 8 - 1)), replace=False)
    amps = 0.1 * rng.uniform(-1.0, 1.0, size=ks_.size)
    u0 = i * dx
    for a, k in zip(amps, ks_):
        u0 = u0 + a * np.cos(np.pi * k * i / (n - 1))
    return Problem("heat_insulated", n, dt, dx, 1.0, steps, u0, modes=ks_, amps=amps)


def ks(n: int = 2 ** 16, seed: int = 2, steps: int = 20000) -> Problem:
    dx = 0.5
    dt = 0.005
    rng = _rng(seed)
    x = np.arange(n, dtype=np.float64) * dx
    u0 = np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0)) + 1e-3 * rng.standard_normal(n)
    return Problem("ks", n, dt, dx, 0.0, steps, u0)


def batch_sizes(rng: np.random.Generator, nprob: int, nmin_log2: float = 8.0, nmax_log2: float = 16.0) -> np.ndarray:
    """N_p = round(2^U(nmin, nmax)): log-uniform integer grid sizes."""
    raw = 2.0 ** rng.uniform(nmin_log2, nmax_log2, size=nprob)
    return np.rint(raw).astype(np.int64)


def heat_batch(nprob: int = 4096, seed: int = 3, steps: int = 5000, nmin_log2: float = 8.0,
               nmax_log2: float = 16.0) -> list[Problem]:
    ss = np.random.SeedSequence(seed)
    top = np.random.default_rng(ss)
    sizes = batch_sizes(top, nprob, nmin_log2, nmax_log2)
    fos = top.uniform(0.05, 0.45, size=nprob)
    out = []
    for p, child in enumerate(ss.spawn(nprob)):
        n = int(sizes[p])
        dx = 1.0 / n
        dt = float(fos[p]) * dx * dx
        u0, ks_, amps = mode_sum(n, np.random.default_rng(child))
        out.append(Problem("heat", n, dt, dx, 1.0, steps, u0, modes=ks_, amps=amps,
                           extra={"fo_drawn": float(fos[p])}))
    return out


def ks_batch(nprob: int = 4096, seed: int = 6, steps: int = 5000, nmin_log2: float = 8.0,
             nmax_log2: float = 16.0) -> list[Problem]:
    """Independent periodic KS problems (dx = 0.5, dt = 0.005) of log-uniform size,
    u0 = cos(x/16)(1 + sin(x/16)) + 1e-3 N(0,1) on each ring."""
    ss = np.random.SeedSequence(seed)
    top = np.random.default_rng(ss)
    sizes = batch_sizes(top, nprob, nmin_log2, nmax_log2)
    out = []
    for p, child in enumerate(ss.spawn(nprob)):
        n = int(sizes[p])
        rng = np.random.default_rng(child)
        x = np.arange(n, dtype=np.float64) * 0.5
        u0 = np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0)) + 1e-3 * rng.standard_normal(n)
        out.append(Problem("ks", n, 0.005, 0.5, 0.0, steps, u0))
    return out


def heat_adjoint(batch: int = 64, n: int = 2 ** 18, seed: int = 4, target_seed: int = 5,
                 steps: int = 10000):
    """Returns (u0[batch,n], alpha[batch], u0_target_source[batch,n],
    alpha_target[batch], dt, dx, steps).  The target y is produced by running
    the forward scheme from the second state with the perturbed alphas."""
    dx = 1.0 / n
    dt = dx * dx
    rng = _rng(seed)
    alpha = rng.uniform(0.05, 0.45, size=batch)
    u0 = np.stack([mode_sum(n, rng)[0] for _ in range(batch)])
    rt = _rng(target_seed)
    u0t = np.stack([mode_sum(n, rt)[0] for _ in range(batch)])
    alpha_t = alpha * (1.0 + 0.1 * rt.uniform(-1.0, 1.0, size=batch))
    return u0, alpha, u0t, alpha_t, dt, dx, steps


def ks_adjoint(batch: int = 1, n: int = 2 ** 20, seed: int = 6, target_seed: int = 7, steps: int = 20000):
    """Returns (u0[batch,n], u0_target_source[batch,n], dt, dx, steps) for the KS
    gradient workload: the KS initial state of the forward workload (dx = 0.5,
    dt = 0.005) with seeded noise per grid; the target y is produced by running
    the forward scheme from the second set of states."""
    dx = 0.5
    dt = 0.005
    x = np.arange(n, dtype=np.float64) * dx
    base = np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0))
    rng = _rng(seed)
    u0 = np.stack([base + 1e-3 * rng.standard_normal(n) for _ in range(batch)])
    rt = _rng(target_seed)
    u0t = np.stack([base + 1e-3 * rt.standard_normal(n) for _ in range(batch)])
    return u0, u0t, dt, dx, steps

def dyadic_grid(n: int, seed: int, lo: int = -64, hi: int = 64) -> np.ndarray:
    """Small integer-valued grid: every FTCS step at Fo = 1/4 is then exact in FP64."""
    return _rng(seed).integers(lo, hi + 1, size=n).astype(np.float64)
