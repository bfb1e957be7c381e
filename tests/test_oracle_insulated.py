"""Pins of the insulated-rod heat oracle (arXiv 1612.02495, Sec. 4.1: a rod
with insulated ends; Appendix: FTCS with mirror ghosts at both ends).

Each pin checks the oracle against something other than its own code:
  * the even extension: an insulated rod of n nodes evolves exactly as the
    periodic ring of 2(n-1) nodes built by reflecting it about both end nodes
    (the periodic oracle is pinned on its own in test_oracle_pins.py);
  * the discrete cosine modes cos(pi k i/(n-1)), eigenvectors of the mirrored
    operator with amplification 1 - 4 Fo sin^2(pi k / (2(n-1)));
  * conservation of the trapezoid-weighted sum u_0/2 + u_1 + .. + u_{n-2} +
    u_{n-1}/2 (exact for dyadic data at Fo = 1/4);
  * exact brute force at Fo = 1/4 with Python integers: T steps of the
    binomial filter [1 2 1]/4 on the even extension;
  * symmetry: a rod symmetric about its middle stays exactly symmetric.
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle


def _even_extension(u):
    u = np.asarray(u)
    return np.concatenate([u, u[-2:0:-1]])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [2, 3, 5, 16, 37, 1024])
def test_equals_periodic_even_extension(n, dtype):
    rng = np.random.default_rng(n)
    u0 = rng.standard_normal(n)
    dx = 1.0 / n
    dt = 0.37 * dx * dx
    steps = 57
    got = oracle.heat_insulated(u0.astype(dtype), 1.0, dt, dx, steps, dtype=dtype)
    ext = _even_extension(u0.astype(dtype))
    ring = oracle.heat(ext, 1.0, dt, dx, steps, dtype=dtype)
    assert np.array_equal(got, ring[:n])
    assert np.array_equal(ring[n:], got[-2:0:-1])  # the reflected half stays the mirror image


@pytest.mark.parametrize("k", [0, 1, 3, 17, 62])
def test_cosine_modes_decay_by_their_amplification(k):
    n, steps = 64, 300
    fo = 0.3
    i = np.arange(n)
    u0 = np.cos(np.pi * k * i / (n - 1))
    g = 1.0 - 4.0 * fo * np.sin(np.pi * k / (2.0 * (n - 1))) ** 2
    got = oracle.heat_insulated(u0, fo, 1.0, 1.0, steps)
    want = g ** steps * u0
    assert np.max(np.abs(got - want)) <= 1e-12


def test_weighted_sum_conserved():
    rng = np.random.default_rng(4)
    n = 50
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    u0 = rng.integers(-64, 65, size=n).astype(np.float64)
    # Fo = 1/4: every value is a multiple of 4^-T, exact in FP64 while 7 + 2T
    # bits fit in the mantissa; sum in exact rationals
    got = oracle.heat_insulated(u0, 1.0, 0.25, 1.0, 20)
    exact = lambda v: sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(w, v))
    assert exact(got) == exact(u0)
    v0 = rng.standard_normal(n)
    v = oracle.heat_insulated(v0, 1.0, 0.31, 1.0, 500)
    assert abs(w @ v - w @ v0) <= 1e-12 * np.abs(v0).sum()


def test_brute_force_binomial_exact():
    rng = np.random.default_rng(7)
    n, steps = 16, 7
    u0 = [int(v) for v in rng.integers(-64, 65, size=n)]
    ext = u0 + u0[-2:0:-1]
    m = len(ext)
    # T steps of [1 2 1]/4 = binomial(2T) / 4^T, exactly, on the periodic extension
    exact = [sum(comb(2 * steps, j) * ext[(x - steps + j) % m] for j in range(2 * steps + 1)) for x in range(n)]
    got = oracle.heat_insulated(np.array(u0, dtype=np.float64), 1.0, 0.25, 1.0, steps)
    assert [int(round(v * 4 ** steps)) for v in got] == exact
    assert np.array_equal(got * 4.0 ** steps, np.array(exact, dtype=np.float64))


def test_symmetric_rod_stays_symmetric():
    rng = np.random.default_rng(9)
    half = rng.standard_normal(20)
    u0 = np.concatenate([half, half[::-1]])
    got = oracle.heat_insulated(u0, 1.0, 0.21, 1.0, 333)
    assert np.array_equal(got, got[::-1])


def test_differs_from_periodic_and_rejects_tiny_rods():
    rng = np.random.default_rng(2)
    u0 = rng.standard_normal(32)
    assert not np.array_equal(oracle.heat_insulated(u0, 1.0, 0.25, 1.0, 5), oracle.heat(u0, 1.0, 0.25, 1.0, 5))
    with pytest.raises(Exception):
        oracle.heat_insulated(np.zeros(1), 1.0, 0.25, 1.0, 1)
