"""Pins for the CPU oracle against facts that do not come from the oracle itself.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
flipped sign, a shifted index, a transposed neighbour, forward Euler instead of
RK2, u_x^2 instead of (u^2)_x, a broken wrap-around) fails at least one of them:

heat FTCS (Eq. HeatDisc)
  * discrete Fourier amplification G_k = 1 - 4 Fo sin^2(pi k / N) per mode,
    applied through an FFT to arbitrary data                    (closed form)
  * at Fo = 1/4 the scheme is a binomial filter: exact integer arithmetic
    on small integer grids, compared bit for bit                 (brute force)
  * sum(u) is conserved on the periodic ring                     (invariant)
  * translation equivariance and mirror symmetry, bit for bit    (invariant)
Kuramoto-Sivashinsky (Eq. KSDisc, RK2 midpoint of the Appendix)
  * a constant state is a fixed point, exactly                   (special case)
  * small-amplitude modes grow by 1 + z + z^2/2 per step with
    z = dt (4 s / dx^2 - 16 s^2 / dx^4), s = sin^2(pi k / N)     (closed form)
  * one step from a smooth field reproduces -(u u_x + u_xx + u_xxxx)
    of the continuous equation to O(dt + dx^2)                   (consistency)
  * sum(u) is conserved                                          (invariant)
  * translation equivariance bit for bit; u -> -u(-x) symmetry   (invariant)
heat adjoint
  * dJ/du0 = A^T (u_T - y) through the FFT                       (closed form)
  * dJ/dalpha = T (dt/dx^2) <u_T - y, L u_{T-1}>, L the periodic
    second difference (A and L commute)                          (closed form)
  * central finite differences of J computed with the forward oracle
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import inputs

EPS = np.finfo(np.float64).eps


# ------------------------------------------------------------------ heat --

def _heat_fft(u0, fo, steps):
    n = u0.size
    k = np.arange(n)
    g = 1.0 - 4.0 * fo * np.sin(np.pi * k / n) ** 2
    return np.real(np.fft.ifft(np.fft.fft(u0) * g ** steps))


@pytest.mark.parametrize("fo", [0.25, 0.1, 0.4, 0.49])
@pytest.mark.parametrize("k", [1, 3, 17, 31])
def test_heat_single_mode_amplification(fo, k):
    n, steps = 64, 200
    dx = 1.0 / n
    dt = fo * dx * dx  # alpha = 1
    i = np.arange(n)
    u0 = np.sin(2 * np.pi * k * i / n)
    got = oracle.heat(u0, 1.0, dt, dx, steps)
    fo_eff = (1.0 * dt) / (dx * dx)
    g = 1.0 - 4.0 * fo_eff * math.sin(math.pi * k / n) ** 2
    want = g ** steps * u0
    assert np.max(np.abs(got - want)) <= 4 * steps * EPS * max(1.0, abs(g) ** steps) + 1e-300


def test_heat_fft_closed_form_small_workload():
    p = inputs.heat_small()
    got = oracle.heat(p.u0, p.alpha, p.dt, p.dx, p.steps)
    want = _heat_fft(p.u0, 0.25, p.steps)
    rel = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert rel <= 1e-12, rel


def test_heat_fft_closed_form_mode_sum():
    n, steps = 4096, 1500
    p = inputs.heat_large(n=n, steps=steps)
    got = oracle.heat(p.u0, p.alpha, p.dt, p.dx, steps)
    want = _heat_fft(p.u0, 0.25, steps)
    rel = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert rel <= 1e-12, rel


@pytest.mark.parametrize("steps", [0, 1, 2, 7, 15, 20])
def test_heat_binomial_exact_fo_quarter(steps):
    # Fo = 1/4: T_i^{m+1} = (T_{i-1} + 2 T_i + T_{i+1}) / 4, so after m steps
    # u_m[i] = 4^-m sum_j C(2m, j) u0[(i - m + j) mod n].  Integer data keeps
    # every FP64 intermediate exact, so the oracle must agree bit for bit.
    n = 16
    u0 = inputs.dyadic_grid(n, seed=11)
    dx = 2.0 ** -4
    dt = dx * dx / 4.0
    got = oracle.heat(u0, 1.0, dt, dx, steps)
    ints = [int(v) for v in u0]
    want = []
    for i in range(n):
        acc = sum(math.comb(2 * steps, j) * ints[(i - steps + j) % n] for j in range(2 * steps + 1))
        want.append(Fraction(acc, 4 ** steps))
    assert [Fraction(v) for v in got] == want


@pytest.mark.parametrize("steps", [1, 2, 7, 9])
def test_heat_binomial_exact_fo_quarter_f32(steps):
    # The same binomial closed form in single precision: with integers in
    # [-64, 64] every intermediate of up to 9 steps is k / 4^t with |k| <= 2^24,
    # so FP32 arithmetic is exact too and the FP32 oracle must match bit for bit.
    n = 16
    u0 = inputs.dyadic_grid(n, seed=12)
    dx = 2.0 ** -4
    dt = dx * dx / 4.0
    got = oracle.heat(u0, 1.0, dt, dx, steps, dtype=np.float32)
    assert got.dtype == np.float32
    ints = [int(v) for v in u0]
    for i in range(n):
        acc = sum(math.comb(2 * steps, j) * ints[(i - steps + j) % n] for j in range(2 * steps + 1))
        assert Fraction(float(got[i])) == Fraction(acc, 4 ** steps), i


def test_heat_conservation():
    n, steps, fo = 256, 500, 0.3
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-1, 1, n)
    dx = 1.0 / n
    got = oracle.heat(u0, 1.0, fo * dx * dx, dx, steps)
    assert abs(got.sum() - u0.sum()) <= 4 * steps * n * EPS
    # integer data at Fo = 1/4: exact
    ui = inputs.dyadic_grid(n, seed=3)
    gi = oracle.heat(ui, 1.0, dx * dx / 4, dx, 12)
    assert math.fsum(gi) == math.fsum(ui)


def test_heat_translation_and_mirror_bitwise():
    n, steps = 97, 60  # odd n exercises the wrap on both sides
    rng = np.random.default_rng(6)
    u0 = rng.standard_normal(n)
    dx = 1.0 / n
    dt = 0.37 * dx * dx
    base = oracle.heat(u0, 1.0, dt, dx, steps)
    for s in (1, 5, 50):
        assert np.array_equal(oracle.heat(np.roll(u0, s), 1.0, dt, dx, steps), np.roll(base, s))
    assert np.array_equal(oracle.heat(u0[::-1], 1.0, dt, dx, steps), base[::-1])


def test_heat_f32_tracks_f64():
    p = inputs.heat_small()
    g64 = oracle.heat(p.u0, p.alpha, p.dt, p.dx, p.steps)
    g32 = oracle.heat(p.u0, p.alpha, p.dt, p.dx, p.steps, dtype=np.float32)
    assert g32.dtype == np.float32
    rel = np.max(np.abs(g32.astype(np.float64) - g64)) / np.max(np.abs(g64))
    assert 1e-9 < rel < 1e-5


# -------------------------------------------------------------------- KS --

def test_ks_constant_state_fixed_point():
    u0 = np.full(32, 3.0)
    got = oracle.ks(u0, 0.005, 0.5, 100)
    assert np.array_equal(got, u0)


@pytest.mark.parametrize("k", [1, 2, 5, 11, 16, 31, 32])
def test_ks_linear_mode_rk2_amplification(k):
    # Small amplitude: the nonlinear flux is O(amp^2) and drops below rounding.
    n, steps, dt, dx, amp = 64, 50, 0.005, 0.5, 1e-8
    i = np.arange(n)
    phase = 0.3
    u0 = amp * np.cos(2 * np.pi * k * i / n + phase)
    got = oracle.ks(u0, dt, dx, steps)
    s = math.sin(math.pi * k / n) ** 2
    z = dt * (4 * s / dx ** 2 - 16 * s ** 2 / dx ** 4)
    g = 1 + z + z * z / 2
    want = g ** steps * u0
    assert np.max(np.abs(got - want)) <= 1e-6 * amp * max(1.0, abs(g) ** steps)


def test_ks_linear_mode_rejects_forward_euler():
    # At the highest mode z = -1.2: RK2 gives 0.52 per step, forward Euler -0.2.
    n, dt, dx = 64, 0.005, 0.5
    i = np.arange(n)
    u0 = 1e-8 * np.cos(np.pi * i)  # k = n/2
    got = oracle.ks(u0, dt, dx, 1)
    ratio = got[0] / u0[0]
    assert abs(ratio - 0.52) < 1e-9


def test_ks_one_step_consistency_with_pde():
    # u = sin(2x) on [0, 2 pi):  u u_x = sin(4x),  u_xx = -4 sin 2x,
    # u_xxxx = 16 sin 2x, so u_t = -(sin 4x + 12 sin 2x).
    n = 256
    dx = 2 * math.pi / n
    dt = 1e-10
    x = np.arange(n) * dx
    u0 = np.sin(2 * x)
    got = oracle.ks(u0, dt, dx, 1)
    rate = (got - u0) / dt
    want = -(np.sin(4 * x) + 12 * np.sin(2 * x))
    err = np.max(np.abs(rate - want)) / np.max(np.abs(want))
    assert err < 1e-2, err
    # the "1/2 u_x^2" misreading of the nonlinear term would give -(2 cos^2 2x + 12 sin 2x)
    wrong = -(2 * np.cos(2 * x) ** 2 + 12 * np.sin(2 * x))
    assert np.max(np.abs(rate - wrong)) / np.max(np.abs(want)) > 0.05


def test_ks_conservation():
    n, steps = 128, 400
    p = inputs.ks(n=n, steps=steps)
    got = oracle.ks(p.u0, p.dt, p.dx, steps)
    scale = np.max(np.abs(p.u0)) + np.max(np.abs(got))
    assert abs(got.sum() - p.u0.sum()) <= 64 * steps * n * EPS * scale


def test_ks_translation_bitwise_and_parity_symmetry():
    n, steps = 67, 80
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal(n)
    base = oracle.ks(u0, 0.005, 0.5, steps)
    for s in (1, 2, 33):
        assert np.array_equal(oracle.ks(np.roll(u0, s), 0.005, 0.5, steps), np.roll(base, s))
    # if u(x, t) solves KS then so does -u(-x, t)
    mirrored = -np.roll(u0[::-1], 1)  # v_i = -u_{-i mod n}
    got = oracle.ks(mirrored, 0.005, 0.5, steps)
    want = -np.roll(base[::-1], 1)
    # the order of every sum is symmetric and the flux term antisymmetric, so
    # the mirror is exact
    assert np.array_equal(got, want)


def test_ks_f32_translation_bitwise():
    # the FP32 path is as shift-invariant as the FP64 one: rolling the input
    # rolls the output bit for bit (every point gets the same operations)
    p = inputs.ks(n=200, steps=60)
    base = oracle.ks(p.u0, p.dt, p.dx, p.steps, dtype=np.float32)
    for s in (1, 3, 199):
        got = oracle.ks(np.roll(p.u0, s), p.dt, p.dx, p.steps, dtype=np.float32)
        assert np.array_equal(got, np.roll(base, s))


def test_ks_f32_tracks_f64_short_horizon():
    p = inputs.ks(n=256, steps=200)
    g64 = oracle.ks(p.u0, p.dt, p.dx, p.steps)
    g32 = oracle.ks(p.u0, p.dt, p.dx, p.steps, dtype=np.float32)
    rel = np.max(np.abs(g32.astype(np.float64) - g64)) / np.max(np.abs(g64))
    assert rel < 1e-4


# ---------------------------------------------------------- heat adjoint --

def _adjoint_case(n=32, steps=50, alpha=0.3, seed=21):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    dt = dx * dx
    u0 = rng.standard_normal(n)
    y = rng.standard_normal(n)
    return u0, y, alpha, dt, dx, steps


def test_adjoint_closed_forms():
    u0, y, alpha, dt, dx, steps = _adjoint_case()
    n = u0.size
    J, g, ga = oracle.heat_adjoint(u0, y, alpha, dt, dx, steps)
    fo = alpha * dt / (dx * dx)
    uT = _heat_fft(u0, fo, steps)
    lamT = uT - y
    assert abs(J - 0.5 * np.sum(lamT ** 2)) <= 1e-12 * max(1.0, J)
    want_g = _heat_fft(lamT, fo, steps)  # A symmetric and circulant
    assert np.max(np.abs(g - want_g)) <= 1e-12 * np.max(np.abs(want_g))
    uT1 = _heat_fft(u0, fo, steps - 1)
    k = np.arange(n)
    lap = np.real(np.fft.ifft(np.fft.fft(uT1) * (-4.0 * np.sin(np.pi * k / n) ** 2)))
    want_ga = steps * (dt / (dx * dx)) * np.dot(lamT, lap)
    assert abs(ga - want_ga) <= 1e-10 * abs(want_ga)


def test_adjoint_checkpoint_invariance():
    u0, y, alpha, dt, dx, steps = _adjoint_case(n=40, steps=37)
    ref = oracle.heat_adjoint(u0, y, alpha, dt, dx, steps, ckpt=1)
    for K in (0, 5, 36, 37, 100):
        got = oracle.heat_adjoint(u0, y, alpha, dt, dx, steps, ckpt=K)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1])
        assert abs(got[2] - ref[2]) <= 1e-13 * abs(ref[2])


def test_adjoint_central_differences():
    u0, y, alpha, dt, dx, steps = _adjoint_case()
    J, g, ga = oracle.heat_adjoint(u0, y, alpha, dt, dx, steps)

    def jval(u, a):
        uT = oracle.heat(u, a, dt, dx, steps)
        return 0.5 * math.fsum((uT - y) ** 2)

    h = 1e-6
    fd = (jval(u0, alpha + h) - jval(u0, alpha - h)) / (2 * h)
    assert abs(fd - ga) <= 1e-6 * max(abs(ga), 1e-3)
    rng = np.random.default_rng(22)
    for _ in range(4):
        d = rng.standard_normal(u0.size)
        d /= np.linalg.norm(d)
        fdu = (jval(u0 + h * d, alpha) - jval(u0 - h * d, alpha)) / (2 * h)
        assert abs(fdu - np.dot(g, d)) <= 1e-6 * max(abs(np.dot(g, d)), 1e-3)


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
@pytest.mark.parametrize("n", [5, 97, 4096, 30011])
def test_all_cores_oracle_gives_the_single_thread_bits(n, threads):
    # the OpenMP leg used for the CPU baseline on all host cores splits each
    # step's points over threads; every point's update is unchanged, so the
    # result is the single-thread oracle's bit for bit
    u = np.random.default_rng(n).standard_normal(n)
    a = oracle.heat(u, 1.0, 0.2 / n / n, 1.0 / n, 37)
    b, used = oracle.heat_mt(u, 1.0, 0.2 / n / n, 1.0 / n, 37, threads=threads)
    assert used == threads and np.array_equal(a, b)
    a = oracle.ks(u, 0.005, 0.5, 11)
    b, used = oracle.ks_mt(u, 0.005, 0.5, 11, threads=threads)
    assert used == threads and np.array_equal(a, b)
