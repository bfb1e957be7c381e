"""Pins of the KS adjoint oracle (reverse sweep of the periodic KS RK2 scheme,
arXiv 1612.02495 Sec. 4.1 and Appendix, for J = 1/2 ||u_T - y||^2).

None of these calls the oracle's own Jacobian code twice:
  * J itself from the (separately pinned) forward KS oracle;
  * central finite differences of that forward oracle along random
    directions, at two step sizes (second-order agreement);
  * the zero state: f(0) = 0 and the Jacobian there is the circulant linear
    part, so dJ/du0 = IFFT(G_k^T FFT(-y)) with G_k = 1 + z + z^2/2,
    z = dt (4 s / dx^2 - 16 s^2 / dx^4), s = sin^2(pi k / N);
  * the dot-product identity <dJ/du0, d> = <u_T - y, M d> with M the
    tangent-linear model of the scheme, written here from the forward
    formulas (Jacobian-vector products, not transposes);
  * invariance to the checkpoint interval (bit for bit).
"""
import numpy as np
import pytest

import oracle

DT, DX = 0.005, 0.5


def _ks_state(n, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(n) * DX
    return np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0)) + 1e-3 * rng.standard_normal(n), rng


def _J(u0, y, steps):
    v = oracle.ks(u0, DT, DX, steps)
    return 0.5 * float(np.sum((v - y) ** 2))


def test_objective_matches_forward_oracle():
    u0, rng = _ks_state(96, 1)
    y = 0.1 * rng.standard_normal(u0.size)
    J, _ = oracle.ks_adjoint(u0, y, DT, DX, 150)
    assert abs(J - _J(u0, y, 150)) <= 1e-13 * J


@pytest.mark.parametrize("steps", [1, 37, 200])
def test_central_differences(steps):
    u0, rng = _ks_state(64, steps)
    y = 0.1 * rng.standard_normal(u0.size)
    _, g = oracle.ks_adjoint(u0, y, DT, DX, steps)
    for _ in range(4):
        d = rng.standard_normal(u0.size)
        errs = []
        for h in (1e-3, 1e-4, 1e-5):
            fd = (_J(u0 + h * d, y, steps) - _J(u0 - h * d, y, steps)) / (2 * h)
            errs.append(abs(fd - g @ d) / abs(g @ d))
        assert min(errs[1:]) <= 1e-8
        # truncation-dominated between 1e-3 and 1e-4: second order, about 100x closer
        assert errs[1] <= errs[0] / 10


def test_zero_state_closed_form():
    n, steps = 128, 60
    rng = np.random.default_rng(5)
    y = rng.standard_normal(n)
    J, g = oracle.ks_adjoint(np.zeros(n), y, DT, DX, steps)
    assert J == pytest.approx(0.5 * float(y @ y), rel=1e-15)
    s = np.sin(np.pi * np.arange(n) / n) ** 2
    z = DT * (4.0 * s / DX ** 2 - 16.0 * s ** 2 / DX ** 4)
    want = np.real(np.fft.ifft((1.0 + z + z * z / 2.0) ** steps * np.fft.fft(-y)))
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def _jv(v, d):
    """Jacobian of the KS right-hand side at v applied to d (forward form)."""
    i4dx, idx2 = 1.0 / (4.0 * DX), 1.0 / (DX * DX)
    idx4 = idx2 * idx2
    r = lambda a, k: np.roll(a, -k)  # r(a, k)[i] = a[i + k]
    nl = 2.0 * i4dx * (r(v, 1) * r(d, 1) - r(v, -1) * r(d, -1))
    d2 = idx2 * (r(d, 1) + r(d, -1) - 2.0 * d)
    d4 = idx4 * (r(d, 2) - 4.0 * r(d, 1) + 6.0 * d - 4.0 * r(d, -1) + r(d, -2))
    return -(nl + d2 + d4)


def _rhs(v):
    i4dx, idx2 = 1.0 / (4.0 * DX), 1.0 / (DX * DX)
    idx4 = idx2 * idx2
    r = lambda a, k: np.roll(a, -k)
    return -((r(v, 1) ** 2 - r(v, -1) ** 2) * i4dx + (r(v, 1) + r(v, -1) - 2 * v) * idx2
             + (r(v, 2) - 4 * r(v, 1) + 6 * v - 4 * r(v, -1) + r(v, -2)) * idx4)


def test_dot_product_with_tangent_linear_model():
    n, steps = 80, 120
    u0, rng = _ks_state(n, 9)
    y = 0.1 * rng.standard_normal(n)
    _, g = oracle.ks_adjoint(u0, y, DT, DX, steps)
    d0 = rng.standard_normal(n)
    u, d = u0.copy(), d0.copy()
    for _ in range(steps):
        q = u + 0.5 * DT * _rhs(u)
        dq = d + 0.5 * DT * _jv(u, d)
        d = d + DT * _jv(q, dq)
        u = u + DT * _rhs(q)
    lhs = float(g @ d0)
    rhs = float((u - y) @ d)
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)


def test_checkpoint_interval_does_not_change_bits():
    u0, rng = _ks_state(72, 3)
    y = 0.1 * rng.standard_normal(u0.size)
    ref = oracle.ks_adjoint(u0, y, DT, DX, 97, ckpt=0)
    for c in (1, 5, 97, 500):
        J, g = oracle.ks_adjoint(u0, y, DT, DX, 97, ckpt=c)
        assert J == ref[0] and np.array_equal(g, ref[1])
