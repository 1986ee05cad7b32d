"""Pins for the oracle at orders 1 < alpha <= 2 (eq. (1) of arXiv:1611.08678
with ceil(alpha) = 2 initial values: y(0) and y'(0) enter every step through
the Taylor polynomial y(0) + t y'(0); the weights keep their Section 2 forms).

Independent facts used:
  * weights against the product-integration quadrature of the kernel
    (t - s)^(alpha-1)/Gamma(alpha), and at alpha = 2 the closed forms of the
    integrals of s against the cell and hat functions: b_m = m + 1/2,
    a_m = m + 1, c_n = (3n + 2)/6;
  * constant forcing c: y = y(0) + t y'(0) + c t^alpha/Gamma(alpha+1) exactly
    (both rules integrate constants exactly); affine forcing: the corrector
    is exact (product trapezoid on a linear integrand);
  * D^alpha y = -y with (y(0), y'(0)) = (1, 0) and (0, 1): the Mittag-Leffler
    solutions E_alpha(-t^alpha) and t E_{alpha,2}(-t^alpha) (series summed in
    mpmath), error order 2;
  * alpha = 2 is y'' = -y: cos t, order 2;
  * a manufactured smooth solution 1 + 2t + t^4: order 2;
  * tiny N against the 50-digit mpmath implementation with the slope term;
  * batch = single with two initial rows per instance, instances with
    alpha <= 1 ignoring the second row; the teacher-forced single step.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_solver import _mp_pece
from tests.test_oracle_weights import quad_a, quad_b, quad_c


def _lin(A, b0, b1):
    return np.concatenate([np.ravel(A), np.ravel(b0), np.ravel(b1)]).astype(float)


def _ml(a, b, z):
    """Mittag-Leffler E_{a,b}(z) by its power series in 40-digit arithmetic."""
    import mpmath
    mpmath.mp.dps = 40
    z = mpmath.mpf(z)
    s, k = mpmath.mpf(0), 0
    while True:
        t = z ** k / mpmath.gamma(a * k + b)
        s += t
        k += 1
        if k > 10 and abs(t) < mpmath.mpf(10) ** -35:
            return float(s)


@pytest.mark.parametrize("alpha", [1.3, 1.5, 1.9, 2.0])
def test_weights_quadrature_above_one(orc, alpha):
    lags = [0, 1, 2, 3, 16, 17, 100, 1000, 65535]
    b, a, c = orc.weights(alpha, max(lags) + 1)
    for m in lags:
        assert b[m] == pytest.approx(quad_b(m, alpha), rel=2e-13), ("b", m)
        assert a[m] == pytest.approx(quad_a(m, alpha), rel=2e-13), ("a", m)
        assert c[m] == pytest.approx(quad_c(m, alpha), rel=2e-13), ("c", m)


def test_weights_alpha_two_closed_form(orc):
    n = 5000
    b, a, c = orc.weights(2.0, n)
    m = np.arange(n, dtype=np.float64)
    assert np.array_equal(b, m + 0.5)
    assert np.array_equal(a, m + 1.0)
    assert np.allclose(c, (3 * m + 2) / 6, rtol=2e-16, atol=0)


@pytest.mark.parametrize("alpha", [1.3, 1.7, 2.0])
def test_constant_forcing_with_slope_exact(orc, alpha):
    d, N, h = 2, 2000, 0.01
    cst = np.array([1.5, -0.25])
    th = _lin(np.zeros((d, d)), cst, np.zeros(d))
    init = np.array([[0.3, 2.0], [-1.1, 0.6]])
    y, yp, _, st = orc.solve(orc.LINEAR, th, alpha, h, N, init)
    assert st == 0
    t = np.arange(N + 1) * h
    exact = (init[0][None, :] + t[:, None] * init[1][None, :] +
             cst[None, :] * (t ** alpha / math.gamma(alpha + 1))[:, None])
    scale = np.abs(exact).max()
    assert np.abs(y - exact).max() <= 1e-13 * scale
    assert np.abs(yp - exact).max() <= 1e-13 * scale


@pytest.mark.parametrize("alpha", [1.5, 2.0])
def test_affine_forcing_with_slope_corrector_exact(orc, alpha):
    N, h = 2500, 0.004
    c0, c1 = 0.7, -1.3
    y, _, _, st = orc.solve(orc.LINEAR, _lin([[0.0]], [c0], [c1]), alpha, h, N, [[0.5], [-0.8]])
    t = np.arange(N + 1) * h
    exact = (0.5 - 0.8 * t + c0 * t ** alpha / math.gamma(alpha + 1) +
             c1 * t ** (alpha + 1) / math.gamma(alpha + 2))
    assert st == 0
    assert np.abs(y[:, 0] - exact).max() <= 1e-13 * np.abs(exact).max()


@pytest.mark.parametrize("alpha", [1.5, 1.8])
@pytest.mark.parametrize("init", [(1.0, 0.0), (0.0, 1.0)])
def test_mittag_leffler_above_one(orc, alpha, init):
    """D^alpha y = -y on [0, 5]: y(0) E_alpha(-t^alpha) + y'(0) t E_{alpha,2}(-t^alpha)."""
    y0, y1 = init
    errs = []
    for N in (250, 500, 1000):
        h = 5.0 / N
        y, _, _, st = orc.solve(orc.LINEAR, _lin([[-1.0]], [0.0], [0.0]), alpha, h, N,
                                [[y0], [y1]])
        assert st == 0
        t = np.arange(0, N + 1, N // 50) * h
        ex = np.array([y0 * _ml(alpha, 1, -s ** alpha) + y1 * s * _ml(alpha, 2, -s ** alpha)
                       for s in t])
        errs.append(np.abs(y[:: N // 50, 0] - ex).max())
    assert errs[0] < 5e-5  # h = 0.02 (recorded 1.9e-5 .. 4.2e-5)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < o < 2.25 for o in orders), orders


def test_alpha_two_is_second_order_oscillator(orc):
    """alpha = 2, y'' = -y, y(0) = 1, y'(0) = 0: cos t, order 2."""
    errs = []
    for N in (100, 200, 400, 800):
        h = 4.0 / N
        y, _, _, _ = orc.solve(orc.LINEAR, _lin([[-1.0]], [0.0], [0.0]), 2.0, h, N, [[1.0], [0.0]])
        t = np.arange(N + 1) * h
        errs.append(np.abs(y[:, 0] - np.cos(t)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert abs(orders[-1] - 2.0) < 0.05, orders


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_convergence_order_manufactured_quartic(orc, alpha):
    """y = 1 + 2t + t^4 solves D^alpha y = 24 t^(4-alpha)/Gamma(5-alpha) - (y - (1 + 2t + t^4))
    with y(0) = 1, y'(0) = 2 (the Caputo derivative of 1 + 2t vanishes for alpha > 1)."""
    g = math.gamma(5 - alpha)

    def rhs(t, y):
        return [24.0 * t ** (4 - alpha) / g - (y[0] - (1 + 2 * t + t ** 4))]

    errs = []
    for N in (64, 128, 256, 512):
        y, _, _, _ = orc.solve_callback(rhs, alpha, 1.0 / N, N, [[1.0], [2.0]])
        t = np.arange(N + 1) / N
        errs.append(np.abs(y[:, 0] - (1 + 2 * t + t ** 4)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert abs(orders[-1] - 2.0) < 0.1, orders


def test_tiny_n_with_slope_against_mpmath(orc):
    mu = 0.8

    def vdp(t, y):
        return [y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]]

    alpha, h, N = 1.6, 0.05, 12
    init = [[0.4, -1.0], [1.5, 0.25]]
    ref = _mp_pece(vdp, alpha, h, N, init[0], y1=init[1])
    y, _, _, _ = orc.solve(orc.VDP, [mu], alpha, h, N, init)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()


def test_batch_with_two_initial_rows(orc):
    """[B][2][d] initial values: every instance equals its single solve; the
    instances with alpha <= 1 ignore the second row."""
    rng = np.random.default_rng(5)
    B = 6
    alphas = np.array([0.7, 1.2, 1.0, 1.5, 1.9, 2.0])
    Ns = rng.integers(40, 200, B)
    init = rng.uniform(-1, 1, (B, 2, 2))
    th = rng.uniform(0.5, 1.5, (B, 1))
    y, off, st = orc.solve_batch(orc.VDP, th, alphas, np.full(B, 0.01), Ns, init)
    assert np.all(st == 0)
    for i in range(B):
        yi, _, _, _ = orc.solve(orc.VDP, th[i], alphas[i], 0.01, int(Ns[i]), init[i])
        assert np.array_equal(y[off[i]: off[i] + Ns[i] + 1], yi)
        if alphas[i] <= 1.0:
            y1, _, _, _ = orc.solve(orc.VDP, th[i], alphas[i], 0.01, int(Ns[i]), init[i][0])
            assert np.array_equal(yi, y1)


def test_step_from_history_with_slope(orc):
    th = [1.1]
    alpha, h, N = 1.4, 0.01, 700
    init = [[1.0, -0.5], [0.3, 0.8]]
    y, _, f, st = orc.solve(orc.VDP, th, alpha, h, N, init)
    assert st == 0
    wts = orc.weights(alpha, N)
    for t in (1, 2, 256, 257, N):
        yt, _ = orc.step_from_history(orc.VDP, th, alpha, h, t, init, f, wts)
        assert np.array_equal(yt, y[t])
