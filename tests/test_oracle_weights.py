"""Pins for the oracle's weights b_m, a_m, c_m (Section 2 of arXiv:1611.08678,
the predictor weights after eq. (2) and the corrector weights).

Each weight is a product-integration weight: the Riemann-Liouville kernel
(t_{n+1} - s)^(alpha-1) / Gamma(alpha) integrated against a basis function of
the interpolant (a cell indicator for the predictor's product rectangle rule, a
hat function for the corrector's product trapezoid rule). The pins below use
that independent definition (numerical quadrature), the telescoping identities
it implies (zeroth and first moments are exact), and the alpha = 1 limit.
"""
import math

import numpy as np
import pytest
from scipy import integrate

ALPHAS = [0.1, 0.5, 0.8, 0.95, 1.0]
LAGS = [0, 1, 2, 3, 7, 15, 16, 17, 100, 1000, 65535]


def _kernel_integral(lo, hi, g, alpha, singular_at_lo):
    """(1/Gamma(alpha)) * int_lo^hi s^(alpha-1) g(s) ds."""
    if singular_at_lo:
        val, _ = integrate.quad(lambda s: g(s), lo, hi, weight="alg", wvar=(alpha - 1.0, 0.0),
                                epsabs=0, epsrel=2e-14, limit=200)
    else:
        val, _ = integrate.quad(lambda s: s ** (alpha - 1.0) * g(s), lo, hi, epsabs=0,
                                epsrel=2e-14, limit=200)
    return val / math.gamma(alpha)


def quad_b(m, alpha):
    # cell [k, k+1] seen from t_{n+1}, lag m = n - k: s = t_{n+1} - tau in [m, m+1]
    return _kernel_integral(m, m + 1, lambda s: 1.0, alpha, m == 0)


def quad_a(m, alpha):
    # hat centred at source j, lag m = n - j: s in [m, m+2], peak at s = m + 1
    left = _kernel_integral(m, m + 1, lambda s: s - m, alpha, m == 0)
    right = _kernel_integral(m + 1, m + 2, lambda s: m + 2 - s, alpha, False)
    return left + right


def quad_c(n, alpha):
    # half hat at source 0 seen from target n + 1: s in [n, n+1], value s - n
    return _kernel_integral(n, n + 1, lambda s: s - n, alpha, n == 0)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_weights_match_product_integration_quadrature(orc, alpha):
    n = max(LAGS) + 1
    b, a, c = orc.weights(alpha, n)
    for m in LAGS:
        assert b[m] == pytest.approx(quad_b(m, alpha), rel=2e-13), ("b", m)
        assert a[m] == pytest.approx(quad_a(m, alpha), rel=2e-13), ("a", m)
        assert c[m] == pytest.approx(quad_c(m, alpha), rel=2e-13), ("c", m)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.95])
def test_weight_moments_telescope(orc, alpha):
    """Zeroth moment of the rectangle weights and zeroth/first moments of the
    trapezoid weights equal the exact integrals of 1 and s against the kernel."""
    n = 1 << 16
    b, a, c = orc.weights(alpha, n + 1)
    g1, g2 = math.gamma(alpha + 1), math.gamma(alpha + 2)
    for t in [1, 2, 5, 33, 1000, n]:  # target index t = n' + 1
        np_ = t - 1
        exact0 = t ** alpha / g1
        assert math.fsum(b[:t]) == pytest.approx(exact0, rel=1e-14)
        trap0 = math.fsum([c[np_]] + list(a[:np_]) + [1.0 / g2])
        assert trap0 == pytest.approx(exact0, rel=1e-14)
        # first moment: weights times source time j (j = 0..t), exact = t^(alpha+1)/Gamma(alpha+2)
        js = np.arange(1, np_ + 1, dtype=np.float64)
        trap1 = math.fsum(list(a[np_ - js.astype(np.int64)] * js) + [t / g2])
        assert trap1 == pytest.approx(t ** (alpha + 1) / g2, rel=1e-13)


def test_alpha_one_is_classical(orc):
    b, a, c = orc.weights(1.0, 4096)
    assert np.all(b == 1.0)
    assert np.all(a == 1.0)
    assert np.all(c == 0.5)


def test_weights_large_lag_against_mpmath_second_difference(orc):
    """At m near 2^20 the defining power differences cancel to ~40 bits; the
    oracle's binary128 evaluation must still be within a few ulp of a 60-digit
    evaluation (mpmath, an independent library)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    alpha = 0.95
    n = (1 << 20) + 3
    b, a, c = orc.weights(alpha, n)
    al = mpmath.mpf(alpha)
    g1, g2 = mpmath.gamma(al + 1), mpmath.gamma(al + 2)
    for m in [(1 << 20) - 1, (1 << 20) + 2, 999_999]:
        M = mpmath.mpf(m)
        eb = ((M + 1) ** al - M ** al) / g1
        ea = ((M + 2) ** (al + 1) - 2 * (M + 1) ** (al + 1) + M ** (al + 1)) / g2
        ec = (M ** (al + 1) - (M - al) * (M + 1) ** al) / g2
        for got, exp in ((b[m], eb), (a[m], ea), (c[m], ec)):
            assert abs(got - float(exp)) <= 4 * np.spacing(abs(float(exp)))
