"""Pins for the oracle's right-hand sides and for its teacher-forced history
sums (Section 2 of arXiv:1611.08678: the predictor eq. (2) and the corrector).

The paper names the systems (Section 1; Hindmarsh-Rose in Section 4) but
prints no equations for them; the oracle uses the textbook forms. Independent
facts used here:
  * every system through an independent 50-digit mpmath PECE with the paper's
    naive weight formulas and the system written out in this file, started
    away from any equilibrium (a sign flip or a swapped term in any branch of
    the oracle's right-hand side changes the first step);
  * Chen's mirror symmetry (x, y, z) -> (-x, -y, z), a property of the system
    and not a restatement of it;
  * order one: the scheme is classical Adams AB1/AM2 PECE, so the oracle's
    Rossler trajectory converges at order two to a fine classical RK4
    solution of the same ODE;
  * history sums: closed forms of the product-integration rules for a
    constant and a ramp history (both fix the corrector's c_{t-1} f_0 term and
    its lag index), and the plain definition on a random history, evaluated
    here with numpy and weights from exact mpmath formulas.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_solver import _mp_pece


def _rossler(a, b, c):
    def f(t, y):
        x, yy, z = y
        return [-(yy + z), x + a * yy, b + z * (x - c)]
    return f


def _financial(a, b, c):
    def f(t, y):
        x, yy, z = y
        return [z + (yy - a) * x, 1 - b * yy - x * x, -x - c * z]
    return f


def _hindmarsh_rose(a, b, c, d, r, s, xr, I):
    def f(t, y):
        x, yy, z = y
        return [yy - a * x ** 3 + b * x ** 2 - z + I, c - d * x ** 2 - yy, r * (s * (x - xr) - z)]
    return f


def _vdp(mu):
    def f(t, y):
        x, v = y
        return [v, mu * (1 - x * x) * v - x]
    return f


def _linear(A, b0, b1):
    def f(t, y):
        return [sum(A[i][j] * y[j] for j in range(len(y))) + b0[i] + b1[i] * t
                for i in range(len(y))]
    return f


CASES = {
    # name: (oracle id, theta, mpmath rhs, y0, alpha, h)
    "rossler": (2, [0.2, 0.2, 5.7], _rossler(0.2, 0.2, 5.7), [1.3, -2.1, 0.7], 0.93, 0.05),
    "financial": (4, [3.0, 0.1, 1.0], _financial(3.0, 0.1, 1.0), [0.5, 1.7, -0.3], 0.85, 0.05),
    "hindmarsh_rose": (5, [1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6, 3.25],
                       _hindmarsh_rose(1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6, 3.25),
                       [-1.2, -7.0, 2.5], 0.95, 0.02),
    "vdp": (3, [1.3], _vdp(1.3), [1.1, -0.7], 0.9, 0.05),
    "linear": (0, [-2.0, 0.3, 0.15, -1.1, 0.2, -0.1, 0.05, 0.3],
               _linear([[-2.0, 0.3], [0.15, -1.1]], [0.2, -0.1], [0.05, 0.3]),
               [0.4, -1.2], 0.8, 0.05),
}


@pytest.mark.parametrize("name", list(CASES))
def test_system_against_mpmath_brute_force(orc, name):
    sid, th, fn, y0, alpha, h = CASES[name]
    N = 12
    ref = _mp_pece(fn, alpha, h, N, y0)
    y, _, _, st = orc.solve(sid, th, alpha, h, N, y0)
    assert st == 0
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()
    # every component moves (a wrong term in any of them shows at 1e-14)
    assert np.all(np.abs(ref[-1] - ref[0]) > 1e-8 * np.abs(ref).max())


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_values_against_written_out_systems(orc, name):
    """f itself at a handful of random points (every term of every component)."""
    import mpmath
    sid, th, fn, y0, alpha, h = CASES[name]
    rng = np.random.default_rng(17)
    for _ in range(5):
        y = rng.uniform(-3, 3, len(y0))
        t = float(rng.uniform(0, 5))
        mpmath.mp.dps = 40
        ref = np.array([float(v) for v in fn(mpmath.mpf(t), [mpmath.mpf(v) for v in y])])
        got = orc.rhs(sid, th, t, y)
        assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


def test_chen_mirror_symmetry(orc):
    th = [35.0, 3.0, 28.0]
    y0 = np.array([-9.0, -5.0, 14.0])
    a, _, _, sa = orc.solve(orc.CHEN, th, 0.95, 0.001, 3000, y0)
    b, _, _, sb = orc.solve(orc.CHEN, th, 0.95, 0.001, 3000, y0 * [-1, -1, 1])
    assert sa == sb == 0
    assert np.array_equal(a * [-1, -1, 1], b)


def test_rossler_order_one_converges_to_rk4(orc):
    """At alpha = 1 the scheme integrates the classical Rossler ODE with
    second-order accuracy; the reference is a classical RK4 at a step 64 times
    smaller than the finest one checked."""
    a, b, c = 0.2, 0.2, 5.7
    fn = _rossler(a, b, c)
    T = 4.0
    y0 = np.array([1.3, -2.1, 0.7])

    def rk4(n):
        hh = T / n
        y = y0.copy()
        out = [y.copy()]
        for k in range(n):
            t = k * hh
            k1 = np.array(fn(t, y))
            k2 = np.array(fn(t + hh / 2, y + hh / 2 * k1))
            k3 = np.array(fn(t + hh / 2, y + hh / 2 * k2))
            k4 = np.array(fn(t + hh, y + hh * k3))
            y = y + hh / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            out.append(y.copy())
        return np.array(out)

    fine = rk4(400 * 64)
    errs = []
    for n in (100, 200, 400):
        y, _, _, st = orc.solve(orc.ROSSLER, [a, b, c], 1.0, T / n, n, y0)
        assert st == 0
        errs.append(np.abs(y[-1] - fine[-1]).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(o - 2.0) < 0.15 for o in orders), (errs, orders)


def _mp_weights(alpha, n):
    """b_m, a_m, c_m (Section 2) from the defining power differences at 50 digits."""
    import mpmath
    mpmath.mp.dps = 50
    al = mpmath.mpf(alpha)
    g1, g2 = mpmath.gamma(al + 1), mpmath.gamma(al + 2)
    b = np.array([float(((m + 1) ** al - mpmath.mpf(m) ** al) / g1) for m in range(n)])
    a = np.array([float(((m + 2) ** (al + 1) - 2 * (m + 1) ** (al + 1) + mpmath.mpf(m) ** (al + 1))
                        / g2) for m in range(n)])
    c = np.array([float((mpmath.mpf(m) ** (al + 1) - (m - al) * (m + 1) ** al) / g2)
                  for m in range(n)])
    return b, a, c


@pytest.mark.parametrize("alpha", [0.35, 0.8, 1.0, 1.6])
def test_history_sums_closed_forms(orc, alpha):
    """Constant history f_k = 1: the product rectangle and product trapezoid
    rules integrate constants exactly, so P_t = t^a / Gamma(a+1) and
    C_t + 1/Gamma(a+2) = t^a / Gamma(a+1) (the corrector's own newest term
    weighs 1/Gamma(a+2)). Ramp f_k = k: the trapezoid rule is exact for linear
    integrands, so C_t + t/Gamma(a+2) = t^(a+1)/Gamma(a+2). Component 2 is
    u + v k, which checks linearity across the two."""
    N = 3000
    k = np.arange(N, dtype=np.float64)
    f = np.stack([np.ones(N), k, 0.75 - 0.002 * k], axis=1)
    P, C, Pa, Ca = orc.history_sums(alpha, f)
    t = np.arange(1, N + 1, dtype=np.float64)
    g1, g2 = math.gamma(alpha + 1), math.gamma(alpha + 2)
    P1 = t ** alpha / g1
    C1 = t ** alpha / g1 - 1.0 / g2
    Cr = (t ** (alpha + 1) - t) / g2
    assert np.abs(P[:, 0] - P1).max() <= 1e-13 * P1.max()
    assert np.abs(C[:, 0] - C1).max() <= 1e-13 * np.abs(C1).max()
    assert np.abs(C[:, 1] - Cr).max() <= 1e-13 * np.abs(Cr).max()
    assert np.abs(C[:, 2] - (0.75 * C1 - 0.002 * Cr)).max() <= 1e-13 * np.abs(Ca[:, 2]).max()
    # the magnitude sums are the sums of |w f|: equal to the sums for f >= 0
    assert np.abs(Pa[:, 0] - P[:, 0]).max() <= 1e-13 * P1.max()


@pytest.mark.parametrize("alpha", [0.45, 0.95])
def test_history_sums_random_history_definition(orc, alpha):
    """P_t = sum_{k<t} b_{t-1-k} f_k and C_t = c_{t-1} f_0 + sum_{1<=k<t} a_{t-1-k} f_k
    on a random history, with weights from exact formulas and numpy sums."""
    N, d = 400, 3
    rng = np.random.default_rng(23)
    f = rng.standard_normal((N, d))
    f[0] *= 7.0  # make the f_0 term stand out
    b, a, c = _mp_weights(alpha, N)
    P, C, Pa, Ca = orc.history_sums(alpha, f)
    for t in range(1, N + 1):
        k = np.arange(t)
        p = (b[t - 1 - k][:, None] * f[k]).sum(0)
        q = c[t - 1] * f[0] + (a[t - 1 - k[1:]][:, None] * f[k[1:]]).sum(0)
        pa = (np.abs(b[t - 1 - k])[:, None] * np.abs(f[k])).sum(0)
        assert np.all(np.abs(P[t - 1] - p) <= 1e-14 * pa + 1e-300), t
        assert np.all(np.abs(C[t - 1] - q) <= 1e-14 * Ca[t - 1] + 1e-300), t
        assert np.allclose(Pa[t - 1], pa, rtol=1e-13)


def test_history_sums_rows_are_the_full_sums(orc):
    """The row-subset form returns exactly the rows of the full form."""
    rng = np.random.default_rng(29)
    f = rng.standard_normal((2500, 2)) * [3.0, 0.5]
    full = orc.history_sums(0.7, f)
    rows = np.array([1, 2, 255, 256, 257, 1024, 2499, 2500])
    part = orc.history_sums_rows(0.7, f, rows)
    for a, b in zip(full, part):
        assert np.array_equal(a[rows - 1], b)
