"""Pins for the oracle's PECE solver (Section 2 of arXiv:1611.08678: eq. (1),
the predictor eq. (2) and the corrector).

Independent facts used:
  * constant forcing: both the product-rectangle predictor and the
    product-trapezoid corrector integrate a constant exactly, so
    y_n = y0 + c t_n^alpha / Gamma(alpha+1) to rounding;
  * affine forcing c0 + c1 t: the product trapezoid rule is exact for
    piecewise-linear integrands, so the corrector gives
    y0 + c0 t^alpha/Gamma(alpha+1) + c1 t^(alpha+1)/Gamma(alpha+2);
  * the linear test equation D^1/2 y = -y, y(0) = 1 has the closed form
    E_{1/2}(-sqrt t) = erfcx(sqrt t) (scipy's scaled complementary error function);
  * a manufactured smooth solution y = t^3 shows the method's convergence order
    min(2, 1 + alpha);
  * alpha = 1 reduces the scheme to classical Adams-Bashforth-1 /
    Adams-Moulton-2 PECE in integral form, an O(N) running-sum recurrence;
  * tiny N against an independent 50-digit mpmath implementation;
  * the time-block partition of the paper's parallel algorithm (Section 3):
    per-block partial history sums added at the owner equal the full sum.
"""
import math

import numpy as np
import pytest
from scipy.special import erfcx


def _lin_theta(A, b0, b1):
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    return np.concatenate([A.ravel(), np.asarray(b0, float).ravel(), np.asarray(b1, float).ravel()])


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.95, 1.0])
def test_constant_forcing_exact(orc, alpha):
    d, N, h = 2, 3000, 0.01
    cst = np.array([1.5, -0.25])
    th = _lin_theta(np.zeros((d, d)), cst, np.zeros(d))
    y0 = np.array([0.3, 2.0])
    y, yp, f, st = orc.solve(orc.LINEAR, th, alpha, h, N, y0)
    assert st == 0
    t = np.arange(N + 1) * h
    exact = y0[None, :] + cst[None, :] * (t ** alpha / math.gamma(alpha + 1))[:, None]
    scale = np.abs(exact).max()
    assert np.abs(y - exact).max() <= 1e-13 * scale
    assert np.abs(yp - exact).max() <= 1e-13 * scale


@pytest.mark.parametrize("alpha", [0.4, 0.8, 1.0])
def test_affine_forcing_corrector_exact(orc, alpha):
    d, N, h = 1, 2500, 0.004
    c0, c1 = 0.7, -1.3
    th = _lin_theta([[0.0]], [c0], [c1])
    y, yp, f, st = orc.solve(orc.LINEAR, th, alpha, h, N, [0.5])
    t = np.arange(N + 1) * h
    exact = 0.5 + c0 * t ** alpha / math.gamma(alpha + 1) + c1 * t ** (alpha + 1) / math.gamma(alpha + 2)
    assert np.abs(y[:, 0] - exact).max() <= 1e-13 * np.abs(exact).max()
    # the predictor (product rectangle) is not exact for the linear part
    if alpha < 1.0:
        assert np.abs(yp[1:, 0] - exact[1:]).max() > 1e-8


def test_mittag_leffler_linear_test_equation(orc):
    """D^{1/2} y = -y, y(0) = 1 on [0, 10], h = 0.005 (N = 2000): exact
    solution erfcx(sqrt t). The largest error sits at t = h, where the
    solution behaves like t^{1/2}; at t = 10 the error falls like h^{1+alpha}."""
    emax, eend = [], []
    for N in (500, 1000, 2000, 4000):
        h = 10.0 / N
        y, _, _, st = orc.solve(orc.LINEAR, _lin_theta([[-1.0]], [0.0], [0.0]), 0.5, h, N, [1.0])
        assert st == 0
        t = np.arange(N + 1) * h
        e = np.abs(y[:, 0] - erfcx(np.sqrt(t)))
        emax.append(e.max())
        eend.append(e[-1])
    # the configuration's step: recorded values 5.0e-4 (max, at t = h), 1.27e-6 (t = 10)
    assert emax[2] < 6e-4 and eend[2] < 1.4e-6
    assert all(emax[i + 1] < emax[i] for i in range(3))
    orders = [math.log2(eend[i] / eend[i + 1]) for i in range(3)]
    assert all(abs(o - 1.5) < 0.15 for o in orders), orders


@pytest.mark.parametrize("alpha", [0.5, 0.8])
def test_convergence_order_manufactured_cubic(orc, alpha):
    """y = t^3 solves D^alpha y = 6 t^(3-alpha)/Gamma(4-alpha) + lam (y - t^3)."""
    lam, T = -1.0, 1.0
    g = math.gamma(4 - alpha)

    def rhs(t, y):
        return [6.0 * t ** (3 - alpha) / g + lam * (y[0] - t ** 3)]

    errs = []
    for N in (64, 128, 256, 512):
        y, _, _, _ = orc.solve_callback(rhs, alpha, T / N, N, [0.0])
        t = np.arange(N + 1) * (T / N)
        errs.append(np.abs(y[:, 0] - t ** 3).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    expect = min(2.0, 1.0 + alpha)
    assert abs(orders[-1] - expect) < 0.1, orders


def _adams_integral_form(rhs, h, N, y0):
    """Classical AB1 predictor / AM2 corrector in integral (Volterra) form."""
    d = len(y0)
    y = np.empty((N + 1, d))
    y[0] = y0
    f0 = np.asarray(rhs(0.0, y0))
    S = f0.copy()
    for n in range(N):
        t1 = (n + 1) * h
        yp = y0 + h * S
        fp = np.asarray(rhs(t1, yp))
        y[n + 1] = y0 + h * (S - 0.5 * f0 + 0.5 * fp)
        S = S + np.asarray(rhs(t1, y[n + 1]))
    return y


def test_alpha_one_reduces_to_classical_adams(orc):
    mu = 1.3
    th = np.array([mu])

    def vdp(t, y):
        return orc.rhs(orc.VDP, th, t, y)

    N, h = 1500, 0.01
    y0 = np.array([1.2, -0.4])
    y, _, _, st = orc.solve(orc.VDP, th, 1.0, h, N, y0)
    ref = _adams_integral_form(vdp, h, N, y0)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_alpha_one_second_order(orc):
    errs = []
    for N in (100, 200, 400, 800):
        h = 2.0 / N
        y, _, _, _ = orc.solve(orc.LINEAR, _lin_theta([[-1.0]], [0.0], [0.0]), 1.0, h, N, [1.0])
        t = np.arange(N + 1) * h
        errs.append(np.abs(y[:, 0] - np.exp(-t)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert abs(orders[-1] - 2.0) < 0.1, orders


def _mp_pece(system_rhs, alpha, h, N, y0, dps=50, y1=None):
    """Brute-force PECE straight from the paper's weight formulas in mpmath;
    with y1 (= y'(0), for 1 < alpha <= 2) the initial part of every step is
    y0 + t y1."""
    import mpmath
    mpmath.mp.dps = dps
    al = mpmath.mpf(alpha)
    hh = mpmath.mpf(h)
    g1, g2 = mpmath.gamma(al + 1), mpmath.gamma(al + 2)
    bw = lambda m: ((m + 1) ** al - mpmath.mpf(m) ** al) / g1
    aw = lambda m: ((m + 2) ** (al + 1) - 2 * (m + 1) ** (al + 1) + mpmath.mpf(m) ** (al + 1)) / g2
    cw = lambda n: (mpmath.mpf(n) ** (al + 1) - (n - al) * (n + 1) ** al) / g2
    Y0 = [mpmath.mpf(v) for v in y0]
    Y1 = [mpmath.mpf(v) for v in (y1 if y1 is not None else [0.0] * len(y0))]
    ys, fs = [Y0], [system_rhs(mpmath.mpf(0), Y0)]
    ha = hh ** al
    for n in range(N):
        t1 = (n + 1) * hh
        P = [sum(bw(n - k) * fs[k][i] for k in range(n + 1)) for i in range(len(y0))]
        Cc = [cw(n) * fs[0][i] + sum(aw(n - k) * fs[k][i] for k in range(1, n + 1))
              for i in range(len(y0))]
        base = [Y0[i] + t1 * Y1[i] for i in range(len(y0))]
        yp = [base[i] + ha * P[i] for i in range(len(y0))]
        fp = system_rhs(t1, yp)
        yn = [base[i] + ha * (Cc[i] + fp[i] / g2) for i in range(len(y0))]
        ys.append(yn)
        fs.append(system_rhs(t1, yn))
    return np.array([[float(v) for v in row] for row in ys])


def test_tiny_n_against_mpmath_brute_force(orc):
    a_, b_, c_ = 35.0, 3.0, 28.0

    def chen(t, y):
        x, yy, z = y
        return [a_ * (yy - x), (c_ - a_) * x - x * z + c_ * yy, x * yy - b_ * z]

    alpha, h, N = 0.95, 0.001, 14
    y0 = [-9.0, -5.0, 14.0]
    ref = _mp_pece(chen, alpha, h, N, y0)
    y, _, _, _ = orc.solve(orc.CHEN, [a_, b_, c_], alpha, h, N, y0)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()


def test_system_equilibria(orc):
    """Each right-hand side vanishes at its textbook equilibrium."""
    a, b, c = 35.0, 3.0, 28.0
    s = math.sqrt(b * (2 * c - a))
    for y in ([s, s, 2 * c - a], [-s, -s, 2 * c - a], [0.0, 0.0, 0.0]):
        assert np.abs(orc.rhs(orc.CHEN, [a, b, c], 0.0, y)).max() < 1e-12
    a, b, c = 0.2, 0.2, 5.7
    disc = math.sqrt(c * c - 4 * a * b)
    for x in ((c - disc) / 2, (c + disc) / 2):
        y = [x, -x / a, x / a]
        assert np.abs(orc.rhs(orc.ROSSLER, [a, b, c], 0.0, y)).max() < 1e-12
    assert np.abs(orc.rhs(orc.VDP, [1.7], 0.0, [0.0, 0.0])).max() == 0.0
    # financial system (a, b, c): equilibrium (0, 1/b, 0)
    assert np.abs(orc.rhs(orc.FINANCIAL, [3.0, 0.1, 1.0], 0.0, [0.0, 10.0, 0.0])).max() < 1e-12
    # Hindmarsh-Rose: with y* = c - d x*^2 and z* = s (x* - xr), x* is a real root
    # of -a x^3 + (b - d) x^2 - s x + (c + s xr + I) (numpy's polynomial roots)
    th = [1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6, 3.25]
    a, b, c, d, r, sg, xr, I = th
    roots = np.roots([-a, b - d, -sg, c + sg * xr + I])
    xs = [z.real for z in roots if abs(z.imag) < 1e-12]
    assert xs
    for x in xs:
        y = [x, c - d * x * x, sg * (x - xr)]
        assert np.abs(orc.rhs(orc.HINDMARSH_ROSE, th, 0.0, y)).max() < 1e-12
    # linear: A y* + b0 = 0
    A = np.array([[-2.0, 0.3], [0.1, -1.0]])
    b0 = np.array([0.4, -0.2])
    ys = np.linalg.solve(A, -b0)
    assert np.abs(orc.rhs(orc.LINEAR, _lin_theta(A, b0, [0, 0]), 0.0, ys)).max() < 1e-14


def test_time_block_partition_identity(orc):
    """Section 3: with P virtual processes owning contiguous blocks of N/P
    history rows, the owner of target t adds the partial sums of every lower
    block to its own local sum; the result equals the full history sum."""
    alpha, N, Pn = 0.7, 4096, 8
    rng = np.random.default_rng(5)
    f = rng.standard_normal((N, 3))
    P, Cc, _, _ = orc.history_sums(alpha, f)
    b, a, c = orc.weights(alpha, N)
    nbar = N // Pn
    for t in (1, 7, nbar, nbar + 1, 3 * nbar + 5, N):
        owner = (t - 1) // nbar  # block holding the newest source row t-1
        S = np.zeros(3)
        for p in range(owner + 1):
            lo, hi = p * nbar, min((p + 1) * nbar, t)
            k = np.arange(lo, hi)
            S += (b[t - 1 - k][:, None] * f[k]).sum(axis=0)
        assert np.allclose(S, P[t - 1], rtol=1e-13, atol=1e-13 * np.abs(P[t - 1]).max())


def test_blow_up_is_flagged_and_frozen(orc):
    th = _lin_theta([[60.0]], [0.0], [0.0])
    y, _, _, st = orc.solve(orc.LINEAR, th, 0.9, 0.5, 400, [1.0])
    assert st > 0
    assert np.all(np.isfinite(y[:st]))
    assert np.all(np.isnan(y[st:]))


def test_batch_equals_single_and_thread_invariant(orc, monkeypatch):
    rng = np.random.default_rng(11)
    B = 6
    alphas = rng.uniform(0.9, 1.0, B)
    Ns = rng.integers(50, 300, B)
    y0 = rng.uniform(-5, 5, (B, 3))
    th = np.tile([0.2, 0.2, 5.7], (B, 1))
    y, off, st = orc.solve_batch(orc.ROSSLER, th, alphas, np.full(B, 0.005), Ns, y0)
    for i in range(B):
        yi, _, _, _ = orc.solve(orc.ROSSLER, th[i], alphas[i], 0.005, int(Ns[i]), y0[i])
        assert np.array_equal(y[off[i]: off[i] + Ns[i] + 1], yi)


def test_step_from_history_matches_solver_rows(orc):
    """The teacher-forced single step is the solver's step: fed the solver's own
    history it reproduces every sampled row exactly, and its magnitude sum is
    at least the size of the history part of the update."""
    th = [35.0, 3.0, 28.0]
    alpha, h, N = 0.95, 0.001, 3000
    y0 = [-9.0, -5.0, 14.0]
    y, _, f, st = orc.solve(1, th, alpha, h, N, y0)
    assert st == 0
    assert np.array_equal(orc.rhs_rows(1, th, h, y), f)
    wts = orc.weights(alpha, N)
    for t in (1, 2, 255, 256, 257, 1777, N):
        yt, mag = orc.step_from_history(1, th, alpha, h, t, y0, f, wts)
        assert np.array_equal(yt, y[t])
        assert np.all(mag > 0) and np.all(np.abs(y[t] - np.asarray(y0)) <= mag + 1.0)
