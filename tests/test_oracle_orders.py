"""Pins for the oracle's non-commensurate solver (eq. (1) of arXiv:1611.08678
with a separate order alpha_i per component; each component runs the
Section 2 scheme with its own weights, h^alpha_i and Gamma(alpha_i + 2)).

Independent facts used:
  * equal orders reduce to the commensurate solver (pinned on its own);
  * a diagonal linear system decouples: component i is the Mittag-Leffler
    solution y_i(0) E_{a_i}(lam_i t^a_i) + y_i'(0) t E_{a_i,2}(lam_i t^a_i),
    and permuting the components permutes the result exactly;
  * a coupled manufactured solution (t^3, 1 + t^2) converges at the order of
    its slowest component;
  * tiny N against a 50-digit mpmath implementation with per-component
    weights;
  * batch = single;
  * the per-component adjoint: equal orders give the commensurate adjoint
    bitwise, and every gradient entry matches central differences of the
    per-component forward solve.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_slope import _ml


def _lin(A, b0, b1):
    return np.concatenate([np.ravel(A), np.ravel(b0), np.ravel(b1)]).astype(float)


@pytest.mark.parametrize("alpha,init", [(0.85, [[1.0, -0.4, 2.0]]),
                                        (1.4, [[1.0, -0.4, 2.0], [0.3, 0.0, -1.0]])])
def test_equal_orders_are_the_commensurate_solver(orc, alpha, init):
    th = [0.2, 0.2, 5.7]
    a, _, _, sa = orc.solve(orc.ROSSLER, th, alpha, 0.005, 1500, np.squeeze(init))
    b, _, _, sb = orc.solve_orders(orc.ROSSLER, th, [alpha] * 3, 0.005, 1500, np.squeeze(init))
    assert sa == sb and np.array_equal(a, b)


def test_decoupled_components_follow_their_own_order(orc):
    alphas = np.array([0.5, 0.9, 1.5, 1.9])
    lam = np.array([-1.0, -0.7, -1.2, -0.5])
    init = np.array([[1.0, 0.5, 1.0, 0.0], [0.0, 0.0, 0.5, 1.0]])
    th = _lin(np.diag(lam), np.zeros(4), np.zeros(4))
    errs = []
    for N in (250, 500, 1000):
        h = 5.0 / N
        y, _, _, st = orc.solve_orders(orc.LINEAR, th, alphas, h, N, init)
        assert st == 0
        idx = np.arange(0, N + 1, N // 25)
        t = idx * h
        e = []
        for i in range(4):
            ex = np.array([init[0, i] * _ml(alphas[i], 1, lam[i] * s ** alphas[i]) +
                           (init[1, i] * s * _ml(alphas[i], 2, lam[i] * s ** alphas[i])
                            if alphas[i] > 1 else 0.0) for s in t])
            e.append(np.abs(y[idx, i] - ex)[-1])
        errs.append(e)
    errs = np.array(errs)
    # end-point error falls like h^(min(2, 1 + alpha_i)) in each component
    for i in range(4):
        o = math.log2(errs[1, i] / errs[2, i])
        assert abs(o - min(2.0, 1.0 + alphas[i])) < 0.2, (i, o, errs[:, i])
    # a permutation of the components permutes the result bitwise
    perm = np.array([2, 0, 3, 1])
    thp = _lin(np.diag(lam[perm]), np.zeros(4), np.zeros(4))
    y, _, _, _ = orc.solve_orders(orc.LINEAR, th, alphas, 0.01, 500, init)
    yp, _, _, _ = orc.solve_orders(orc.LINEAR, thp, alphas[perm], 0.01, 500, init[:, perm])
    assert np.array_equal(yp, y[:, perm])


def test_coupled_manufactured_solution(orc):
    """(t^3, 1 + t^2) solves D^{a1} y1 = 6 t^(3-a1)/Gamma(4-a1) + (y2 - 1 - t^2),
    D^{a2} y2 = 2 t^(2-a2)/Gamma(3-a2) - (y1 - t^3) with y(0) = (0, 1),
    y'(0) = (0, 0); orders (0.6, 1.5)."""
    a1, a2 = 0.6, 1.5
    g1, g2 = math.gamma(4 - a1), math.gamma(3 - a2)

    def rhs(t, y):
        return [6.0 * t ** (3 - a1) / g1 + (y[1] - 1 - t * t),
                2.0 * t ** (2 - a2) / g2 - (y[0] - t ** 3)]

    errs = []
    for N in (64, 128, 256, 512):
        y, _, _, st = orc.solve_orders_callback(rhs, [a1, a2], 1.0 / N, N, [[0.0, 1.0], [0.0, 0.0]])
        assert st == 0
        t = np.arange(N + 1) / N
        errs.append(np.abs(y - np.stack([t ** 3, 1 + t * t], axis=1)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert abs(orders[-1] - min(2.0, 1.0 + a1)) < 0.15, orders


def _mp_orders(rhs, alphas, h, N, init, dps=50):
    """Per-component PECE in mpmath straight from the Section 2 weight formulas."""
    import mpmath
    mpmath.mp.dps = dps
    d = len(alphas)
    hh = mpmath.mpf(h)
    al = [mpmath.mpf(a) for a in alphas]
    g1 = [mpmath.gamma(a + 1) for a in al]
    g2 = [mpmath.gamma(a + 2) for a in al]
    bw = lambda i, m: ((m + 1) ** al[i] - mpmath.mpf(m) ** al[i]) / g1[i]
    aw = lambda i, m: ((m + 2) ** (al[i] + 1) - 2 * (m + 1) ** (al[i] + 1) +
                       mpmath.mpf(m) ** (al[i] + 1)) / g2[i]
    cw = lambda i, n: (mpmath.mpf(n) ** (al[i] + 1) - (n - al[i]) * (n + 1) ** al[i]) / g2[i]
    Y0 = [mpmath.mpf(v) for v in init[0]]
    Y1 = [mpmath.mpf(v) for v in init[1]]
    ys, fs = [Y0], [rhs(mpmath.mpf(0), Y0)]
    for n in range(N):
        t1 = (n + 1) * hh
        base = [Y0[i] + (t1 * Y1[i] if alphas[i] > 1 else 0) for i in range(d)]
        P = [sum(bw(i, n - k) * fs[k][i] for k in range(n + 1)) for i in range(d)]
        Cc = [cw(i, n) * fs[0][i] + sum(aw(i, n - k) * fs[k][i] for k in range(1, n + 1))
              for i in range(d)]
        yp = [base[i] + hh ** al[i] * P[i] for i in range(d)]
        fp = rhs(t1, yp)
        yn = [base[i] + hh ** al[i] * (Cc[i] + fp[i] / g2[i]) for i in range(d)]
        ys.append(yn)
        fs.append(rhs(t1, yn))
    return np.array([[float(v) for v in row] for row in ys])


def test_tiny_n_against_mpmath(orc):
    a_, b_, c_ = 3.0, 0.1, 1.0

    def fin(t, y):
        return [y[2] + (y[1] - a_) * y[0], 1 - b_ * y[1] - y[0] ** 2, -y[0] - c_ * y[2]]

    alphas, h, N = [0.7, 1.3, 0.95], 0.05, 12
    init = [[0.5, 1.0, -0.3], [0.0, 0.8, 0.0]]
    ref = _mp_orders(fin, alphas, h, N, init)
    y, _, _, _ = orc.solve_orders(orc.FINANCIAL, [a_, b_, c_], alphas, h, N, init)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()


def test_orders_batch_equals_single(orc):
    rng = np.random.default_rng(2)
    B = 5
    al = rng.uniform(0.5, 1.8, (B, 2))
    Ns = rng.integers(30, 300, B)
    init = rng.uniform(-1, 1, (B, 2, 2))
    th = rng.uniform(0.5, 1.5, (B, 1))
    y, off, st = orc.solve_orders_batch(orc.VDP, th, al, np.full(B, 0.01), Ns, init)
    for i in range(B):
        yi, _, _, si = orc.solve_orders(orc.VDP, th[i], al[i], 0.01, int(Ns[i]), init[i])
        assert st[i] == si and np.array_equal(y[off[i]: off[i] + Ns[i] + 1], yi)


def test_orders_adjoint_equal_orders_is_commensurate_adjoint(orc):
    th = [1.3]
    for alpha, init in ((0.9, [1.1, -0.7]), (1.5, [[1.1, -0.7], [0.4, 0.9]])):
        g = np.random.default_rng(1).standard_normal((301, 2))
        a0, at, sa = orc.adjoint(orc.VDP, th, alpha, 0.01, 300, init, g)
        b0, bt, sb = orc.adjoint_orders(orc.VDP, th, [alpha, alpha], 0.01, 300, init, g)
        assert sa == sb == 0 and np.array_equal(a0, b0) and np.array_equal(at, bt)


@pytest.mark.parametrize("sid,theta,alphas,init", [
    (3, [1.3], [0.7, 0.95], [1.1, -0.7]),
    (3, [0.8], [1.6, 0.8], [[1.1, -0.7], [0.4, 0.9]]),
    (4, [3.0, 0.1, 1.0], [0.85, 1.3, 0.7], [[0.5, 1.0, -0.3], [0.2, -0.4, 0.6]]),
])
def test_orders_adjoint_vs_central_differences(orc, sid, theta, alphas, init):
    """Gradients with respect to every initial value and theta against central
    differences of the oracle's own per-component forward solve."""
    theta, init = np.asarray(theta, float), np.asarray(init, float)
    N, h = 250, 0.01
    g = np.random.default_rng(3).standard_normal((N + 1, init.shape[-1]))

    def loss(th, y0):
        y, _, _, st = orc.solve_orders(sid, th, alphas, h, N, y0)
        assert st == 0
        return float(np.sum(g * y))

    gy0, gth, st = orc.adjoint_orders(sid, theta, alphas, h, N, init, g)
    assert st == 0
    for label, base, grad in (("y0", init, gy0), ("theta", theta, gth)):
        flat, gflat = base.ravel(), np.ravel(grad)
        for i in range(flat.size):
            errs = []
            for rel in (1e-4, 1e-5):
                dl = rel * max(1.0, abs(flat[i]))
                p, m = flat.copy(), flat.copy()
                p[i] += dl
                m[i] -= dl
                if label == "y0":
                    fd = (loss(theta, p.reshape(base.shape)) - loss(theta, m.reshape(base.shape))) / (2 * dl)
                else:
                    fd = (loss(p, init) - loss(m, init)) / (2 * dl)
                errs.append(abs(fd - gflat[i]))
            scale = max(abs(gflat[i]), 1e-3 * np.abs(gflat).max(), 1e-12)
            assert min(errs) <= 2e-6 * scale, (label, i, gflat[i], errs)
    if init.ndim == 2:  # components at or below order one: zero y'(0) gradient
        for i, a in enumerate(alphas):
            if a <= 1.0:
                assert gy0[1][i] == 0.0
