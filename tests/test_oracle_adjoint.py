"""Pins for the oracle's discrete adjoint (reverse mode of the PECE scheme of
Section 2 of arXiv:1611.08678) for L = sum_n <g_n, y_n>:
  * central finite differences of the oracle's own forward solve, at two
    step sizes so that the truncation error is seen to shrink;
  * torch.autograd (float64, CPU) through an independent tensor implementation
    of the forward recursion at small N.
"""
import math

import numpy as np
import pytest

SYSTEMS = {
    # name: (id, theta, y0, alpha, h, N)
    "vdp": (3, [1.3], [1.1, -0.7], 0.9, 0.01, 300),
    "chen": (1, [35.0, 3.0, 28.0], [-9.0, -5.0, 14.0], 0.95, 0.001, 200),
    "rossler": (2, [0.2, 0.2, 5.7], [1.0, -2.0, 0.5], 0.93, 0.005, 250),
    "financial": (4, [3.0, 0.1, 1.0], [0.5, 1.0, -0.3], 0.85, 0.01, 200),
    "hindmarsh_rose": (5, [1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6, 3.25], [-1.2, -7.0, 2.5], 0.95,
                       0.01, 200),
    "linear": (0, None, [0.4, -1.2], 0.8, 0.01, 250),
    # 1 < alpha <= 2: y(0) and y'(0); the gradient has a row for each
    "vdp_slope": (3, [1.3], [[1.1, -0.7], [0.4, 0.9]], 1.5, 0.01, 300),
    "linear_alpha2": (0, None, [[0.4, -1.2], [-0.3, 0.5]], 2.0, 0.01, 250),
}


def _theta(name):
    sid, th, y0, alpha, h, N = SYSTEMS[name]
    if th is None:
        A = np.array([[-2.0, 0.3], [0.15, -1.1]])
        th = np.concatenate([A.ravel(), [0.2, -0.1], [0.05, 0.3]])
    return sid, np.asarray(th, float), np.asarray(y0, float), alpha, h, N


def _loss(orc, sid, th, alpha, h, N, y0, g):
    y, _, _, st = orc.solve(sid, th, alpha, h, N, y0)
    assert st == 0
    return float(np.sum(g * y))


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_adjoint_vs_central_differences(orc, name):
    sid, th, y0, alpha, h, N = _theta(name)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((N + 1, y0.shape[-1]))
    gy0, gth, st = orc.adjoint(sid, th, alpha, h, N, y0, g)
    assert st == 0
    shape = y0.shape
    y0, gy0 = y0.ravel(), gy0.ravel()
    params = [("y0", y0, gy0), ("theta", th, gth)]
    for label, base, grad in params:
        for i in range(base.size):
            errs = []
            for rel in (1e-4, 1e-5):
                dlt = rel * max(1.0, abs(base[i]))
                p, m = base.copy(), base.copy()
                p[i] += dlt
                m[i] -= dlt
                if label == "y0":
                    p, m = p.reshape(shape), m.reshape(shape)
                    fd = (_loss(orc, sid, th, alpha, h, N, p, g) - _loss(orc, sid, th, alpha, h, N, m, g)) / (2 * dlt)
                else:
                    y0s = y0.reshape(shape)
                    fd = (_loss(orc, sid, p, alpha, h, N, y0s, g) - _loss(orc, sid, m, alpha, h, N, y0s, g)) / (2 * dlt)
                errs.append(abs(fd - grad[i]))
            scale = max(abs(grad[i]), 1e-3 * np.abs(grad).max(), 1e-12)
            assert min(errs) <= 2e-6 * scale, (label, i, grad[i], errs)


def _torch_forward(torch, sid, th, y0, alpha, h, N):
    """Independent tensor implementation of the PECE recursion (naive weights)."""
    dt = torch.float64
    al = torch.tensor(alpha, dtype=dt)
    m = torch.arange(N + 2, dtype=dt)
    g1 = math.gamma(alpha + 1)
    g2 = math.gamma(alpha + 2)
    bw = ((m + 1) ** al - m ** al) / g1
    aw = ((m + 2) ** (al + 1) - 2 * (m + 1) ** (al + 1) + m ** (al + 1)) / g2
    cw = (m ** (al + 1) - (m - al) * (m + 1) ** al) / g2
    ha = h ** alpha

    def f(t, y):
        if sid == 3:
            mu = th[0]
            return torch.stack([y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]])
        if sid == 1:
            a, b, c = th[0], th[1], th[2]
            return torch.stack([a * (y[1] - y[0]), (c - a) * y[0] - y[0] * y[2] + c * y[1],
                                y[0] * y[1] - b * y[2]])
        if sid == 2:
            a, b, c = th[0], th[1], th[2]
            return torch.stack([-y[1] - y[2], y[0] + a * y[1], b + y[2] * (y[0] - c)])
        if sid == 4:
            a, b, c = th[0], th[1], th[2]
            return torch.stack([y[2] + (y[1] - a) * y[0], 1 - b * y[1] - y[0] ** 2, -y[0] - c * y[2]])
        if sid == 5:
            a, b, c, dd, r, s, xr, I = (th[j] for j in range(8))
            return torch.stack([y[1] - a * y[0] ** 3 + b * y[0] ** 2 - y[2] + I,
                                c - dd * y[0] ** 2 - y[1], r * (s * (y[0] - xr) - y[2])])
        d = y.shape[0]
        A = th[: d * d].reshape(d, d)
        return A @ y + th[d * d: d * d + d] + th[d * d + d:] * t

    ys = [y0]
    fs = [f(0.0, y0)]
    for n in range(N):
        F = torch.stack(fs)  # [n+1, d]
        k = torch.arange(n + 1)
        P = (bw[n - k][:, None] * F).sum(0)
        Cc = cw[n] * F[0] + (aw[n - k[1:]][:, None] * F[1:]).sum(0)
        t1 = (n + 1) * h
        yp = y0 + ha * P
        fp = f(t1, yp)
        yn = y0 + ha * (Cc + fp / g2)
        ys.append(yn)
        fs.append(f(t1, yn))
    return torch.stack(ys)


@pytest.mark.parametrize("name", ["vdp", "chen", "rossler", "financial", "hindmarsh_rose", "linear"])
def test_adjoint_vs_torch_autograd(orc, name):
    torch = pytest.importorskip("torch")
    sid, th, y0, alpha, h, N = _theta(name)
    N = min(N, 120)
    rng = np.random.default_rng(9)
    g = rng.standard_normal((N + 1, y0.shape[-1]))
    tth = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    ty0 = torch.tensor(y0, dtype=torch.float64, requires_grad=True)
    Y = _torch_forward(torch, sid, tth, ty0, alpha, h, N)
    yo, _, _, _ = orc.solve(sid, th, alpha, h, N, y0)
    assert np.abs(Y.detach().numpy() - yo).max() <= 1e-12 * np.abs(yo).max()
    L = (Y * torch.tensor(g)).sum()
    L.backward()
    gy0, gth, _ = orc.adjoint(sid, th, alpha, h, N, y0, g)
    ref0, refth = ty0.grad.numpy(), tth.grad.numpy()
    sc = max(np.abs(ref0).max(), np.abs(refth).max())
    assert np.abs(gy0 - ref0).max() <= 1e-12 * sc
    assert np.abs(gth - refth).max() <= 1e-12 * sc
