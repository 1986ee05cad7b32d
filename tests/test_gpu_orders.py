"""GPU parity of non-commensurate orders (a separate alpha per component;
plans with FABM_PLAN_PER_COMPONENT_ORDER) against the oracle's per-component
solver, through the C ABI: ragged batches on the DIRECT workgroup-per-instance
kernel and the batched BLOCKED pipeline, single long trajectories on the
whole-GPU DIRECT kernel and the BLOCKED step kernels, orders above one with
y'(0), blow-up status, and equal orders giving the commensurate result
bitwise (DIRECT). 1e-11 normwise, as for every FP64 path."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.test_gpu_direct import _to_np, relerr

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def F():
    import paper_1611_08678_amd as F
    F.load()
    return F


def _lin(d, seed):
    rng = np.random.default_rng(seed)
    A = -(2 * np.eye(d) + rng.standard_normal((d, d)) / 8)
    return np.concatenate([A.ravel(), rng.standard_normal(d), 0.05 * rng.standard_normal(d)])


SYSTEMS = {  # name: (id, d, theta of instance i)
    "vdp": (3, 2, lambda rng, i: rng.uniform(0.5, 2, 1)),
    "financial": (4, 3, lambda rng, i: np.array([3.0, 0.1, 1.0])),
    "hindmarsh_rose": (5, 3, lambda rng, i: np.array([1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6,
                                                     3.25])),
    "linear3": (0, 3, lambda rng, i: _lin(3, 50 + i)),
    "linear1": (0, 1, lambda rng, i: _lin(1, 70 + i)),
}


def _horizons(orc, sid, th, al, hs, Ns, init, ref, off, rows):
    """Per instance, the rows a correct binary64 evaluation must reproduce:
    those before the solution leaves |y| < 1e10 (a blow-up then climbs toward
    overflow) and before a one-ulp change of y(0) has grown past 1e-13 of the
    solution's size in the oracle itself (the reading used for chaotic
    trajectories); bounded, non-chaotic instances keep every row."""
    i2 = np.array(init, dtype=np.float64, copy=True)
    first = i2[:, 0] if i2.ndim == 3 else i2
    first[:, 0] = np.nextafter(first[:, 0], np.inf)
    alt, _, _ = orc.solve_orders_batch(sid, th, al, hs, Ns, i2)
    out = []
    for i in range(len(Ns)):
        seg, sa = ref[off[i]: off[i] + rows[i]], alt[off[i]: off[i] + rows[i]]
        big = np.nonzero(np.abs(seg).max(axis=1) > 1e10)[0]
        g = int(big[0]) if big.size else rows[i]
        scale = np.abs(seg[:g]).max()
        bad = np.nonzero(np.abs(sa[:g] - seg[:g]).max(axis=1) > 1e-13 * scale)[0]
        out.append(int(bad[0]) if bad.size else g)
    return out


def _compare(F, orc, sysname, th, al, hs, Ns, init, tol=1e-11, path="direct", far_prec="fp64",
             errs=None):
    """Status equal (or one step apart at the top of the binary64 range, as
    for commensurate orders), NaN rows from there on, and the rows of
    _horizons within tol normwise."""
    sid = SYSTEMS[sysname][0] if sysname in SYSTEMS else {"chen": 1}[sysname]
    name = "linear" if sysname.startswith("linear") else sysname
    y, off, st = F.solve_batch(name, th, al, hs, Ns, init, path=path, far_prec=far_prec)
    ref, roff, rst = orc.solve_orders_batch(sid, th, al, hs, Ns, init)
    assert np.array_equal(off, roff)
    yy, gst = _to_np(y), _to_np(st)
    rows = []
    for i in range(len(Ns)):
        if gst[i] != rst[i]:
            k = int(min(gst[i], rst[i]))
            assert k > 0 and abs(int(gst[i]) - int(rst[i])) == 1, (i, gst[i], rst[i])
            assert np.abs(ref[off[i] + k - 1]).max() > np.finfo(np.float64).max / 1e3
        rows.append(int(min(x for x in (gst[i], rst[i], Ns[i] + 1) if x)))
        if gst[i]:
            assert np.all(np.isnan(yy[off[i] + int(gst[i]): off[i] + Ns[i] + 1]))
    hz = _horizons(orc, sid, th, al, hs, Ns, init, ref, off, rows)
    for i in range(len(Ns)):
        assert hz[i] >= min(rows[i], 100) or hz[i] >= rows[i] - 8, (i, hz[i], rows[i])
        sl = slice(off[i], off[i] + hz[i])
        err = relerr(yy[sl], ref[sl])
        assert err <= tol, (i, err, hz[i], rows[i])
        if errs is not None:
            errs.append(err)
    return rst


@pytest.mark.parametrize("path", ["direct", "blocked"])
@pytest.mark.parametrize("sysname", list(SYSTEMS))
@pytest.mark.parametrize("slope", [False, True])
def test_batch_per_component_orders(F, orc, sysname, slope, path):
    sid, d, th_of = SYSTEMS[sysname]
    rng = np.random.default_rng(60 + sid + 10 * slope)
    B = 10
    th = np.stack([th_of(rng, i) for i in range(B)])
    al = rng.uniform(0.6, 2.0 if slope else 1.0, (B, d))
    if slope:
        al[0] = 2.0
        al[1] = np.minimum(al[1], 1.0)  # all components at or below one: y'(0) unused
    hs = rng.uniform(0.005, 0.015, B)
    Ns = rng.integers(100, 2500, B, endpoint=True)
    Ns[:3] = [1, 255, 1024]
    init = 0.5 * rng.uniform(-1, 1, (B, 2, d) if slope else (B, d))
    _compare(F, orc, sysname, th, al, hs, Ns, init, path=path)


@pytest.mark.parametrize("sysname", ["vdp", "hindmarsh_rose", "linear3"])
def test_batch_per_component_orders_fp32_windows(F, orc, sysname):
    """Binary32 far windows with per-component orders (one binary32 A operand
    per component): within the FP32 bound of the commensurate paths, and
    visibly different from FP64."""
    sid, d, th_of = SYSTEMS[sysname]
    rng = np.random.default_rng(120 + sid)
    B = 10
    th = np.stack([th_of(rng, i) for i in range(B)])
    al = rng.uniform(0.6, 1.0, (B, d))
    hs = rng.uniform(0.005, 0.015, B)
    Ns = rng.integers(300, 2500, B, endpoint=True)
    Ns[:2] = [1, 1024]
    init = 0.5 * rng.uniform(-1, 1, (B, d))
    errs = []
    _compare(F, orc, sysname, th, al, hs, Ns, init, tol=1e-5, path="blocked", far_prec="fp32",
             errs=errs)
    from tests import reduced_bounds as RB
    RB.check(f"orders_fp32_{sysname}", max(errs), 1e-5)
    name = "linear" if sysname.startswith("linear") else sysname
    y32, _, _ = F.solve_batch(name, th, al, hs, Ns, init, path="blocked", far_prec="fp32")
    y64, _, _ = F.solve_batch(name, th, al, hs, Ns, init, path="blocked")
    assert relerr(_to_np(y32), _to_np(y64)) > 1e-12


@pytest.mark.parametrize("path", ["direct", "blocked"])
@pytest.mark.parametrize("sysname,al,N", [("vdp", [0.8, 0.95], 9000),
                                          ("hindmarsh_rose", [0.9, 1.0, 0.95], 10000),
                                          ("linear3", [0.6, 1.6, 1.95], 8500)])
def test_single_long_trajectory(F, orc, sysname, al, N, path):
    """N >= 8192: one trajectory on the whole-GPU DIRECT kernel or the BLOCKED
    step kernels (35-40 blocks of 256 rows, far windows in every launch)."""
    sid, d, th_of = SYSTEMS[sysname]
    rng = np.random.default_rng(4)
    th = th_of(rng, 0)[None]
    init = 0.5 * rng.uniform(-1, 1, (1, 2, d))
    _compare(F, orc, sysname, th, np.array([al]), [0.01], [N], init, path=path)
    # the single-trajectory convenience call takes the per-component orders too
    name = "linear" if sysname.startswith("linear") else sysname
    y, st = F.solve(name, th[0], al, 0.01, N, init[0], path=path)
    ref, _, _, rst = orc.solve_orders(sid, th[0], al, 0.01, N, init[0])
    assert int(st.item()) == rst == 0 and relerr(_to_np(y), ref) <= 1e-11


def test_equal_orders_match_commensurate_direct_bitwise(F):
    rng = np.random.default_rng(7)
    B, d = 8, 3
    th = np.tile([0.2, 0.2, 5.7], (B, 1))
    a = rng.uniform(0.7, 1.0, B)
    hs, Ns = np.full(B, 0.005), rng.integers(100, 3000, B)
    y0 = rng.uniform(-5, 5, (B, d))
    y1, _, s1 = F.solve_batch("rossler", th, a, hs, Ns, y0, path="direct")
    y2, _, s2 = F.solve_batch("rossler", th, np.repeat(a[:, None], d, axis=1), hs, Ns, y0,
                              path="direct")
    assert np.array_equal(_to_np(y1), _to_np(y2)) and np.array_equal(_to_np(s1), _to_np(s2))


def test_blow_up_status_per_component(F, orc):
    """Chen with some orders above one leaves every bounded set; the first
    non-finite step matches the oracle's (or, at the top of the binary64
    range, comes one step apart, as for commensurate orders) and the earlier
    rows agree to the bound of _compare."""
    rng = np.random.default_rng(13)
    B = 6
    th = np.tile([35.0, 3.0, 28.0], (B, 1))
    al = np.column_stack([rng.uniform(1.2, 1.9, B), rng.uniform(0.8, 1.0, B),
                          rng.uniform(0.9, 1.5, B)])
    init = np.concatenate([np.tile([[[-9.0, -5.0, 14.0]]], (B, 1, 1)),
                           rng.uniform(-0.5, 0.5, (B, 1, 3))], axis=1)
    rst = _compare(F, orc, "chen", th, al, np.full(B, 0.001), np.full(B, 2500), init)
    assert np.any(rst > 0)


@pytest.mark.parametrize("sysname", ["vdp", "hindmarsh_rose", "linear3"])
@pytest.mark.parametrize("slope", [False, True])
def test_adjoint_per_component_orders(F, orc, sysname, slope):
    """Gradients with respect to y(0) (and y'(0)) and theta against the
    oracle's per-component reverse mode; components at or below order one get
    a zero y'(0) gradient."""
    sid, d, th_of = SYSTEMS[sysname]
    name = "linear" if sysname.startswith("linear") else sysname
    rng = np.random.default_rng(90 + sid + 10 * slope)
    B = 8
    th = np.stack([th_of(rng, i) for i in range(B)])
    al = rng.uniform(0.6, 2.0 if slope else 1.0, (B, d))
    if slope:
        al[0] = np.minimum(al[0], 1.0)
    hs = np.full(B, 0.01)
    Ns = rng.integers(200, 1500, B, endpoint=True)
    Ns[:2] = [1, 256]
    init = 0.5 * rng.uniform(-1, 1, (B, 2, d) if slope else (B, d))
    gy = rng.standard_normal((int((Ns + 1).sum()), d))
    gy0, gth, st = F.adjoint_batch(name, th, al, hs, Ns, init, gy)
    gy0, gth, st = _to_np(gy0), _to_np(gth), _to_np(st)
    off = np.concatenate([[0], np.cumsum(Ns + 1)[:-1]]).astype(np.int64)
    worst = 0.0
    for i in range(B):
        rg0, rgt, rst = orc.adjoint_orders(sid, th[i], al[i], hs[i], int(Ns[i]), init[i],
                                           gy[off[i]:off[i] + Ns[i] + 1])
        assert st[i] == rst == 0
        ref = np.concatenate([np.ravel(rg0), rgt])
        got = np.concatenate([np.ravel(gy0[i]), gth[i]])
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
        if slope:
            assert np.all(gy0[i][1][al[i] <= 1.0] == 0.0)
    assert worst <= 1e-10, worst


def test_autograd_per_component_orders(F):
    """torch.autograd through the two-call adjoint with per-component orders:
    gradients bitwise equal to the one-call adjoint."""
    import torch
    rng = np.random.default_rng(6)
    B, d = 4, 2
    th = torch.tensor(rng.uniform(0.5, 2, (B, 1)), device="cuda", requires_grad=True)
    init = torch.tensor(0.5 * rng.uniform(-1, 1, (B, 2, d)), device="cuda", requires_grad=True)
    al, hs = rng.uniform(0.7, 1.8, (B, d)), np.full(B, 0.01)
    Ns = np.array([600, 257, 1000, 40], dtype=np.int64)
    y = F.solve_batch_autograd(init, th, "vdp", al, hs, Ns)
    gy = torch.tensor(rng.standard_normal(tuple(y.shape)), device="cuda")
    (y * gy).sum().backward()
    g0, gt, _ = F.adjoint_batch("vdp", th.detach(), al, hs, Ns, init.detach(), gy)
    assert torch.equal(init.grad, g0) and torch.equal(th.grad, gt)
