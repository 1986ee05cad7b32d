"""GPU parity of the sub-quadratic far history (plan field fft_level: dyadic
block squares of the far sums by FFT convolution, the rest on the
matrix-core windows) against the CPU oracle, through the C ABI.

The method's sums are unchanged (Section 2); only their rounding differs.
FFT convolution is accurate normwise: an output's error is about
log2(M) u ||v||_2 ||x||_2 for a transform of length M, weights v and history
x, instead of the per-term bound of a direct sum. The bars:
  * whole trajectories of non-chaotic systems: 1e-11 normwise, as for the
    matrix-core path;
  * Chen and the financial system: 1e-11 up to the oracle's own one-ulp
    sensitivity horizon (the row where a one-ulp change of y(0) has grown
    past 1e-13 of the scale in the oracle);
  * full size (N = 3e6): sampled rows re-formed by the oracle from the GPU's
    own history, to the recursive-summation bound of the other full-size
    tests plus 8 log2(M) u h^alpha max(||b||_2, ||a||_2) ||f_i||_2 over the
    rows the sum uses;
  * a level above the highest square runs no transform and must equal the
    matrix-core path bit for bit.
"""
import math

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.test_gpu_direct import _chen_horizon, _to_np, relerr

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
    th = np.concatenate([A.ravel(), rng.standard_normal(d), 0.05 * rng.standard_normal(d)])
    return th, rng.uniform(-1.5, 1.5, d)


def _top_level(N):
    """Highest square level for N steps (blocks of 256 rows): floor(log2(NB - 4))."""
    nb = (N + 1 + 255) // 256
    return int(math.floor(math.log2(nb - 4))) if nb - 4 >= 1 else -1


@pytest.mark.parametrize("level", [1, 2, 4, 6])
def test_fft_far_vdp_every_level(F, orc, level):
    """N = 2^15 (129 blocks, squares of levels up to 6: transforms of 1024 to
    65536 points, so both the single-pass and the four-step routes run)."""
    N, th, y0 = 1 << 15, [1.3], [0.4, -0.7]
    assert _top_level(N) == 6
    ref, _, _, rst = orc.solve(3, th, 0.9, 0.01, N, y0)
    y, st = F.solve("vdp", th, 0.9, 0.01, N, y0, path="blocked", fft_level=level)
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


@pytest.mark.parametrize("sysname,d,theta,alpha,h,N,level", [
    ("linear", 4, None, 0.95, 0.01, 20000, 1),
    ("linear", 1, [-1.0, 0.0, 0.0], 0.5, 0.005, 9000, 2),
    ("financial", 3, [3.0, 0.1, 1.0], 0.85, 0.01, 12345, 1),
    ("linear", 2, None, 0.3, 0.01, 6 * 256 - 1, 1),  # NB = 6: one square, half past the end
])
def test_fft_far_systems(F, orc, sysname, d, theta, alpha, h, N, level):
    rng = np.random.default_rng(5)
    if theta is None:
        theta, y0 = _lin(d, 9)
    else:
        y0 = rng.uniform(-1, 1, d) if sysname != "linear" else np.ones(d)
    sid = {"financial": 4, "linear": 0}[sysname]
    # the financial system amplifies a one-ulp change of y(0) to 2.8e-12 by
    # the last row in the oracle itself: compare up to the oracle's own
    # sensitivity horizon (the whole trajectory for the linear cases)
    w = dict(system=sid, theta=[np.asarray(theta, float)], alpha=[alpha], h=[h], y0=[y0])
    hz, ref, _ = _chen_horizon(orc, w, N)
    assert hz > (8000 if sysname == "financial" else N)
    y, st = F.solve(sysname, theta, alpha, h, N, y0, path="blocked", fft_level=level)
    assert int(st.item()) == 0
    assert relerr(_to_np(y)[:hz], ref[:hz]) <= 1e-11


def test_fft_far_with_initial_slope(F, orc):
    """Order 1.6 with y'(0): the Taylor term enters the band only."""
    th, _ = _lin(2, 4)
    init = np.array([[0.5, -0.2], [1.0, 0.3]])
    N = 15000
    ref, _, _, rst = orc.solve(0, th, 1.6, 0.002, N, init)
    y, st = F.solve("linear", th, 1.6, 0.002, N, init, path="blocked", fft_level=2)
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


def test_fft_far_chen_prefix(F, orc):
    from paper_1611_08678_amd import workloads as W
    N = 1 << 14
    w = W.chen(N=N)
    hz, ref, _ = _chen_horizon(orc, w, N)
    y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, w["y0"][0],
                    path="blocked", fft_level=1)
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert relerr(yy[:hz], ref[:hz]) <= 1e-11
    assert np.all(np.isfinite(yy)) and np.abs(yy).max() < 200.0


def test_fft_far_above_top_level_is_matrix_core_path(F):
    N, th, y0 = 1 << 15, [1.3], [0.4, -0.7]
    a, _ = F.solve("vdp", th, 0.9, 0.01, N, y0, path="blocked")
    for level in (_top_level(N) + 1, 15):
        b, _ = F.solve("vdp", th, 0.9, 0.01, N, y0, path="blocked", fft_level=level)
        assert np.array_equal(_to_np(a), _to_np(b))


def test_fft_far_deterministic_and_blowup(F, orc):
    th, y0 = [1.3], [0.4, -0.7]
    ys = [_to_np(F.solve("vdp", th, 0.9, 0.01, 9000, y0, path="blocked", fft_level=1)[0])
          for _ in range(2)]
    assert np.array_equal(ys[0], ys[1])
    th = np.array([60.0, 0.0, 0.0])
    y, st = F.solve("linear", th, 0.9, 0.5, 6000, [1.0], path="blocked", fft_level=1)
    _, _, _, rst = orc.solve(0, th, 0.9, 0.5, 6000, [1.0])
    assert int(st.item()) == rst > 0
    yy = _to_np(y)
    assert np.all(np.isnan(yy[rst:])) and np.all(np.isfinite(yy[:rst]))


def test_fft_far_kernel_class_and_unsupported(F):
    import torch
    N = 20000
    plan = F.fabm_plan("vdp", 2, "blocked", "fp64", 1, N, fft_level=3)
    ws = torch.empty(F.fabm_workspace_size(plan, [N]), dtype=torch.uint8, device="cuda")
    y0 = torch.tensor([0.4, -0.7], dtype=torch.float64, device="cuda")
    th = torch.tensor([1.3], dtype=torch.float64, device="cuda")
    y = torch.empty((N + 1, 2), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int64, device="cuda")
    F.fabm_plan_set_profiling(plan, True)
    F.fabm_solve(plan, ws, 0.9, 0.01, N, y0, th, y, st)
    torch.cuda.synchronize()
    kt = F.fabm_plan_kernel_times(plan)
    # NB = 79: one spectra launch plus one square per launch s with ctz(s + 2) in 3..6
    nb = (N + 1 + 255) // 256
    squares = sum(1 for s in range(nb - 5)
                  if 3 <= ((s + 2) & -(s + 2)).bit_length() - 1 <= _top_level(N))
    assert kt["fft_far"][1] == 1 + squares and kt["fft_far"][0] > 0
    assert kt["blocked_step"][1] == nb
    with pytest.raises(RuntimeError, match="unsupported"):
        F.fabm_adjoint_workspace_size(plan, [N])  # the reverse pass has no FFT form


def test_fft_far_hindmarsh_rose_longest_table_size(F, orc):
    """N = 3e6 in the benchmark's configuration of the variant (fft_level 8):
    status 0, bounded, the first 4096 rows against the oracle, and sampled
    rows re-formed by the oracle from the GPU's own history."""
    from paper_1611_08678_amd import workloads as W
    N = W.TABLE2_N[-1]
    w = W.hindmarsh_rose(N=N)
    th, a, h, y0 = w["theta"][0], w["alpha"][0], w["h"][0], w["y0"][0]
    y, st = F.solve("hindmarsh_rose", th, a, h, N, y0, path="blocked", fft_level=8)
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert np.all(np.isfinite(yy))
    assert np.all(np.abs(yy[:, 0]) < 3) and np.all(np.abs(yy[:, 1]) < 20)
    assert np.all(np.abs(yy[:, 2]) < 6)
    ref, _, _, _ = orc.solve(w["system"], th, a, h, 4096, y0)
    assert relerr(yy[:4097], ref) <= 1e-11
    u = np.finfo(np.float64).eps / 2
    wts = orc.weights(a, N)
    b_, a_ = wts[0], wts[1]
    f = orc.rhs_rows(w["system"], th, h, yy)
    log2M = 9 + _top_level(N)
    for t in (4097, 100_000, 1_000_000, 2_000_003, N - 255, N):
        yt, mag = orc.step_from_history(w["system"], th, a, h, t, y0, f, wts)
        wn = max(np.linalg.norm(b_[:t]), np.linalg.norm(a_[:t]))
        fn = np.linalg.norm(f[:t], axis=0)
        fft = 8.0 * log2M * u * h ** a * wn * fn
        tol = 10.0 * np.sqrt(t) * u * mag + 4 * u * np.abs(yt) + fft
        assert np.all(np.abs(yy[t] - yt) <= tol), (t, yy[t], yt, mag, fft)


def test_fft_far_with_fp32_windows(F, orc):
    """FP32 windows inside each group, binary64 transforms for the squares:
    the FP32 path's bound (the far sums of the windows rounded to binary32)."""
    from tests.test_gpu_blocked import FP32_BOUND
    N, th, y0 = 1 << 15, [1.3], [0.8, -0.4]
    ref, _, _, rst = orc.solve(3, th, 0.9, 0.01, N, y0)
    y, st = F.solve("vdp", th, 0.9, 0.01, N, y0, path="blocked", far_prec="fp32", fft_level=2)
    err = relerr(_to_np(y), ref)
    assert int(st.item()) == rst == 0
    assert 1e-12 < err <= FP32_BOUND, err
    from tests import reduced_bounds as RB
    RB.check("fft_far_fp32_windows", err, FP32_BOUND)


@pytest.mark.parametrize("alphas,slope", [([0.75, 0.95], False), ([0.85, 1.5], True)])
def test_fft_far_per_component_orders(F, orc, alphas, slope):
    """One weight spectrum per component (non-commensurate orders), with y'(0)
    for the component above order one."""
    N, th, h = 20000, [1.1], 0.005
    init = np.array([[0.5, -0.3], [0.2, 0.4]]) if slope else np.array([0.5, -0.3])
    ref, _, _, rst = orc.solve_orders(orc.VDP, th, alphas, h, N, init)
    plan = F.fabm_plan("vdp", 2, "blocked", "fp64", 1, N, initial_slope=slope,
                       per_component_order=True, fft_level=2)
    y, off, st = F.solve_batch("vdp", np.reshape(th, (1, -1)), np.reshape(alphas, (1, -1)),
                               [h], [N], init[None], plan=plan)
    assert int(st.cpu().numpy()[0]) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


def test_fft_far_graph_replays_match_eager(F):
    """The FFT squares are ordinary launches on the call's stream: a captured
    solve of a plan with fft_level replays (with new initial values each time,
    and eager solves in between) bit for bit like the eager call."""
    import torch
    N, d = 1 << 15, 2
    th = np.array([[1.3]])
    Ns = np.array([N], dtype=np.int64)
    gplan = F.fabm_plan("vdp", d, "blocked", "fp64", 1, N, fft_level=2)
    eplan = F.fabm_plan("vdp", d, "blocked", "fp64", 1, N, fft_level=2)
    ws = F._workspace(F.fabm_workspace_size(gplan, Ns))
    y0s = np.array([[0.4, -0.7]])
    y0 = torch.tensor(y0s, device="cuda")
    thd = torch.tensor(th, device="cuda")
    y = torch.full((N + 1, d), -7.0, dtype=torch.float64, device="cuda")
    st = torch.full((1,), -3, dtype=torch.int64, device="cuda")
    g = F.fabm_graph_solve_batch(gplan, ws, [0.9], [0.01], Ns, y0, thd, [0], y, st)
    torch.cuda.synchronize()
    assert torch.all(y == -7.0)
    for rep in range(3):
        y0.copy_(torch.tensor(y0s * (1.0 + 0.05 * rep), device="cuda"))
        g.launch()
        torch.cuda.synchronize()
        got, gst = y.clone(), st.clone()
        ref, _, rst = F.solve_batch("vdp", thd, [0.9], [0.01], Ns, y0, plan=eplan)
        torch.cuda.synchronize()
        assert torch.equal(gst, rst) and int(rst.item()) == 0, rep
        assert torch.equal(got, ref), rep
    del g
    torch.cuda.synchronize()
