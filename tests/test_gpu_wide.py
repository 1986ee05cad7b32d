"""GPU parity of the shared-grid batch path (LINEAR systems whose instances
share alpha, h and N: 64-row blocks, far sums of all instances as one
Toeplitz-times-history product on the matrix cores, one wavefront per
instance for the rows of a block) against the CPU oracle, through the C ABI.

Tolerances: FP64 far tiles 1e-11 normwise over whole trajectories (the
arithmetic is the oracle's up to summation order). FP32 and FP16X2 far tiles:
twice the error measured for each case (tests/reduced_bounds.py, with the
a-priori model: operands carry 24 (FP32) or 22 (hi + lo) significant bits and
each block of 64 source rows is summed in binary32 before it is added in
binary64, so a far sum is off by at most ~64 u32 of its magnitude), under the
sanity cap 1e-5 normwise."""
import numpy as np
import pytest

from tests import reduced_bounds as RB
from tests.conftest import gpu_available
from tests.test_gpu_direct import _batch_parity, _to_np, relerr

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

REDUCED_BOUND = 1e-5


@pytest.fixture(scope="module")
def F():
    import paper_1611_08678_amd as F
    F.load()
    return F


def _linear_batch(B, d, N, seed, blow=None, alpha=0.8, h=0.01, scale=1.0):
    rng = np.random.default_rng(seed)
    A = -scale * (2 * np.eye(d)[None] + rng.standard_normal((B, d, d)) / 8)
    if blow is not None:
        for i, g in blow.items():
            A[i] += g * np.eye(d)
    th = np.concatenate([A.reshape(B, -1), 0.1 * rng.standard_normal((B, d)),
                         0.05 * rng.standard_normal((B, d))], axis=1)
    return dict(system="linear", theta=th, alpha=np.full(B, alpha), h=np.full(B, h),
                N=np.full(B, N, dtype=np.int64), y0=rng.standard_normal((B, d)))


def _parity(F, orc, w, prec, tol, tile_L=0):
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                               path="blocked", far_prec=prec, tile_L=tile_L)
    ref, roff, rst = orc.solve_batch(0, w["theta"], w["alpha"], w["h"], w["N"], w["y0"])
    assert np.array_equal(off, roff)
    yy, gst = _to_np(y), _to_np(st)
    assert np.array_equal(gst, rst), (gst, rst)
    worst = 0.0
    for i in range(len(off)):
        sl = slice(off[i], off[i] + int(w["N"][i]) + 1)
        k = int(rst[i]) or int(w["N"][i]) + 1
        worst = max(worst, relerr(yy[sl][:k], ref[sl][:k]))
        if rst[i]:
            assert np.all(np.isnan(yy[sl][k:]))
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("B,d,N", [(3, 64, 700), (7, 5, 500), (2, 17, 1), (4, 8, 63),
                                   (3, 33, 64), (5, 6, 129)])
def test_wide_fp64_matches_oracle(F, orc, B, d, N):
    _parity(F, orc, _linear_batch(B, d, N, seed=B * 100 + d), "fp64", 1e-11)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_wide_small_states_when_asked(F, orc, d):
    """The 64-row shared-grid form for d <= 4 (tile_L = 64)."""
    _parity(F, orc, _linear_batch(6, d, 400, seed=40 + d), "fp64", 1e-11, tile_L=64)


@pytest.mark.parametrize("prec", ["fp32", "fp16x2"])
def test_wide_reduced_precision(F, orc, prec):
    worst = _parity(F, orc, _linear_batch(3, 64, 900, seed=11), prec, REDUCED_BOUND)
    assert worst > 1e-12  # the far tiles really ran in reduced precision
    RB.check(f"wide_reduced_{prec}", worst, REDUCED_BOUND)


@pytest.mark.parametrize("prec", ["fp64", "fp16x2"])
def test_wide_blowup_status(F, orc, prec):
    """Instances 1 and 3 overflow (binary64) at different steps; the others
    stay finite. The split binary16 operands carry their scale, so they
    overflow where binary64 does."""
    w = _linear_batch(5, 4, 500, seed=5, blow={1: 300.0, 3: 150.0})
    worst = _parity(F, orc, w, prec, 1e-11 if prec == "fp64" else REDUCED_BOUND)
    if prec != "fp64":
        RB.check(f"wide_blowup_{prec}", worst, REDUCED_BOUND)


def test_wide_fp32_blowup_within_binary32_range(F, orc):
    """Binary32 far operands overflow once |f| passes 3.4e38, so an instance
    that blows up is reported at the first block whose far sums hold such a
    value: no later than the binary64 oracle, rows before agree, rows from the
    status on are NaN; finite instances are unaffected."""
    w = _linear_batch(5, 4, 500, seed=5, blow={1: 300.0, 3: 150.0})
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                               path="blocked", far_prec="fp32")
    ref, _, rst = orc.solve_batch(0, w["theta"], w["alpha"], w["h"], w["N"], w["y0"])
    yy, gst = _to_np(y), _to_np(st)
    worst = 0.0
    for i in range(5):
        sl = slice(off[i], off[i] + 501)
        if rst[i] == 0:
            assert gst[i] == 0
            worst = max(worst, relerr(yy[sl], ref[sl]))
            continue
        k = int(gst[i])
        assert 0 < k <= rst[i]
        assert np.all(np.isnan(yy[sl][k:]))
        worst = max(worst, relerr(yy[sl][:k], ref[sl][:k]))
        # the far sums at step k hold a history value beyond binary32's range
        assert np.abs(ref[sl][:k]).max() > 1e30 or k == rst[i]
    RB.check("wide_fp32_blowup", worst, REDUCED_BOUND)


def test_wide_rejects_unshared_grid(F):
    w = _linear_batch(3, 8, 100, seed=2)
    w["alpha"][1] = 0.7
    with pytest.raises(F.FabmError) as e:
        F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"])
    assert e.value.code == 2


@pytest.mark.parametrize("prec", ["fp64", "fp16x2"])
def test_wide_deterministic(F, prec):
    w = _linear_batch(6, 16, 700, seed=9)
    args = (w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"])
    y1, _, s1 = F.solve_batch(*args, far_prec=prec)
    y2, _, s2 = F.solve_batch(*args, far_prec=prec)
    assert np.array_equal(_to_np(y1), _to_np(y2)) and np.array_equal(_to_np(s1), _to_np(s2))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x2"])
def test_wide_linear64_full_size(F, orc, prec):
    """The linear d = 64 workload at full size (512 instances, N = 2^16), in
    the benchmark's launch configuration: every status 0, sampled instances
    finite and bounded, their first 1500 steps against the oracle, and sampled
    rows anywhere re-formed by the oracle from the GPU's own history (f_k =
    f(t_k, y_k) of the GPU rows). FP64 bound: 1e-13 times the magnitude
    of the history terms (the teacher-forced contraction bound) plus 4 u |y_t|;
    reduced precision: twice the measured error, relative to that magnitude."""
    import torch
    from paper_1611_08678_amd import workloads as W
    w = W.linear64_batch()
    B, d, N = 512, 64, int(w["N"][0])
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                               path="blocked", far_prec=prec)
    assert int(_to_np(st).max()) == 0 and int(_to_np(st).min()) == 0
    u = np.finfo(np.float64).eps / 2
    wts = orc.weights(0.8, N)
    wpre = wref = 0.0
    for i in (0, 257, 511):
        yi = y[int(off[i]):int(off[i]) + N + 1].cpu().numpy()
        assert np.all(np.isfinite(yi)) and np.abs(yi).max() < 1e3
        ref, _, _, rst = orc.solve(0, w["theta"][i], 0.8, 0.01, 1500, w["y0"][i])
        assert rst == 0
        e = relerr(yi[:1501], ref)
        assert e <= (1e-11 if prec == "fp64" else REDUCED_BOUND)
        wpre = max(wpre, e)
        f = orc.rhs_rows(0, w["theta"][i], 0.01, yi)
        for t in (1501, 20000 + i, N - 63, N):
            yt, mag = orc.step_from_history(0, w["theta"][i], 0.8, 0.01, t, w["y0"][i], f, wts)
            tol = (1e-13 if prec == "fp64" else REDUCED_BOUND) * mag + 4 * u * np.abs(yt)
            assert np.all(np.abs(yi[t] - yt) <= tol), (i, t, np.abs(yi[t] - yt).max(), mag.max())
            wref = max(wref, float((np.maximum(np.abs(yi[t] - yt) - 4 * u * np.abs(yt), 0)
                                    / mag).max()))
    if prec != "fp64":
        RB.check(f"wide_linear64_{prec}_prefix", wpre, REDUCED_BOUND)
        RB.check(f"wide_linear64_{prec}_reformed", wref, REDUCED_BOUND)
    del y, st
    torch.cuda.empty_cache()


def test_wide_linear64_fp64_full_trajectories_2p14(F, orc):
    """The d = 64 workload's systems (A = -(2 I + G/8), seed 3) at N = 2^14 on
    the shared grid with FP64 far tiles: the whole trajectories of three
    instances (first, middle, last of the batch of 512) against the oracle at
    1e-11 normwise (the system is stable, so parity holds at every step)."""
    from paper_1611_08678_amd import workloads as W
    w = W.linear64_batch(N=1 << 14)
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                               path="blocked", far_prec="fp64")
    assert int(_to_np(st).max()) == 0
    idx = np.array([0, 255, 511])
    ref, roff, rst = orc.solve_batch(0, w["theta"][idx], w["alpha"][idx], w["h"][idx],
                                     w["N"][idx], w["y0"][idx])
    assert np.all(rst == 0)
    N = 1 << 14
    for k, i in enumerate(idx):
        yi = y[int(off[i]):int(off[i]) + N + 1].cpu().numpy()
        assert relerr(yi, ref[roff[k]:roff[k] + N + 1]) <= 1e-11, i


@pytest.mark.parametrize("prec", ["fp16x2", "fp32"])
def test_wide_instances_of_very_different_magnitude(F, orc, prec):
    """Scaling y0, b0 and b1 of a linear system by k scales its solution by k.
    Instances 1e-8 .. 1e12 apart share the far product; each history column
    carries its own power-of-two scale (FP16X2), so every instance keeps its
    own relative accuracy (normwise per instance)."""
    w = _linear_batch(4, 12, 600, seed=13)
    d = 12
    for i, k in enumerate([1e-8, 1.0, 1e5, 1e12]):
        w["y0"][i] *= k
        w["theta"][i, d * d:] *= k
    RB.check(f"wide_magnitudes_{prec}", _parity(F, orc, w, prec, REDUCED_BOUND), REDUCED_BOUND)


@pytest.mark.parametrize("alpha", [0.05, 1.0])
def test_wide_alpha_range(F, orc, alpha):
    # eigenvalues near -0.2: the explicit predictor is stable at alpha = 0.05
    w = _linear_batch(3, 9, 700, seed=17, alpha=alpha, scale=0.1)
    assert np.all(orc.solve_batch(0, w["theta"], w["alpha"], w["h"], w["N"], w["y0"])[2] == 0)
    _parity(F, orc, w, "fp64", 1e-11)
    RB.check(f"wide_alpha{alpha}_fp16x2", _parity(F, orc, w, "fp16x2", REDUCED_BOUND),
             REDUCED_BOUND)
