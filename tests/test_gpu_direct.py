"""GPU parity of the weight generation and the DIRECT path against the CPU
oracle (Section 2 of arXiv:1611.08678), called through the C ABI.

Tolerances:
  * weights: binary64 evaluation of cancellation-free forms vs the oracle's
    binary128 evaluation of the defining formulas: <= 32 ulp per entry and
    <= 4 ulp on average. The forms round 4-6 times and call pow, expm1 and
    log1p of the device math library; measured on MI355X: max 17 ulp (b at
    alpha = 0.95, m ~ 7e5), mean 2.95 ulp (b at alpha = 0.8). 32 ulp is a
    relative 7e-15, three orders below what the 1e-11 trajectory bound can
    feel;
  * FP64 trajectories of non-chaotic systems: normwise relative error
    max_n |y_n - y_n^ref|_inf / max_n |y_n^ref|_inf <= 1e-11;
  * chaotic systems (Chen): the same bound on the prefix before a one-ulp
    perturbation of y0 grows past 1e-13 in the oracle itself, plus
    teacher-forced history sums within 1e-13 * sum |w||f| at every target.
"""
import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def F():
    import paper_1611_08678_amd as F
    F.load()
    return F


def relerr(y, ref):
    return np.abs(y - ref).max() / np.abs(ref).max()


def _to_np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("alpha", [0.1, 0.5, 0.8, 0.95, 1.0])
def test_weights_parity(F, orc, alpha):
    import torch
    n = (1 << 20) if alpha == 0.95 else (1 << 16)
    b, a, c = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
    F.fabm_weights(alpha, n, b, a, c)
    torch.cuda.synchronize()
    rb, ra, rc = orc.weights(alpha, n)
    for got, ref, name in ((b, rb, "b"), (a, ra, "a"), (c, rc, "c")):
        g = _to_np(got)
        ulps = np.abs(g - ref) / np.spacing(np.abs(ref))
        assert ulps.max() <= 32, (name, int(np.argmax(ulps)), ulps.max())
        assert ulps.mean() <= 4.0, (name, ulps.mean())


def test_scalar_linear_direct(F, orc):
    from paper_1611_08678_amd import workloads as W
    w = W.scalar_linear()
    y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], int(w["N"][0]),
                    w["y0"][0], path="direct")
    ref, _, _, rst = orc.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0],
                               int(w["N"][0]), w["y0"][0])
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


def _batch_parity(F, orc, w, tol=1e-11, path="direct"):
    path, _, prec = path.partition("_")
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                               path=path, far_prec=prec or "fp64")
    ref, roff, rst = orc.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"])
    assert np.array_equal(off, roff)
    yy = _to_np(y)
    gst = _to_np(st)
    worst = 0.0
    for i in range(len(off)):
        sl = slice(off[i], off[i] + int(w["N"][i]) + 1)
        if gst[i] != rst[i]:
            # The first non-finite step is decided at the top of the binary64
            # range: the oracle rounds the whole corrector sum C_t to binary64,
            # the GPU band adds the newest history term after scaling by h^alpha,
            # so one side may overflow one step before the other. Accepted only
            # when the last row both agree on is within 1e3 of the overflow.
            k = int(min(gst[i], rst[i]))
            assert k > 0 and abs(int(gst[i]) - int(rst[i])) == 1, (i, gst[i], rst[i])
            assert np.abs(ref[sl][k - 1]).max() > np.finfo(np.float64).max / 1e3, (i, k)
        if gst[i]:
            assert np.all(np.isnan(yy[sl][int(gst[i]):]))
        if rst[i] or gst[i]:
            k = int(min(x for x in (gst[i], rst[i]) if x))
            worst = max(worst, relerr(yy[sl][:k], ref[sl][:k]))
        else:
            worst = max(worst, relerr(yy[sl], ref[sl]))
    assert worst <= tol, worst
    return worst


def test_rossler_ragged_batch_direct(F, orc):
    from paper_1611_08678_amd import workloads as W
    w = W.rossler_batch(batch=24, n_lo=100, n_hi=1500, seed=7)
    _batch_parity(F, orc, w)


def _hr_theta(rng, B):
    """Hindmarsh-Rose parameters of the bursting set with the applied current I
    drawn from [2.5, 3.5] per instance."""
    from paper_1611_08678_amd import workloads as W
    theta = np.tile(W.HR_THETA, (B, 1))
    theta[:, 7] = rng.uniform(2.5, 3.5, B)
    return theta


@pytest.mark.parametrize("sysname", ["vdp", "financial", "hindmarsh_rose", "linear1", "linear2",
                                     "linear3", "linear4"])
def test_systems_direct(F, orc, sysname):
    rng = np.random.default_rng(17)
    B = 6
    if sysname == "vdp":
        theta, d, sid = rng.uniform(0.5, 2, (B, 1)), 2, 3
    elif sysname == "financial":
        theta, d, sid = np.tile([3.0, 0.1, 1.0], (B, 1)), 3, 4
    elif sysname == "hindmarsh_rose":
        theta, d, sid = _hr_theta(rng, B), 3, 5
    else:
        d, sid = int(sysname[-1]), 0
        A = -(2 * np.eye(d) + rng.standard_normal((B, d, d)) / 8)
        theta = np.concatenate([A.reshape(B, -1), rng.standard_normal((B, d)),
                                0.1 * rng.standard_normal((B, d))], axis=1)
    w = dict(system=sid, theta=theta, alpha=rng.uniform(0.6, 1.0, B), h=np.full(B, 0.01),
             N=rng.integers(50, 900, B), y0=rng.uniform(-1.5, 1.5, (B, d)))
    _batch_parity(F, orc, w)


def test_hindmarsh_rose_direct(F, orc):
    """The Hindmarsh-Rose neuron over 20000 steps (T = 200, several bursts):
    the oracle's own one-ulp sensitivity horizon spans the whole trajectory, so
    every row is compared."""
    from paper_1611_08678_amd import workloads as W
    w = W.hindmarsh_rose(N=20000)
    y, st = F.solve("hindmarsh_rose", w["theta"][0], w["alpha"][0], w["h"][0], 20000,
                    w["y0"][0], path="direct")
    ref, _, _, rst = orc.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], 20000,
                               w["y0"][0])
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


def test_blow_up_status_matches_oracle(F, orc):
    B = 4
    A = np.array([-1.0, 60.0, -2.0, 40.0]).reshape(B, 1, 1)
    theta = np.concatenate([A.reshape(B, 1), np.zeros((B, 2))], axis=1)
    w = dict(system=0, theta=theta, alpha=np.full(B, 0.9), h=np.full(B, 0.5),
             N=np.array([300, 400, 350, 500]), y0=np.ones((B, 1)))
    _batch_parity(F, orc, w)


def _chen_horizon(orc, w, N, thresh=1e-13):
    """First row where a one-ulp change of y0 has grown past `thresh` (normwise)
    in the oracle itself: beyond it no two correct FP64 runs need agree."""
    y0 = w["y0"][0]
    ref, _, f, _ = orc.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, y0)
    y0p = y0.copy()
    y0p[0] = np.nextafter(y0p[0], np.inf)
    alt, _, _, _ = orc.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, y0p)
    scale = np.abs(ref).max()
    bad = np.nonzero(np.abs(alt - ref).max(axis=1) > thresh * scale)[0]
    return (int(bad[0]) if bad.size else N + 1), ref, f


def test_chen_grid_direct_prefix_and_teacher_forced(F, orc):
    import torch
    from paper_1611_08678_amd import workloads as W
    N = 1 << 14  # >= the single-trajectory grid threshold
    w = W.chen(N=N)
    hz, ref, fref = _chen_horizon(orc, w, N)
    assert hz > 500
    y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, w["y0"][0],
                    path="direct")
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert relerr(yy[:hz], ref[:hz]) <= 1e-11
    assert np.all(np.isfinite(yy)) and np.abs(yy).max() < 200.0
    # teacher forcing: contract the oracle's own history on the GPU
    fh = torch.as_tensor(fref[:N], device="cuda").contiguous()
    P = torch.empty_like(fh)
    Cs = torch.empty_like(fh)
    ws = torch.empty(F.fabm_history_workspace_size(N, 3), dtype=torch.uint8, device="cuda")
    F.fabm_history_sums(w["alpha"][0], N, 3, fh, P, Cs, "direct", "fp64", ws)
    rP, rC, aP, aC = orc.history_sums(w["alpha"][0], fref[:N])
    assert np.all(np.abs(_to_np(P) - rP) <= 1e-13 * aP + 1e-300)
    assert np.all(np.abs(_to_np(Cs) - rC) <= 1e-13 * aC + 1e-300)


def test_grid_direct_blowup(F, orc):
    """The whole-GPU kernel (N >= 8192 single trajectory): y' = 2 y overflows
    binary64 at the oracle's step; every workgroup forms that row, finds it
    non-finite and stops at the same step; rows after it are NaN."""
    th = np.array([2.0, 0.0, 0.0])
    N = 9000
    y, st = F.solve("linear", th, 0.9, 0.05, N, [1.0], path="direct")
    ref, _, _, rst = orc.solve(0, th, 0.9, 0.05, N, [1.0])
    g = int(st.item())
    assert rst > 0 and abs(g - rst) <= 1, (g, rst)
    if g != rst:  # both sides at the top of the binary64 range (see _batch_parity)
        assert np.abs(ref[min(g, rst) - 1]).max() > np.finfo(np.float64).max / 1e3
    yy = _to_np(y)
    assert np.all(np.isnan(yy[g:])) and np.all(np.isfinite(yy[:g]))
    k = min(g, rst)
    assert relerr(yy[:k], ref[:k]) <= 1e-11


def test_grid_direct_deterministic(F):
    from paper_1611_08678_amd import workloads as W
    w = W.chen(N=9000)
    ys = []
    for _ in range(2):
        y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], 9000, w["y0"][0],
                        path="direct")
        ys.append(_to_np(y))
    assert np.array_equal(ys[0], ys[1])


def test_direct_vdp_batch_full_size(F, orc):
    """The Van der Pol batch at full size (1024 instances, N = 2^15) on the
    DIRECT workgroup-per-instance kernel, as the benchmark runs it: every status
    0, every row finite, and two whole instances against the oracle."""
    from paper_1611_08678_amd import workloads as W
    w = W.vdp_adjoint()
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                               path="direct")
    yy, gst = _to_np(y), _to_np(st)
    assert np.all(gst == 0) and np.all(np.isfinite(yy))
    N = int(w["N"][0])
    for i in (0, 777):
        ref, _, _, rst = orc.solve(w["system"], w["theta"][i], w["alpha"][i], w["h"][i], N,
                                   w["y0"][i])
        assert rst == 0 and relerr(yy[off[i]: off[i] + N + 1], ref) <= 1e-11, i
