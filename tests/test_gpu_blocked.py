"""GPU parity of the BLOCKED single-trajectory path (band + MFMA windows)
against the CPU oracle, through the C ABI. Same tolerances as the DIRECT
tests: 1e-11 normwise for non-chaotic systems over the whole trajectory; for
Chen, 1e-11 up to the oracle's own one-ulp sensitivity horizon."""
import numpy as np
import pytest

from tests import reduced_bounds as RB
from tests.conftest import gpu_available
from tests.test_gpu_direct import _batch_parity, _chen_horizon, _hr_theta, _to_np, relerr

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


@pytest.mark.parametrize("N", [1, 255, 256, 511, 600, 5000])
def test_blocked_linear_full_trajectory(F, orc, N):
    th, y0 = _lin(2, 31)
    y, st = F.solve("linear", th, 0.8, 0.01, N, y0, path="blocked")
    ref, _, _, rst = orc.solve(0, th, 0.8, 0.01, N, y0)
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


@pytest.mark.parametrize("sysname,d,theta,alpha,h,N", [
    ("vdp", 2, [1.3], 0.9, 0.01, 7000),
    ("financial", 3, [3.0, 0.1, 1.0], 0.85, 0.01, 4100),
    ("linear", 1, [-1.0, 0.0, 0.0], 0.5, 0.005, 2000),
    ("linear", 4, None, 0.95, 0.01, 3333),
])
def test_blocked_systems(F, orc, sysname, d, theta, alpha, h, N):
    rng = np.random.default_rng(5)
    if theta is None:
        theta, y0 = _lin(d, 9)
    else:
        y0 = rng.uniform(-1, 1, d) if sysname != "linear" else np.ones(d)
    y, st = F.solve(sysname, theta, alpha, h, N, y0, path="blocked")
    sid = {"vdp": 3, "financial": 4, "linear": 0}[sysname]
    ref, _, _, rst = orc.solve(sid, theta, alpha, h, N, y0)
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


def test_blocked_chen_prefix(F, orc):
    from paper_1611_08678_amd import workloads as W
    N = 1 << 14
    w = W.chen(N=N)
    hz, ref, _ = _chen_horizon(orc, w, N)
    y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, w["y0"][0],
                    path="blocked")
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert relerr(yy[:hz], ref[:hz]) <= 1e-11
    assert np.all(np.isfinite(yy)) and np.abs(yy).max() < 200.0


def test_blocked_deterministic_and_blowup(F, orc):
    from paper_1611_08678_amd import workloads as W
    w = W.chen(N=5000)
    ys = [_to_np(F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], 5000,
                         w["y0"][0], path="blocked")[0]) for _ in range(2)]
    assert np.array_equal(ys[0], ys[1])
    th = np.array([60.0, 0.0, 0.0])
    y, st = F.solve("linear", th, 0.9, 0.5, 2000, [1.0], path="blocked")
    _, _, _, rst = orc.solve(0, th, 0.9, 0.5, 2000, [1.0])
    assert int(st.item()) == rst > 0
    yy = _to_np(y)
    assert np.all(np.isnan(yy[rst:])) and np.all(np.isfinite(yy[:rst]))


def test_blocked_chen_full_size(F, orc):
    """Full N = 2^20 in the benchmark's launch configuration: finite, bounded,
    status 0, and the first 4096 steps match the oracle (before rounding
    differences of a chaotic system amplify)."""
    from paper_1611_08678_amd import workloads as W
    w = W.chen()
    N = int(w["N"][0])
    y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, w["y0"][0],
                    path="blocked")
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert np.all(np.isfinite(yy)) and np.abs(yy).max() < 200.0
    ref, _, _, _ = orc.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], 4096,
                             w["y0"][0])
    assert relerr(yy[:4097], ref) <= 1e-11
    # sampled rows anywhere in the trajectory: the oracle re-forms step t from
    # the GPU's own history (f_k = f(t_k, y_k) of the GPU rows). Both sides sum
    # the same terms; the bound is the teacher-forced contraction bound
    # 1e-13 times the magnitude of the history terms (h^alpha sum |w| |f|),
    # plus 4 u |y_t| for the update itself.
    u = np.finfo(np.float64).eps / 2
    wts = orc.weights(w["alpha"][0], N)
    f = orc.rhs_rows(w["system"], w["theta"][0], w["h"][0], yy)
    for t in (4097, 65541, 1 << 19, N - 257, N):
        yt, mag = orc.step_from_history(w["system"], w["theta"][0], w["alpha"][0], w["h"][0],
                                        t, w["y0"][0], f, wts)
        tol = 1e-13 * mag + 4 * u * np.abs(yt)
        assert np.all(np.abs(yy[t] - yt) <= tol), (t, yy[t], yt, mag)


def test_blocked_chen_attractor_statistics(F, orc):
    """Chen over N = 2^16 (T = 65.5): past the chaotic horizon trajectories of
    different rounding share only the attractor. Statistics over t >= 8.192
    (steps 8192 .. N) of the GPU trajectory against the average of three
    oracle runs (y0, and y0 with one component moved by one ulp either way).
    Tolerances from the spread of such runs (five oracle runs: relative
    standard deviation 0.05% for the mean of z, about 1% for the variances of
    x and y, 5% for the variance of z; the means of x and y, near zero on this
    symmetric attractor, within about 0.05 standard deviations of x): the mean
    of z within 1%, the variances of x and y within 4%, the means of x and y
    within 0.2 standard deviations of zero, and the trajectory bounded."""
    import threading
    from paper_1611_08678_amd import workloads as W
    N, lo = 1 << 16, 8192
    w = W.chen(N=N)
    y, st = F.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N, w["y0"][0],
                    path="blocked")
    yy = _to_np(y)
    assert int(st.item()) == 0 and np.all(np.isfinite(yy)) and np.abs(yy).max() < 60.0
    starts = [w["y0"][0].copy() for _ in range(3)]
    starts[1][0] = np.nextafter(starts[1][0], np.inf)
    starts[2][1] = np.nextafter(starts[2][1], -np.inf)
    refs = [None] * 3

    def run(k):
        refs[k] = orc.solve(w["system"], w["theta"][0], w["alpha"][0], w["h"][0], N,
                            starts[k])[0]

    ts = [threading.Thread(target=run, args=(k,)) for k in range(3)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    g_mean, g_var = yy[lo:].mean(0), yy[lo:].var(0)
    o_mean = np.mean([r[lo:].mean(0) for r in refs], axis=0)
    o_var = np.mean([r[lo:].var(0) for r in refs], axis=0)
    assert abs(g_mean[2] - o_mean[2]) <= 0.01 * abs(o_mean[2]), (g_mean, o_mean)
    assert np.all(np.abs(g_var[:2] - o_var[:2]) <= 0.04 * o_var[:2]), (g_var, o_var)
    assert np.all(np.abs(g_mean[:2]) <= 0.2 * np.sqrt(o_var[0])), (g_mean, o_var)


@pytest.mark.parametrize("far_prec", ["fp64", "fp32"])
def test_blocked_hindmarsh_rose(F, orc, far_prec):
    """Hindmarsh-Rose over 20000 steps, every row against the oracle (its
    one-ulp sensitivity horizon spans the trajectory): 1e-11 for FP64 windows.
    The bursts amplify perturbations (a single relative change of 2^-24 in y0
    grows about 200-fold in the oracle itself), so the FP32 windows, which
    round every far sum to binary32, are held to 30 times the oracle's own
    response to that single perturbation rather than to the bound of the
    non-spiking systems."""
    from paper_1611_08678_amd import workloads as W
    N = 20000
    w = W.hindmarsh_rose(N=N)
    th, a, h, y0 = w["theta"][0], w["alpha"][0], w["h"][0], w["y0"][0]
    y, st = F.solve("hindmarsh_rose", th, a, h, N, y0, path="blocked", far_prec=far_prec)
    ref, _, _, rst = orc.solve(w["system"], th, a, h, N, y0)
    assert int(st.item()) == rst == 0
    err = relerr(_to_np(y), ref)
    if far_prec == "fp64":
        assert err <= 1e-11
        return
    alt, _, _, _ = orc.solve(w["system"], th, a, h, N, y0 * (1 + 2.0 ** -24))
    assert 1e-12 < err <= 30 * relerr(alt, ref), (err, relerr(alt, ref))


def test_blocked_hindmarsh_rose_longest_table_size(F, orc):
    """The longest run of the paper's timing table (N = 3e6, T = 30000) in the
    launch configuration of the N sweep: status 0, finite and inside the
    attractor's box, the first 4096 rows against the oracle, and sampled rows
    anywhere re-formed by the oracle from the GPU's own history with the
    recursive-summation bound used for Chen at full size."""
    from paper_1611_08678_amd import workloads as W
    N = W.TABLE2_N[-1]
    w = W.hindmarsh_rose(N=N)
    th, a, h, y0 = w["theta"][0], w["alpha"][0], w["h"][0], w["y0"][0]
    y, st = F.solve("hindmarsh_rose", th, a, h, N, y0, path="blocked")
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert np.all(np.isfinite(yy))
    assert np.all(np.abs(yy[:, 0]) < 3) and np.all(np.abs(yy[:, 1]) < 20)
    assert np.all(np.abs(yy[:, 2]) < 6)
    ref, _, _, _ = orc.solve(w["system"], th, a, h, 4096, y0)
    assert relerr(yy[:4097], ref) <= 1e-11
    u = np.finfo(np.float64).eps / 2
    wts = orc.weights(a, N)
    f = orc.rhs_rows(w["system"], th, h, yy)
    for t in (4097, 100_000, 1_000_000, 2_000_003, N - 255, N):
        yt, mag = orc.step_from_history(w["system"], th, a, h, t, y0, f, wts)
        tol = 10.0 * np.sqrt(t) * u * mag + 4 * u * np.abs(yt)
        assert np.all(np.abs(yy[t] - yt) <= tol), (t, yy[t], yt, mag)


def test_blocked_hindmarsh_rose_longest_table_size_fp32(F, orc):
    """N = 3e6 with binary32 far windows: while a launch's far targets
    outnumber the far wavefronts (the first ~7650 launches) each target's
    window is split into one work unit per weight table, here in the binary32
    form. Status 0, finite and inside the attractor's box, and sampled rows,
    among them rows formed while those launches ran, re-formed by the oracle
    from the GPU's own history within 2^-17 of the history magnitude (the
    binary32 far sums round each term at 2^-24; the bound used for the
    Rossler batch at full size)."""
    from paper_1611_08678_amd import workloads as W
    N = W.TABLE2_N[-1]
    w = W.hindmarsh_rose(N=N)
    th, a, h, y0 = w["theta"][0], w["alpha"][0], w["h"][0], w["y0"][0]
    y, st = F.solve("hindmarsh_rose", th, a, h, N, y0, path="blocked", far_prec="fp32")
    yy = _to_np(y)
    assert int(st.item()) == 0
    assert np.all(np.isfinite(yy))
    assert np.all(np.abs(yy[:, 0]) < 3) and np.all(np.abs(yy[:, 1]) < 20)
    assert np.all(np.abs(yy[:, 2]) < 6)
    u = np.finfo(np.float64).eps / 2
    wts = orc.weights(a, N)
    f = orc.rhs_rows(w["system"], th, h, yy)
    for t in (4097, 100_000, 1_000_000, 1_900_003, 2_500_000, N):
        yt, mag = orc.step_from_history(w["system"], th, a, h, t, y0, f, wts)
        tol = 2.0 ** -17 * mag + 4 * u * np.abs(yt)
        assert np.all(np.abs(yy[t] - yt) <= tol), (t, yy[t], yt, mag)


def test_blocked_kernel_times(F):
    """The profiling interface reports one step launch per 256-row block."""
    import torch
    from paper_1611_08678_amd import workloads as W
    w = W.chen(N=20000)
    N, d = 20000, 3
    plan = F.fabm_plan(w["system"], d, "blocked", "fp64", 1, N)
    ws = torch.empty(F.fabm_workspace_size(plan, [N]), dtype=torch.uint8, device="cuda")
    y0 = torch.as_tensor(w["y0"][0], device="cuda")
    th = torch.as_tensor(w["theta"][0], device="cuda")
    y = torch.empty((N + 1, d), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int64, device="cuda")
    F.fabm_plan_set_profiling(plan, True)
    F.fabm_solve(plan, ws, float(w["alpha"][0]), float(w["h"][0]), N, y0, th, y, st)
    torch.cuda.synchronize()
    kt = F.fabm_plan_kernel_times(plan)
    assert kt["blocked_step"][1] == (N + 1 + 255) // 256
    assert kt["blocked_step"][0] > 0 and kt["weights"][1] == 1
    assert int(st.item()) == 0


def test_blocked_batch_rossler_ragged(F, orc):
    """Batched BLOCKED path: ragged lengths (one block to a dozen), per-instance
    alpha and y0, against the oracle's batch solver."""
    from paper_1611_08678_amd import workloads as W
    w = W.rossler_batch(batch=40, n_lo=1, n_hi=3000, seed=7)
    w["N"][:4] = [1, 255, 256, 511]  # edge lengths: one row, full block, block + 1 row
    _batch_parity(F, orc, w, path="blocked")


@pytest.mark.parametrize("sysname", ["vdp", "financial", "hindmarsh_rose", "linear2",
                                     "linear4"])
def test_blocked_batch_systems(F, orc, sysname):
    rng = np.random.default_rng(23)
    B = 12
    if sysname == "vdp":
        theta, d, sid = rng.uniform(0.5, 2, (B, 1)), 2, 3
    elif sysname == "financial":
        theta, d, sid = np.tile([3.0, 0.1, 1.0], (B, 1)), 3, 4
    elif sysname == "hindmarsh_rose":
        theta, d, sid = _hr_theta(rng, B), 3, 5
    else:
        d, sid = int(sysname[-1]), 0
        theta = np.stack([_lin(d, 100 + i)[0] for i in range(B)])
    w = dict(system=sid, d=d, theta=theta, alpha=rng.uniform(0.6, 1.0, B),
             h=rng.uniform(0.005, 0.02, B), N=rng.integers(200, 2500, B, endpoint=True),
             y0=rng.uniform(-1.5, 1.5, (B, d)))
    _batch_parity(F, orc, w, path="blocked")


def test_blocked_batch_blowup_and_determinism(F, orc):
    """Instances that blow up are flagged at the oracle's step with NaN rows
    after it, without disturbing the others; two runs agree bitwise."""
    lam = np.array([-1.0, 60.0, -2.0, 3.0, 1.2, -0.5])
    B = lam.size
    theta = np.stack([[l, 0.0, 0.0] for l in lam])
    w = dict(system=0, d=1, theta=theta, alpha=np.full(B, 0.9), h=np.full(B, 0.5),
             N=np.array([2000, 1500, 900, 2200, 1800, 700]), y0=np.ones((B, 1)))
    _batch_parity(F, orc, w, path="blocked")
    runs = [F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], w["N"], w["y0"],
                          path="blocked") for _ in range(2)]
    assert np.array_equal(_to_np(runs[0][0]), _to_np(runs[1][0]), equal_nan=True)


def test_blocked_blowup_rows_at_every_group_position(F, orc):
    """The band checks rows for non-finite values in groups of 8, one group
    late, and hands rows between wavefronts every 64 and between launches
    every 256: blow-ups placed at every position of a group, across a
    wavefront boundary (row 640) and a block boundary (row 768) are flagged
    at the oracle's step, with NaN rows after it and the rows before it at
    1e-11. y' = 20 y grows until binary64 overflows; y0 = 10^-k moves the
    first non-finite step by about two rows per k (steps 603..798)."""
    ks = list(range(0, 24)) + list(range(70, 100))
    B = len(ks)
    w = dict(system=0, d=1, theta=np.tile([20.0, 0.0, 0.0], (B, 1)), alpha=np.full(B, 0.9),
             h=np.full(B, 0.05), N=np.full(B, 1500),
             y0=np.array([[10.0 ** (-k)] for k in ks]))
    _batch_parity(F, orc, w, path="blocked")
    # the single-trajectory pipeline around the wavefront and block boundaries
    for k in (18, 19, 20, 83, 84, 85):
        th = np.array([20.0, 0.0, 0.0])
        y, st = F.solve("linear", th, 0.9, 0.05, 1500, [10.0 ** (-k)], path="blocked")
        ref, _, _, rst = orc.solve(0, th, 0.9, 0.05, 1500, [10.0 ** (-k)])
        g = int(st.item())
        assert g > 0 and abs(g - rst) <= 1, (k, g, rst)
        if g != rst:  # both sides at the top of the binary64 range (see _batch_parity)
            assert np.abs(ref[min(g, rst) - 1]).max() > np.finfo(np.float64).max / 1e3
        yy = _to_np(y)
        assert np.all(np.isnan(yy[g:])) and np.all(np.isfinite(yy[:g]))
        kk = min(g, rst)
        assert relerr(yy[:kk], ref[:kk]) <= 1e-11


# FP32 far windows: weights and history rounded to binary32 and 64 products
# per window summed in binary32, added to binary64 sums. A priori the far sum
# carries about (2 + 64) u32 sum|w||f| (u32 = 2^-24) and y a small multiple of
# h^alpha times that; the bound below is twice the largest error measured on
# MI355X for these cases, rounded up.
FP32_BOUND = 1e-5


def test_blocked_fp32_single(F, orc):
    th = [1.3]
    y0 = [0.8, -0.4]
    N = 7000
    ref, _, _, _ = orc.solve(3, th, 0.9, 0.01, N, y0)
    y64, _ = F.solve("vdp", th, 0.9, 0.01, N, y0, path="blocked", far_prec="fp64")
    y32, st = F.solve("vdp", th, 0.9, 0.01, N, y0, path="blocked", far_prec="fp32")
    e32, e64 = relerr(_to_np(y32), ref), relerr(_to_np(y64), ref)
    assert int(st.item()) == 0
    assert e64 <= 1e-11
    assert 1e-12 < e32 <= FP32_BOUND, e32  # binary32 windows did run, within the bound
    RB.check("blocked_fp32_single", e32, FP32_BOUND)


def test_blocked_fp32_batch(F, orc):
    from paper_1611_08678_amd import workloads as W
    w = W.rossler_batch(batch=24, n_lo=600, n_hi=3000, seed=11)
    worst = _batch_parity(F, orc, w, tol=FP32_BOUND, path="blocked_fp32")
    assert worst > 1e-12
    RB.check("blocked_fp32_batch", worst, FP32_BOUND)


@pytest.mark.skip(reason=(
    "single-launch persistent BLOCKED variant: its launch with far tasks (N=600, three "
    "blocks) did not complete on MI355X, twice; the cause was not found, so the variant was "
    "removed from the library and is never dispatched. The BLOCKED path is the step-kernel "
    "pipeline tested above (no inter-workgroup waits)."))
def test_blocked_persistent_variant_far_tasks():
    pass


@pytest.mark.parametrize("alpha", [0.05, 0.3, 1.0])
def test_blocked_alpha_range(F, orc, alpha):
    """Orders near the ends of (0, 1]: slowly decaying weights (alpha = 0.05)
    and the classical case (alpha = 1), over several blocks and a ragged tail."""
    th, y0 = _lin(3, 77)
    th[:9] *= 0.1  # eigenvalues near -0.2: the explicit predictor is stable at alpha = 0.05
    N = 1300
    y, st = F.solve("linear", th, alpha, 0.01, N, y0, path="blocked")
    ref, _, _, rst = orc.solve(0, th, alpha, 0.01, N, y0)
    assert int(st.item()) == rst == 0
    assert relerr(_to_np(y), ref) <= 1e-11


def test_blocked_batch_alpha_range(F, orc):
    """One batch, per-instance alpha from 0.05 to 1, ragged lengths."""
    rng = np.random.default_rng(71)
    al = np.array([0.05, 0.2, 0.5, 0.75, 0.99, 1.0])
    B, d = len(al), 2
    A = -(0.2 * np.eye(d)[None] + rng.standard_normal((B, d, d)) / 80)
    th = np.concatenate([A.reshape(B, -1), 0.1 * rng.standard_normal((B, 2 * d))], axis=1)
    w = dict(system=0, theta=th, alpha=al, h=np.full(B, 0.01),
             N=np.array([1200, 700, 2049, 256, 1, 900]), y0=rng.uniform(-1, 1, (B, d)))
    _batch_parity(F, orc, w, path="blocked")


@pytest.mark.parametrize("far_prec", ["fp32", "fp64"])
def test_blocked_batch_rossler_full_size(F, orc, far_prec):
    """The Rossler batch at full size (4096 instances, N 2^14..2^17, per-instance
    alpha) in the benchmark's launch configuration (FP32 far windows; FP64
    beside it): every status 0, every row finite and bounded; the first 2000
    rows of four instances against the oracle; and rows at t = 4097, N/2 and N
    of the longest, shortest and two other instances re-formed by the oracle
    from the GPU's own history. Bounds: FP64 as for Chen at full size; FP32
    windows round weights and history to binary32 and sum up to 64 products in
    binary32, at most 2^-18 of the history terms' magnitude (2^-17 the cap),
    and twice the measured error of these rows.
    About 2% of the starting points leave every bounded set within the first
    few hundred steps (the oracle finds 7 of the 300 shortest instances doing
    so, at steps 241-405): their status is checked against the oracle's for
    the three found there, and every such instance has finite rows before its
    status and NaN rows from it."""
    from paper_1611_08678_amd import workloads as W
    w = W.rossler_batch()
    Ns = w["N"]
    y, off, st = F.solve_batch(w["system"], w["theta"], w["alpha"], w["h"], Ns, w["y0"],
                               path="blocked", far_prec=far_prec)
    yy, gst = _to_np(y), _to_np(st)
    assert 0 < int((gst > 0).sum()) < 0.05 * len(Ns)
    for i in range(len(Ns)):
        rows = yy[off[i]: off[i] + Ns[i] + 1]
        k = int(gst[i]) if gst[i] else int(Ns[i]) + 1
        assert np.all(np.isfinite(rows[:k])) and np.abs(rows[:k]).max() < 1e300, i
        if gst[i] == 0:
            assert np.abs(rows).max() < 100.0, i
        else:
            assert np.all(np.isnan(rows[k:])), i
    u = np.finfo(np.float64).eps / 2
    wpre = wref = 0.0
    for i, rst in ((2902, 241), (988, 258), (1823, 307)):  # oracle statuses
        # FP64: the oracle's step, or one apart at the top of the binary64 range;
        # FP32 far operands overflow first, never later
        assert (abs(int(gst[i]) - rst) <= 1 if far_prec == "fp64" else 0 < gst[i] <= rst), \
            (i, gst[i], rst)
        ref, _, _, _ = orc.solve(w["system"], w["theta"][i], w["alpha"][i], w["h"][i], rst - 1,
                                 w["y0"][i])
        rows = yy[off[i]: off[i] + 200]
        e = relerr(rows, ref[:200])
        assert e <= (1e-5 if far_prec == "fp32" else 1e-11), i
        wpre = max(wpre, e)
    order = np.argsort(Ns)
    finite = [int(j) for j in order if gst[j] == 0]
    picks = [finite[-1], finite[0], finite[len(finite) // 3], 1234]
    assert gst[1234] == 0
    for i in picks:
        th, a, h, y0 = w["theta"][i], w["alpha"][i], w["h"][i], w["y0"][i]
        N = int(Ns[i])
        rows = yy[off[i]: off[i] + N + 1]
        ref, _, _, _ = orc.solve(w["system"], th, a, h, 2000, y0)
        e = relerr(rows[:2001], ref)
        assert e <= (1e-5 if far_prec == "fp32" else 1e-11), i
        wpre = max(wpre, e)
        wts = orc.weights(a, N)
        f = orc.rhs_rows(w["system"], th, h, rows)
        for t in (4097, N // 2, N):
            yt, mag = orc.step_from_history(w["system"], th, a, h, t, y0, f, wts)
            tol = (2.0 ** -17 * mag if far_prec == "fp32" else 1e-13 * mag)
            tol = tol + 4 * u * np.abs(yt)
            assert np.all(np.abs(rows[t] - yt) <= tol), (i, t, rows[t], yt, mag)
            wref = max(wref, float((np.maximum(np.abs(rows[t] - yt) - 4 * u * np.abs(yt), 0)
                                    / mag).max()))
    if far_prec == "fp32":
        RB.check("rossler_full_fp32_prefix", wpre, 1e-5)
        RB.check("rossler_full_fp32_reformed", wref, 2.0 ** -17)
