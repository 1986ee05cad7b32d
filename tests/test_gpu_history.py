"""Teacher-forced history sums (the Section 2 predictor sum of eq. (2) and the
corrector sum) on the GPU, fed a given history, against the oracle's sums of
the same history at every target.

BLOCKED runs the solver's own step pipeline (band walk, near and far MFMA
windows of 256-row blocks) with f read from the given rows, so these tests
check the contraction the BLOCKED solver uses, free of the chaotic growth that
limits trajectory parity on Chen. Bound: 1e-13 * sum |w| |f| per target and
component for binary64 (the oracle's long-double magnitude sums); binary32
far windows: every operand rounded once (2u) and each window of 64 products
summed in binary32 (64u), u = 2^-24, so (2 + 64) u * sum |w| |f|."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.test_gpu_direct import _to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

FP64_BOUND = 1e-13
FP32_BOUND = 66 * 2.0 ** -24


@pytest.fixture(scope="module")
def F():
    import paper_1611_08678_amd as F
    F.load()
    return F


def _gpu_sums(F, alpha, f, path="blocked", far_prec="fp64"):
    import torch
    N, d = f.shape
    fh = torch.as_tensor(np.ascontiguousarray(f), device="cuda")
    P = torch.full_like(fh, np.nan)
    Cs = torch.full_like(fh, np.nan)
    ws = torch.empty(F.fabm_history_workspace_size(N, d), dtype=torch.uint8, device="cuda")
    F.fabm_history_sums(alpha, N, d, fh, P, Cs, path, far_prec, ws)
    torch.cuda.synchronize()
    return _to_np(P), _to_np(Cs)


def _check(P, C, rP, rC, aP, aC, bound):
    eP = np.abs(P - rP) / (aP + 1e-300)
    eC = np.abs(C - rC) / (aC + 1e-300)
    assert np.all(np.isfinite(P)) and np.all(np.isfinite(C))
    assert eP.max() <= bound, (eP.max(), np.unravel_index(eP.argmax(), eP.shape))
    assert eC.max() <= bound, (eC.max(), np.unravel_index(eC.argmax(), eC.shape))
    return max(eP.max(), eC.max())


@pytest.mark.parametrize("N,d", [(1, 3), (2, 1), (255, 2), (256, 3), (257, 4), (511, 3),
                                 (767, 1), (1000, 2), (3 * 256 + 5, 3), (5000, 4)])
def test_blocked_history_small_every_target(F, orc, N, d):
    """Ragged lengths around the block edges (255/256/257, 511, 767) and every
    dimension the per-trajectory kernels hold (1..4)."""
    from paper_1611_08678_amd import workloads as W
    f = 30.0 * W.random_history(N, d, seed=N + d)
    rP, rC, aP, aC = orc.history_sums(0.95, f)
    P, C = _gpu_sums(F, 0.95, f)
    _check(P, C, rP, rC, aP, aC, FP64_BOUND)


@pytest.mark.parametrize("alpha", [0.3, 0.8, 1.0, 1.6])
def test_blocked_history_orders(F, orc, alpha):
    """Orders below, at and above one (the weights of 1 < alpha <= 2 grow with
    the lag) over 12 blocks."""
    from paper_1611_08678_amd import workloads as W
    f = W.random_history(3000, 3, seed=11)
    rP, rC, aP, aC = orc.history_sums(alpha, f)
    P, C = _gpu_sums(F, alpha, f)
    _check(P, C, rP, rC, aP, aC, FP64_BOUND)


def test_blocked_history_2p17_every_target(F, orc):
    """Every target of N = 2^17 (512 blocks, far windows of every distance)
    at the headline order alpha = 0.95, against the oracle's long-double sums;
    the DIRECT contraction of the same history agrees as well."""
    from paper_1611_08678_amd import workloads as W
    N = 1 << 17
    f = 30.0 * W.random_history(N, 3, seed=17)
    rP, rC, aP, aC = orc.history_sums(0.95, f)
    P, C = _gpu_sums(F, 0.95, f)
    e = _check(P, C, rP, rC, aP, aC, FP64_BOUND)
    print(f"blocked teacher-forced N=2^17: max err {e:.2e} x sum|w||f|")
    Pd, Cd = _gpu_sums(F, 0.95, f, path="direct")
    _check(Pd, Cd, rP, rC, aP, aC, FP64_BOUND)


def test_blocked_history_2p20_sampled_windows(F, orc):
    """N = 2^20 (4097 blocks, the headline length): every target of three
    512-row windows (the top of the history, across the block edge at 2^19,
    and one mid-block window) against the oracle's sums for those targets."""
    from paper_1611_08678_amd import workloads as W
    N = 1 << 20
    f = 30.0 * W.random_history(N, 3, seed=20)
    P, C = _gpu_sums(F, 0.95, f)
    rows = np.concatenate([np.arange(N - 511, N + 1), np.arange((1 << 19) - 256, (1 << 19) + 256),
                           np.arange(700_000 + 37, 700_000 + 37 + 512)]).astype(np.int64)
    rP, rC, aP, aC = orc.history_sums_rows(0.95, f, rows)
    e = _check(P[rows - 1], C[rows - 1], rP, rC, aP, aC, FP64_BOUND)
    print(f"blocked teacher-forced N=2^20 sampled rows: max err {e:.2e} x sum|w||f|")


def test_blocked_history_fp32_windows(F, orc):
    """Binary32 far windows: within (2 + 64) u of the magnitudes; the near
    part and the band stay binary64, so the first 3 blocks are at the binary64
    bound."""
    from paper_1611_08678_amd import workloads as W
    N = 20000
    f = 30.0 * W.random_history(N, 3, seed=32)
    rP, rC, aP, aC = orc.history_sums(0.9, f)
    P, C = _gpu_sums(F, 0.9, f, far_prec="fp32")
    e = _check(P, C, rP, rC, aP, aC, FP32_BOUND)
    print(f"blocked teacher-forced FP32 windows: max err {e:.2e} x sum|w||f| "
          f"(bound {FP32_BOUND:.2e})")
    # targets whose far part is empty (first 3 blocks: band and near windows only)
    _check(P[:767], C[:767], rP[:767], rC[:767], aP[:767], aC[:767], FP64_BOUND)


def test_blocked_history_constant_closed_form(F):
    """With f = 1 the sums are the weights' partial sums, known in closed form
    (the rule integrates constants exactly): P_t = t^a / Gamma(a+1) and
    C_t + 1/Gamma(a+2) = t^a / Gamma(a+1). No oracle involved."""
    from math import gamma
    N, a = 4000, 0.95
    f = np.ones((N, 2))
    P, C = _gpu_sums(F, a, f)
    t = np.arange(1, N + 1, dtype=np.float64)[:, None]
    ex = t ** a / gamma(a + 1)
    assert np.abs(P - ex).max() / ex.max() <= 1e-13
    assert np.abs(C + 1.0 / gamma(a + 2) - ex).max() / ex.max() <= 1e-13


def test_blocked_history_rejects(F):
    import torch
    f = torch.zeros((10, 5), dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FabmError):
        F.fabm_history_sums(0.9, 10, 5, f, f, f, "blocked", "fp64", ws)
    g = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FabmError):
        F.fabm_history_sums(0.9, 10, 3, g, g, g, "blocked", "fp16x2", ws)
