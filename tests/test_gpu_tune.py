"""fabm_tune: the autotuner times every candidate launch shape of the plan's
path on the caller's inputs and keeps the fastest. Checked: the report
(knob, candidates, positive times, a valid choice), that the tuned plan's
results are right (single trajectory: the far workgroup count does not change
any sum's order, so bitwise equal to the untuned solve; batches: the group
of source blocks per far launch does not either; shared grid: the split
changes the summation order only, so within the FP64 bound of the oracle),
determinism of the tuned plan, and paths with nothing to choose."""
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


def _buffers(F, plan, Ns, y0s, th):
    import torch
    Ns = np.asarray(Ns, dtype=np.int64)
    ws = F._workspace(F.fabm_workspace_size(plan, Ns))
    row_off = np.concatenate([[0], np.cumsum(Ns + 1)[:-1]]).astype(np.int64)
    y = torch.empty((int((Ns + 1).sum()), y0s.shape[1]), dtype=torch.float64, device="cuda")
    st = torch.zeros(len(Ns), dtype=torch.int64, device="cuda")
    return ws, row_off, torch.tensor(y0s, device="cuda"), torch.tensor(th, device="cuda"), y, st


def test_tune_single_trajectory_blocked(F):
    N, th, y0 = 20000, np.array([[35.0, 3.0, 28.0]]), np.array([[-9.0, -5.0, 14.0]])
    plan = F.fabm_plan("chen", 3, "blocked", "fp64", 1, N)
    ws, ro, y0d, thd, y, st = _buffers(F, plan, [N], y0, th)
    rep = F.fabm_tune(plan, ws, [0.95], [0.001], [N], y0d, thd, ro, y, st)
    assert rep["knob"] == "far_workgroups" and rep["candidates"] == [32, 64, 128, 254]
    assert all(t > 0 for t in rep["seconds"]) and 0 <= rep["chosen"] < 4
    y1, s1 = F.solve("chen", th[0], 0.95, 0.001, N, y0[0], path="blocked", plan=plan)
    y2, s2 = F.solve("chen", th[0], 0.95, 0.001, N, y0[0], path="blocked")
    assert int(s1.item()) == 0 and F._lib is not None
    assert np.array_equal(_to_np(y1), _to_np(y2))


def test_tune_shared_grid(F, orc):
    rng = np.random.default_rng(31)
    B, d, N = 8, 16, 1500
    A = -(2 * np.eye(d)[None] + rng.standard_normal((B, d, d)) / 8)
    th = np.concatenate([A.reshape(B, -1), 0.1 * rng.standard_normal((B, 2 * d))], axis=1)
    y0 = rng.standard_normal((B, d))
    al, hs, Ns = np.full(B, 0.8), np.full(B, 0.01), np.full(B, N)
    plan = F.fabm_plan("linear", d, "blocked", "fp64", B, N, B * N)
    ws, ro, y0d, thd, y, st = _buffers(F, plan, Ns, y0, th)
    rep = F.fabm_tune(plan, ws, al, hs, Ns, y0d, thd, ro, y, st)
    assert rep["knob"] == "split_target" and rep["candidates"] == [256, 512, 1024, 2048, 4096]
    assert all(t > 0 for t in rep["seconds"]) and 0 <= rep["chosen"] < 5
    y1, off, s1 = F.solve_batch("linear", th, al, hs, Ns, y0, plan=plan)
    y2, _, _ = F.solve_batch("linear", th, al, hs, Ns, y0, plan=plan)
    assert np.array_equal(_to_np(y1), _to_np(y2))
    ref, _, rst = orc.solve_batch(0, th, al, hs, Ns, y0)
    assert np.all(_to_np(s1) == 0) and np.all(rst == 0)
    assert relerr(_to_np(y1), ref) <= 1e-11


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tune_batched_blocked_source_group(F, orc, prec):
    """The ragged batched BLOCKED path (Rossler, per-instance alpha, lengths
    around the block edges up to 40 blocks): the tuner times groups of 1, 2
    and 4 source blocks per far launch. Every group size adds the same windows
    to every target in the same order, so the rows left by the last candidate
    (4) and the rows of the tuned plan are bitwise those of an untuned plan
    (2), which match the oracle."""
    from paper_1611_08678_amd import workloads as W
    w = W.rossler_batch(batch=48, n_lo=1, n_hi=10000, seed=19)
    w["N"][:6] = [1, 255, 256, 511, 767, 1024]
    Ns, B = w["N"], 48
    plan = F.fabm_plan("rossler", 3, "blocked", prec, B, int(Ns.max()), int(Ns.sum()))
    ws, ro, y0d, thd, y, st = _buffers(F, plan, Ns, w["y0"], w["theta"])
    rep = F.fabm_tune(plan, ws, w["alpha"], w["h"], Ns, y0d, thd, ro, y, st)
    assert rep["knob"] == "source_group" and rep["candidates"] == [1, 2, 4]
    assert all(t > 0 for t in rep["seconds"]) and 0 <= rep["chosen"] < 3
    y4 = _to_np(y).copy()
    y1, _, s1 = F.solve_batch("rossler", w["theta"], w["alpha"], w["h"], Ns, w["y0"], plan=plan)
    y2, _, s2 = F.solve_batch("rossler", w["theta"], w["alpha"], w["h"], Ns, w["y0"],
                              path="blocked", far_prec=prec)
    a, b = _to_np(y1), _to_np(y2)
    assert np.array_equal(_to_np(s1), _to_np(s2))
    same = lambda u, v: np.array_equal(np.isnan(u), np.isnan(v)) and np.array_equal(
        u[~np.isnan(u)], v[~np.isnan(v)])
    assert same(a, b) and same(y4, b)
    ref, roff, rst = orc.solve_batch(2, w["theta"], w["alpha"], w["h"], Ns, w["y0"])
    ok = rst == 0
    assert np.all(_to_np(s2)[ok] == 0)
    for i in np.nonzero(ok)[0][:12]:
        sl = slice(roff[i], roff[i] + Ns[i] + 1)
        assert relerr(b[sl], ref[sl]) <= (1e-5 if prec == "fp32" else 1e-11), i


def test_tune_nothing_to_choose(F):
    rng = np.random.default_rng(2)
    B = 3
    th, y0 = rng.uniform(0.5, 2, (B, 1)), rng.uniform(-2, 2, (B, 2))
    plan = F.fabm_plan("vdp", 2, "direct", "fp64", B, 700, 3 * 700)
    ws, ro, y0d, thd, y, st = _buffers(F, plan, [700, 300, 500], y0, th)
    rep = F.fabm_tune(plan, ws, np.full(B, 0.9), np.full(B, 0.01), [700, 300, 500], y0d, thd,
                      ro, y, st)
    assert rep == {"knob": "none", "candidates": [], "seconds": [], "chosen": None}


def test_tune_single_trajectory_per_component_orders(F, orc):
    """A single trajectory with one order per component (a batch of one on the
    BLOCKED step kernels): the tuned plan's result is bitwise the untuned
    one's and matches the oracle's per-component solver."""
    N = 6000
    th = np.array([[1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6, 3.25]])
    y0 = np.array([[-1.6, -10.0, 2.0]])
    al = np.array([[0.95, 0.9, 1.0]])
    plan = F.fabm_plan("hindmarsh_rose", 3, "blocked", "fp64", 1, N, per_component_order=True)
    ws, ro, y0d, thd, y, st = _buffers(F, plan, [N], y0, th)
    rep = F.fabm_tune(plan, ws, al, [0.01], [N], y0d, thd, ro, y, st)
    assert rep["knob"] == "far_workgroups" and 0 <= rep["chosen"] < 4
    y1, _, s1 = F.solve_batch("hindmarsh_rose", th, al, [0.01], [N], y0, plan=plan)
    y2, _, _ = F.solve_batch("hindmarsh_rose", th, al, [0.01], [N], y0, path="blocked")
    assert int(_to_np(s1)[0]) == 0 and np.array_equal(_to_np(y1), _to_np(y2))
    ref, _, _, rst = orc.solve_orders(5, th[0], al[0], 0.01, N, y0[0])
    assert rst == 0 and relerr(_to_np(y1), ref) <= 1e-11
