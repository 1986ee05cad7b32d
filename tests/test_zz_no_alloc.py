"""fabm_solve_noalloc: the single-trajectory solve with the library's own
device scratch array as its workspace (for callers that cannot allocate).

Through the C ABI, against fabm_solve with a caller workspace on the same
inputs: the rows are bitwise equal (the same kernels in the same order), on
two calls in a row, the second smaller than the first (the scratch array keeps
the last call's contents, and every call must re-initialise what it reads).
One case is also checked against the oracle (1e-11 normwise)."""
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


def _rows(F, plan, alpha, h, N, y0, th, noalloc):
    import torch
    d = plan.dim
    y = torch.full((N + 1, d), np.nan, dtype=torch.float64, device="cuda")
    st = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    y0t = torch.as_tensor(np.asarray(y0, np.float64), device="cuda").contiguous()
    tht = torch.as_tensor(np.asarray(th, np.float64), device="cuda").contiguous()
    if noalloc:
        F.fabm_solve_noalloc(plan, alpha, h, N, y0t, tht, y, st)
    else:
        ws = torch.empty(F.fabm_workspace_size(plan, [N]), dtype=torch.uint8, device="cuda")
        F.fabm_solve(plan, ws, alpha, h, N, y0t, tht, y, st)
    torch.cuda.synchronize()
    return y.cpu().numpy(), int(st.item())


@pytest.mark.parametrize("system,d,path,prec,th,y0,alpha,h,Ns", [
    ("chen", 3, "blocked", "fp64", [35.0, 3.0, 28.0], [-9.0, -5.0, 14.0], 0.95, 0.001,
     (60000, 3000)),
    ("vdp", 2, "blocked", "fp32", [1.3], [0.4, -0.7], 0.9, 0.01, (9000, 700)),
    ("vdp", 2, "direct", "fp64", [1.3], [0.4, -0.7], 0.9, 0.01, (9000, 600)),
    ("financial", 3, "direct", "fp64", [3.0, 0.1, 1.0], [0.5, -0.3, 0.2], 0.85, 0.01,
     (700, 300)),
])
def test_noalloc_matches_solve_twice(F, system, d, path, prec, th, y0, alpha, h, Ns):
    plan = F.fabm_plan(system, d, path, prec, 1, max(Ns))
    for N in Ns:  # the second call is smaller than the first
        a, sa = _rows(F, plan, alpha, h, N, y0, th, noalloc=True)
        b, sb = _rows(F, plan, alpha, h, N, y0, th, noalloc=False)
        assert sa == sb == 0, (N, sa, sb)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), (N, np.abs(a - b).max())


def test_noalloc_initial_slope_and_oracle(F, orc):
    """Order 1.5 with y'(0) (the initial values are split into the scratch
    array too), twice, then the scalar linear equation against the oracle."""
    plan = F.fabm_plan("vdp", 2, "blocked", "fp64", 1, 5000, initial_slope=True)
    init = [[0.4, -0.7], [0.2, 0.1]]
    for N in (5000, 1200):
        a, sa = _rows(F, plan, 1.5, 0.01, N, init, [1.1], noalloc=True)
        b, sb = _rows(F, plan, 1.5, 0.01, N, init, [1.1], noalloc=False)
        assert sa == sb == 0 and np.array_equal(a, b)
    lin = F.fabm_plan("linear", 1, "blocked", "fp64", 1, 2000)
    y, st = _rows(F, lin, 0.5, 0.005, 2000, [1.0], [-1.0, 0.0, 0.0], noalloc=True)
    ref, _, _, rst = orc.solve(0, [-1.0, 0.0, 0.0], 0.5, 0.005, 2000, [1.0])
    assert st == rst == 0
    assert np.abs(y - ref).max() / np.abs(ref).max() <= 1e-11


def test_noalloc_rejects_beyond_scratch(F):
    """A workspace above the scratch size is refused before anything is
    enqueued, with both sizes in the error text; the plan still works."""
    import torch
    N = 1_000_000  # about 96 MB of workspace for d = 3
    plan = F.fabm_plan("chen", 3, "blocked", "fp64", 1, N)
    assert F.fabm_workspace_size(plan, [N]) > F.FABM_NOALLOC_SCRATCH_BYTES
    y = torch.empty((N + 1, 3), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int64, device="cuda")
    y0 = torch.tensor([-9.0, -5.0, 14.0], dtype=torch.float64, device="cuda")
    th = torch.tensor([35.0, 3.0, 28.0], dtype=torch.float64, device="cuda")
    with pytest.raises(F.FabmError) as e:
        F.fabm_solve_noalloc(plan, 0.95, 0.001, N, y0, th, y, st)
    assert e.value.code == 3 and "scratch" in str(e.value)
    a, sa = _rows(F, plan, 0.95, 0.001, 2000, [-9.0, -5.0, 14.0], [35.0, 3.0, 28.0], True)
    b, sb = _rows(F, plan, 0.95, 0.001, 2000, [-9.0, -5.0, 14.0], [35.0, 3.0, 28.0], False)
    assert sa == sb == 0 and np.array_equal(a, b)
