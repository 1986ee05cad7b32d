"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/fabm.h declares, its enumerations agree with the
oracle's own numbering, and plan-time validation rejects bad descriptions."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "fabm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fabm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def fabm():
    import paper_1611_08678_amd as F
    F.load()
    return F


def test_library_exports_every_declared_symbol(fabm):
    import ctypes
    lib = ctypes.CDLL(fabm.SO)
    declared = _declared_functions()
    assert "fabm_solve" in declared and "fabm_plan" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(fabm.EXPORTS) == declared


def test_enums_match_oracle_numbering(fabm):
    from oracle import oracle as O
    assert (fabm.FABM_SYS_LINEAR, fabm.FABM_SYS_CHEN, fabm.FABM_SYS_ROSSLER, fabm.FABM_SYS_VDP,
            fabm.FABM_SYS_FINANCIAL, fabm.FABM_SYS_HINDMARSH_ROSE) == (
        O.LINEAR, O.CHEN, O.ROSSLER, O.VDP, O.FINANCIAL, O.HINDMARSH_ROSE)
    for sysid, d in [(0, 1), (0, 7), (1, 3), (2, 3), (3, 2), (4, 3), (5, 3)]:
        assert fabm.fabm_n_params(sysid, d) == O.n_params(sysid, d)
    assert fabm.fabm_n_params(fabm.FABM_SYS_CHEN, 2) == -1
    assert fabm.fabm_n_params(fabm.FABM_SYS_LINEAR, 65) == -1


def test_kernel_classes_match_header(fabm):
    src = open(os.path.join(ROOT, "include", "fabm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    found = {m.group(1).lower(): int(m.group(2))
             for m in re.finditer(r"FABM_KERNEL_([A-Z_]+)\s*=\s*(\d+)", src)}
    count = found.pop("count")
    assert count == len(fabm.KERNEL_CLASSES)
    assert {k: i for i, k in enumerate(fabm.KERNEL_CLASSES)} == found


def test_status_strings(fabm):
    assert fabm.status_string(0) == "ok"
    assert fabm.status_string(3) == "workspace too small"


@pytest.mark.parametrize("kw,code", [
    (dict(system="chen", dim=2), 1),
    (dict(system="vdp", dim=2, max_steps=0), 1),
    (dict(system="vdp", dim=2, max_batch=0), 1),
    (dict(system="vdp", dim=2, tile_L=100), 1),
    (dict(system=9, dim=2), 1),
])
def test_plan_rejects_bad_descriptions(fabm, kw, code):
    with pytest.raises(fabm.FabmError) as e:
        fabm.fabm_plan(**kw)
    assert e.value.code == code


def test_plan_is_host_only_and_sizes_workspace(fabm):
    p = fabm.fabm_plan("chen", 3, "direct", "fp64", 1, 1 << 20)
    # weights 3N, history (N+1) d, grid partials and flags
    N = 1 << 20
    assert p.workspace_bytes >= 8 * (3 * N + 3 * (N + 1))
    assert fabm.fabm_workspace_size(p, [N]) == p.workspace_bytes
    with pytest.raises(fabm.FabmError):
        fabm.fabm_workspace_size(p, [N + 1])


def test_plan_far_precisions(fabm):
    fabm.fabm_plan("vdp", 2, "blocked", "fp32", 4, 5000)
    with pytest.raises(fabm.FabmError) as e:
        fabm.fabm_plan("vdp", 2, "blocked", "fp16x2", 1, 5000)
    assert e.value.code == 2


def test_batched_blocked_workspace_covers_calls(fabm):
    p = fabm.fabm_plan("rossler", 3, "blocked", "fp32", 8, 3000, 8 * 3000)
    for Ns in ([3000] * 8, [1, 2, 3000, 255, 256, 1000, 7, 2999], [5] * 8, [3000]):
        assert 0 < fabm.fabm_workspace_size(p, Ns) <= p.workspace_bytes
    # the FP32 copies of the weight tables take space only when asked for
    p64 = fabm.fabm_plan("rossler", 3, "blocked", "fp64", 8, 3000, 8 * 3000)
    assert fabm.fabm_workspace_size(p64, [3000] * 8) < fabm.fabm_workspace_size(p, [3000] * 8)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1611_08678_amd as F
    monkeypatch.setattr(F, "_lib", None)
    monkeypatch.setattr(F, "SO", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        F.load()


def test_plan_shared_grid_rules(fabm):
    fabm.fabm_plan("linear", 64, "blocked", "fp64", 512, 1 << 16)
    fabm.fabm_plan("linear", 64, "auto", "fp16x2", 512, 1 << 16)
    fabm.fabm_plan("linear", 3, "blocked", "fp64", 4, 1000, tile_L=64)
    for kw in (dict(system="chen", dim=3, far_prec="fp16x2"),
               dict(system="linear", dim=64, path="direct"),
               dict(system="chen", dim=3, tile_L=64),
               dict(system="linear", dim=64, tile_L=256),
               dict(system="linear", dim=3, tile_L=128),
               dict(system="linear", dim=64, max_batch=(1 << 24) + 1)):
        with pytest.raises(fabm.FabmError) as e:
            fabm.fabm_plan(**kw)
        assert e.value.code == 2, kw


def test_shared_grid_workspace(fabm):
    N = 1 << 16
    sizes = {}
    for prec in ("fp64", "fp32", "fp16x2"):
        p = fabm.fabm_plan("linear", 64, "blocked", prec, 512, N, 512 * N)
        sizes[prec] = fabm.fabm_workspace_size(p, [N] * 512)
        assert sizes[prec] <= p.workspace_bytes
    # one history copy of ceil((N+1)/64)*64 rows x 32768 columns: binary64,
    # binary32, or two binary16 parts
    cells = 1025 * 64 * 32768
    assert sizes["fp64"] >= 8 * cells and sizes["fp32"] >= 4 * cells
    assert sizes["fp16x2"] >= 4 * cells and sizes["fp32"] < sizes["fp64"]


def test_shared_grid_needs_shared_alpha_h_N(fabm):
    """Checked on the host before any device work (placeholder device
    addresses are never touched)."""
    import ctypes as C
    import numpy as np
    p = fabm.fabm_plan("linear", 8, "blocked", "fp64", 3, 100, 300)
    ws = p.workspace_bytes
    fake = C.c_void_p(1 << 40)  # 256-byte aligned placeholder
    for al, hh, Ns in (([0.8, 0.7, 0.8], [0.01] * 3, [100] * 3),
                       ([0.8] * 3, [0.01, 0.01, 0.02], [100] * 3),
                       ([0.8] * 3, [0.01] * 3, [100, 99, 100])):
        al, hh = np.asarray(al, float), np.asarray(hh, float)
        Ns = np.asarray(Ns, np.int64)
        ro = np.concatenate([[0], np.cumsum(Ns + 1)[:-1]]).astype(np.int64)
        lib = fabm.load()
        code = lib.fabm_solve_batch(p.handle, fake, ws, 3, al.ctypes.data_as(fabm._DP),
                                    hh.ctypes.data_as(fabm._DP), Ns.ctypes.data_as(fabm._I64P),
                                    fake, fake, ro.ctypes.data_as(fabm._I64P), fake, fake, None)
        assert code == 2


def test_initial_slope_flag_rules(fabm):
    """Orders above one need y'(0): plans with FABM_PLAN_INITIAL_SLOPE take
    [batch][2][d] initial values (workspace grows by the split copies); without
    it 1 < alpha <= 2 is UNSUPPORTED; alpha > 2 is INVALID_ARG; unknown plan
    flags are INVALID_ARG. All checked on the host before any device work."""
    import ctypes as C
    import numpy as np
    p = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 4, 1000, 4000)
    q = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 4, 1000, 4000, initial_slope=True)
    assert q.initial_slope and not p.initial_slope
    Ns = [1000, 10, 300, 999]
    extra = fabm.fabm_workspace_size(q, Ns) - fabm.fabm_workspace_size(p, Ns)
    assert 2 * 4 * 2 * 8 <= extra <= 2 * 4 * 2 * 8 + 256
    for path in ("direct", "auto"):
        fabm.fabm_plan("chen", 3, path, "fp64", 1, 100, initial_slope=True)
    fabm.fabm_plan("linear", 8, "blocked", "fp16x2", 2, 100, 200, initial_slope=True)
    lib = fabm.load()
    desc = fabm._PlanDesc(fabm.FABM_SYS_VDP, 2, 0, 0, 1, 100, 0, 0, 8)  # unknown flag bit
    h = C.c_void_p()
    assert lib.fabm_plan(C.byref(desc), C.byref(h), None) == 1
    fake = C.c_void_p(1 << 40)
    Nb = np.asarray([100, 100], np.int64)
    ro = np.asarray([0, 101], np.int64)
    hh = np.asarray([0.01, 0.01])
    for plan, alphas, code in ((p, [0.9, 1.5], 2), (p, [0.9, 2.0], 2), (q, [0.9, 2.5], 1),
                               (p, [0.9, 2.5], 1), (q, [0.0, 1.5], 1)):
        al = np.asarray(alphas, float)
        got = lib.fabm_solve_batch(plan.handle, fake, plan.workspace_bytes, 2,
                                   al.ctypes.data_as(fabm._DP), hh.ctypes.data_as(fabm._DP),
                                   Nb.ctypes.data_as(fabm._I64P), fake, fake,
                                   ro.ctypes.data_as(fabm._I64P), fake, fake, None)
        assert got == code, (alphas, got)


def test_per_component_order_rules(fabm):
    """Non-commensurate plans: DIRECT, per-trajectory BLOCKED (FP64 or FP32
    windows) and the adjoint (the shared grid is UNSUPPORTED, so is fabm_solve
    with its single alpha); alpha is [batch][d], every entry
    checked (an order above one needs the slope flag); one weight table per
    component. Host-side checks only."""
    import ctypes as C
    import numpy as np
    F = fabm
    for kw in (dict(path="blocked"), dict(path="auto", tile_L=256), dict(path="direct")):
        F.fabm_plan("chen", 3, max_batch=2, max_steps=100, per_component_order=True, **kw)
    F.fabm_plan("chen", 3, "blocked", "fp32", 2, 100, per_component_order=True)
    with pytest.raises(F.FabmError) as e:
        F.fabm_plan("linear", 4, "blocked", "fp16x2", 2, 100, per_component_order=True)
    assert e.value.code == 2
    pb = F.fabm_plan("vdp", 2, "blocked", "fp64", 3, 2000, per_component_order=True)
    qb = F.fabm_plan("vdp", 2, "blocked", "fp64", 3, 2000)
    for Ns in ([2000], [2000, 5, 700]):  # single and batched layouts: one table set per component
        assert F.fabm_workspace_size(pb, Ns) > F.fabm_workspace_size(qb, Ns)
    with pytest.raises(F.FabmError) as e:
        F.fabm_plan("linear", 8, "auto", "fp64", 2, 100, per_component_order=True)
    assert e.value.code == 2
    p = F.fabm_plan("chen", 3, "auto", "fp64", 2, 100, per_component_order=True)
    q = F.fabm_plan("chen", 3, "auto", "fp64", 2, 100)
    Ns = [100, 60]
    extra = F.fabm_workspace_size(p, Ns) - F.fabm_workspace_size(q, Ns)
    assert extra >= 8 * 3 * 160 * 2  # two more weight tables per instance
    lib = F.load()
    n = C.c_size_t()
    Nb = np.asarray(Ns, np.int64)
    assert lib.fabm_adjoint_workspace_size(p.handle, 2, Nb.ctypes.data_as(F._I64P),
                                           C.byref(n)) == 0 and n.value > 0
    fake = C.c_void_p(1 << 40)
    assert lib.fabm_solve(p.handle, fake, p.workspace_bytes, C.c_double(0.9), C.c_double(0.01),
                          100, fake, fake, fake, fake, None) == 2
    ro = np.asarray([0, 101], np.int64)
    hh = np.asarray([0.01, 0.01])
    ps = F.fabm_plan("chen", 3, "auto", "fp64", 2, 100, per_component_order=True,
                     initial_slope=True)
    for plan, al, code in ((p, [0.9, 0.8, 0.7, 0.9, 1.5, 0.6], 2),
                           (p, [0.9, 0.8, 0.7, 0.9, 0.0, 0.6], 1),
                           (ps, [0.9, 0.8, 0.7, 0.9, 2.5, 0.6], 1)):
        a = np.asarray(al, float)
        got = lib.fabm_solve_batch(plan.handle, fake, plan.workspace_bytes, 2,
                                   a.ctypes.data_as(F._DP), hh.ctypes.data_as(F._DP),
                                   Nb.ctypes.data_as(F._I64P), fake, fake,
                                   ro.ctypes.data_as(F._I64P), fake, fake, None)
        assert got == code, (al, got)


def test_plan_fft_far_rules(fabm):
    """fft_level (sub-quadratic far history): 0 off, 1..15 valid; only for one
    BLOCKED trajectory (FP64 or FP32 windows, one order or one per component);
    the workspace grows by the twiddles, one square's transforms and the
    weight spectra (one set per component with per-component orders)."""
    for lv in (-1, 16):
        with pytest.raises(fabm.FabmError) as e:
            fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, 50000, fft_level=lv)
        assert e.value.code == 1
    for kw in (dict(path="auto"), dict(path="direct"), dict(far_prec="fp16x2"),
               dict(max_batch=2), dict(system="linear", dim=8),
               dict(max_steps=(1 << 24) + 1)):
        a = dict(system="vdp", dim=2, path="blocked", far_prec="fp64", max_batch=1,
                 max_steps=50000)
        a.update(kw)
        with pytest.raises(fabm.FabmError) as e:
            fabm.fabm_plan(a.pop("system"), a.pop("dim"), fft_level=3, **a)
        assert e.value.code == 2, kw
    N = 50000  # 196 blocks: squares up to level 7, longest transform 2^16 points
    p0 = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, N)
    p3 = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, N, fft_level=3)
    p9 = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, N, fft_level=9)  # above the top
    M = 1 << 16
    grow = fabm.fabm_workspace_size(p3, [N]) - fabm.fabm_workspace_size(p0, [N])
    spectra = sum(512 << lv for lv in range(3, 8))
    assert 16 * (M + 2 * M + spectra) <= grow <= 16 * (M + 2 * M + spectra) + 3 * 4096
    assert fabm.fabm_workspace_size(p9, [N]) == fabm.fabm_workspace_size(p0, [N])
    q0 = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, N, per_component_order=True)
    q3 = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, N, per_component_order=True,
                        fft_level=3)
    grow_pc = fabm.fabm_workspace_size(q3, [N]) - fabm.fabm_workspace_size(q0, [N])
    assert 16 * (M + 2 * M + 2 * spectra) <= grow_pc <= 16 * (M + 2 * M + 2 * spectra) + 3 * 4096
    fabm.fabm_plan("vdp", 2, "blocked", "fp32", 1, N, fft_level=3)  # FP32 windows: accepted


def _far_cover_from_schedule(fabm, NB, level):
    """Column-level cover of the far region by the library's schedule: matrix-core
    window of launch s for target J (target column rho, lags 16 s + rho - u,
    u < 16; columns of block s - 1 dropped when skip_prev) and, after launch s,
    the square of level l = square: sources blocks (s + 2 - 2^l) .. s + 1, targets
    s + 5 .. s + 4 + 2^l (< NB). Returns the first-writer order check too."""
    seen, written, ok_first = {}, set(), True
    for s in range(-1, NB - 1):
        jend, skip_prev, square = fabm.fabm_fft_far_schedule(NB, level, s)
        if 0 <= s and s + 2 <= NB - 1:  # near part of target s + 2
            ok_first &= (s == 0) == (s + 2 not in written)
            written.add(s + 2)
        if s >= 0:
            for J in range(s + 3, jend):
                ok_first &= (s == 0) == (J not in written)
                written.add(J)
                for rho in range(16):
                    for u in range(16):
                        kap = 16 * s + rho - u
                        if kap >= 0 and not (skip_prev and kap < 16 * s):
                            key = (J, rho, kap)
                            seen[key] = seen.get(key, 0) + 1
        if square >= 0:
            n = 1 << square
            assert (s + 2) % n == 0 and ((s + 2) // n) % 2 == 1
            first = s + 2 - n == 0
            for J in range(s + 5, min(NB, s + 5 + n)):
                ok_first &= first == (J not in written)
                written.add(J)
                for rho in range(16):
                    for K in range(s + 2 - n, s + 2):
                        for x in range(16):
                            key = (J, rho, 16 * K + x)
                            seen[key] = seen.get(key, 0) + 1
    return seen, ok_first


@pytest.mark.parametrize("NB", [5, 6, 7, 9, 12, 17, 21, 36, 69])
def test_fft_far_schedule_covers_far_region_once(fabm, NB):
    """The far part of target column rho of block J is every source column up
    to 16 (J - 3) + rho; windows and squares must add each one exactly once,
    after it is formed, and the first addition to a target must be the one
    that overwrites (a window of launch 0, or a square whose sources start at
    block 0)."""
    need = {(J, rho, kap) for J in range(3, NB) for rho in range(16)
            for kap in range(0, 16 * (J - 3) + rho + 1)}
    for level in range(0, 6):
        seen, ok_first = _far_cover_from_schedule(fabm, NB, level)
        assert set(seen) == need and all(v == 1 for v in seen.values()), (NB, level)
        assert ok_first, (NB, level)
    with pytest.raises(fabm.FabmError):
        fabm.fabm_fft_far_schedule(NB, 16, 0)
    with pytest.raises(fabm.FabmError):
        fabm.fabm_fft_far_schedule(NB, 1, NB - 1)


def test_noalloc_host_checks(fabm):
    """fabm_solve_noalloc refuses on the host, before any device call
    (placeholder device addresses are never touched): a workspace above the
    scratch array, the shared grid, the FFT far history, bad arguments."""
    import ctypes as C
    lib = fabm.load()
    fake = C.c_void_p(1 << 40)
    big = fabm.fabm_plan("chen", 3, "blocked", "fp64", 1, 1 << 20)
    assert fabm.fabm_workspace_size(big, [1 << 20]) > fabm.FABM_NOALLOC_SCRATCH_BYTES
    assert lib.fabm_solve_noalloc(big.handle, 0.95, 0.001, 1 << 20, fake, fake, fake, fake,
                                  None) == fabm.FABM_ERR_WORKSPACE
    assert b"scratch" in lib.fabm_last_error()
    assert lib.fabm_solve_noalloc(big.handle, 0.0, 0.001, 100, fake, fake, fake, fake,
                                  None) == fabm.FABM_ERR_INVALID_ARG
    assert lib.fabm_solve_noalloc(big.handle, 0.9, 0.001, (1 << 20) + 1, fake, fake, fake,
                                  fake, None) == fabm.FABM_ERR_INVALID_ARG
    wide = fabm.fabm_plan("linear", 8, "blocked", "fp64", 1, 1000)
    assert lib.fabm_solve_noalloc(wide.handle, 0.8, 0.01, 1000, fake, fake, fake, fake,
                                  None) == fabm.FABM_ERR_UNSUPPORTED
    fft = fabm.fabm_plan("vdp", 2, "blocked", "fp64", 1, 100000, fft_level=2)
    assert lib.fabm_solve_noalloc(fft.handle, 0.9, 0.01, 5000, fake, fake, fake, fake,
                                  None) == fabm.FABM_ERR_UNSUPPORTED
