"""MI355X (gfx950) library for the fractional Adams-Bashforth-Moulton
predictor-corrector (Diethelm's method; Section 2 of arXiv:1611.08678).

This module is a thin ctypes binding of the C ABI in ``include/fabm.h``: the
functions carry the same names and arguments; torch tensors stand in for
device pointers and the current torch stream for the HIP stream. All
arithmetic runs in the HIP kernels of ``libfabm.so``; if that library is not
built, every call raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
from dataclasses import dataclass

_exiting = False  # set when the interpreter starts to exit


@atexit.register
def _mark_exit():
    global _exiting
    _exiting = True

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libfabm.so")

# enums of fabm.h
FABM_OK, FABM_ERR_INVALID_ARG, FABM_ERR_UNSUPPORTED, FABM_ERR_WORKSPACE, FABM_ERR_DEVICE = range(5)
(FABM_SYS_LINEAR, FABM_SYS_CHEN, FABM_SYS_ROSSLER, FABM_SYS_VDP, FABM_SYS_FINANCIAL,
 FABM_SYS_HINDMARSH_ROSE) = range(6)
FABM_PATH_AUTO, FABM_PATH_DIRECT, FABM_PATH_BLOCKED = range(3)
FABM_FAR_FP64, FABM_FAR_FP32, FABM_FAR_FP16X2 = range(3)

SYSTEMS = {"linear": FABM_SYS_LINEAR, "chen": FABM_SYS_CHEN, "rossler": FABM_SYS_ROSSLER,
           "vdp": FABM_SYS_VDP, "financial": FABM_SYS_FINANCIAL,
           "hindmarsh_rose": FABM_SYS_HINDMARSH_ROSE}
PATHS = {"auto": FABM_PATH_AUTO, "direct": FABM_PATH_DIRECT, "blocked": FABM_PATH_BLOCKED}
FAR_PRECS = {"fp64": FABM_FAR_FP64, "fp32": FABM_FAR_FP32, "fp16x2": FABM_FAR_FP16X2}

# exported symbols of the C ABI (checked by the test suite against fabm.h)
EXPORTS = ("fabm_last_error", "fabm_status_string", "fabm_n_params", "fabm_plan", "fabm_plan_destroy",
           "fabm_workspace_size", "fabm_solve", "fabm_solve_batch", "fabm_weights",
           "fabm_history_sums", "fabm_history_workspace_size", "fabm_plan_set_profiling",
           "fabm_plan_kernel_times", "fabm_adjoint", "fabm_adjoint_workspace_size",
           "fabm_graph_solve_batch", "fabm_graph_launch", "fabm_graph_destroy", "fabm_tune",
           "fabm_adjoint_forward", "fabm_adjoint_reverse", "fabm_fft_far_schedule",
           "fabm_solve_noalloc")
KERNEL_CLASSES = ("weights", "direct_wg", "direct_grid", "blocked_step", "history", "adjoint",
                  "wide_far", "wide_band", "fft_far")


class FabmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = ""
        # the library's text for device failures, and for a no-allocation
        # solve refused for size (set by that call)
        if code == FABM_ERR_DEVICE or (code == FABM_ERR_WORKSPACE and
                                       where == "fabm_solve_noalloc"):
            try:
                detail = " [" + load().fabm_last_error().decode() + "]"
            except Exception:
                pass
        super().__init__(f"{where}: {status_string(code)} ({code}){detail}")


class _PlanDesc(C.Structure):
    _fields_ = [("system", C.c_int), ("dim", C.c_int32), ("path", C.c_int),
                ("far_prec", C.c_int), ("max_batch", C.c_int64), ("max_steps", C.c_int64),
                ("max_total_steps", C.c_int64), ("tile_L", C.c_int32), ("flags", C.c_int32),
                ("fft_level", C.c_int32)]


_lib = None
_VP = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)


def load():
    """Load libfabm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise ImportError(f"HIP library not built: {SO} is missing "
                          "(run __graft_entry__.build() or python -m paper_1611_08678_amd.build)")
    # torch brings its own HIP runtime (same soname as the system one). Load it
    # first so libfabm binds to the runtime torch uses: two HIP/HSA runtimes in
    # one process cannot both open the device.
    import torch  # noqa: F401
    L = C.CDLL(SO)
    L.fabm_last_error.argtypes = []
    L.fabm_last_error.restype = C.c_char_p
    L.fabm_status_string.argtypes = [C.c_int]
    L.fabm_status_string.restype = C.c_char_p
    L.fabm_n_params.argtypes = [C.c_int, C.c_int32]
    L.fabm_n_params.restype = C.c_int32
    L.fabm_plan.argtypes = [C.POINTER(_PlanDesc), C.POINTER(_VP), C.POINTER(C.c_size_t)]
    L.fabm_plan.restype = C.c_int
    L.fabm_plan_destroy.argtypes = [_VP]
    L.fabm_plan_destroy.restype = None
    L.fabm_workspace_size.argtypes = [_VP, C.c_int64, _I64P, C.POINTER(C.c_size_t)]
    L.fabm_workspace_size.restype = C.c_int
    L.fabm_solve.argtypes = [_VP, _VP, C.c_size_t, C.c_double, C.c_double, C.c_int64, _VP, _VP,
                             _VP, _VP, _VP]
    L.fabm_solve.restype = C.c_int
    L.fabm_solve_noalloc.argtypes = [_VP, C.c_double, C.c_double, C.c_int64, _VP, _VP, _VP, _VP,
                                     _VP]
    L.fabm_solve_noalloc.restype = C.c_int
    L.fabm_solve_batch.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _DP, _DP, _I64P, _VP, _VP,
                                   _I64P, _VP, _VP, _VP]
    L.fabm_solve_batch.restype = C.c_int
    L.fabm_weights.argtypes = [C.c_double, C.c_int64, _VP, _VP, _VP, _VP]
    L.fabm_weights.restype = C.c_int
    _IP = C.POINTER(C.c_int32)
    L.fabm_fft_far_schedule.argtypes = [C.c_int32, C.c_int32, C.c_int32, _IP, _IP, _IP]
    L.fabm_fft_far_schedule.restype = C.c_int
    L.fabm_history_sums.argtypes = [C.c_double, C.c_int64, C.c_int32, _VP, _VP, _VP, C.c_int,
                                    C.c_int, _VP, C.c_size_t, _VP]
    L.fabm_history_sums.restype = C.c_int
    L.fabm_history_workspace_size.argtypes = [C.c_int64, C.c_int32]
    L.fabm_history_workspace_size.restype = C.c_size_t
    L.fabm_plan_set_profiling.argtypes = [_VP, C.c_int32]
    L.fabm_plan_set_profiling.restype = C.c_int
    L.fabm_plan_kernel_times.argtypes = [_VP, _DP, _I64P]
    L.fabm_plan_kernel_times.restype = C.c_int
    L.fabm_adjoint.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _DP, _DP, _I64P, _VP, _VP, _I64P,
                               _VP, _VP, _VP, _VP, _VP]
    L.fabm_adjoint.restype = C.c_int
    L.fabm_adjoint_forward.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _DP, _DP, _I64P, _VP,
                                       _VP, _I64P, _VP, _VP, _VP]
    L.fabm_adjoint_forward.restype = C.c_int
    L.fabm_adjoint_reverse.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _DP, _DP, _I64P, _VP,
                                       _VP, _I64P, _VP, _VP, _VP, _VP]
    L.fabm_adjoint_reverse.restype = C.c_int
    L.fabm_adjoint_workspace_size.argtypes = [_VP, C.c_int64, _I64P, C.POINTER(C.c_size_t)]
    L.fabm_adjoint_workspace_size.restype = C.c_int
    L.fabm_graph_solve_batch.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _DP, _DP, _I64P, _VP,
                                         _VP, _I64P, _VP, _VP, C.POINTER(_VP)]
    L.fabm_graph_solve_batch.restype = C.c_int
    L.fabm_graph_launch.argtypes = [_VP, _VP]
    L.fabm_graph_launch.restype = C.c_int
    L.fabm_graph_destroy.argtypes = [_VP]
    L.fabm_graph_destroy.restype = None
    L.fabm_tune.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _DP, _DP, _I64P, _VP, _VP, _I64P,
                            _VP, _VP, _VP, C.POINTER(_TuneReport)]
    L.fabm_tune.restype = C.c_int
    _lib = L
    return L


def status_string(code: int) -> str:
    try:
        return load().fabm_status_string(int(code)).decode()
    except ImportError:
        return "?"


def _check(code: int, where: str):
    if code != FABM_OK:
        raise FabmError(code, where)


def _ptr(t):
    """Device pointer of a torch tensor (None for None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _enum(v, table):
    return table[v] if isinstance(v, str) else int(v)


def fabm_n_params(system, dim: int) -> int:
    return int(load().fabm_n_params(_enum(system, SYSTEMS), int(dim)))


@dataclass
class Plan:
    handle: C.c_void_p
    workspace_bytes: int
    system: int
    dim: int
    n_params: int
    path: int
    initial_slope: bool = False  # calls pass y0 as [batch][2][d] (y(0), y'(0))
    per_component_order: bool = False  # calls pass alpha as [batch][d]

    def __del__(self):
        # at interpreter exit the process is ending: leave the pinned staging
        # buffer and event to the OS rather than call into a HIP runtime that
        # may already be tearing down
        if self.handle and _lib is not None and not _exiting:
            _lib.fabm_plan_destroy(self.handle)
            self.handle = None


# device scratch array of fabm_solve_noalloc (bytes, per device; fabm.h)
FABM_NOALLOC_SCRATCH_BYTES = 64 << 20
FABM_PLAN_INITIAL_SLOPE = 1
FABM_PLAN_PER_COMPONENT_ORDER = 2
FABM_PLAN_ADJOINT_CHECKPOINT = 4


def fabm_plan(system, dim: int, path="auto", far_prec="fp64", max_batch: int = 1,
              max_steps: int = 1, max_total_steps: int = 0, tile_L: int = 0,
              initial_slope: bool = False, per_component_order: bool = False,
              fft_level: int = 0, adjoint_checkpoint: bool = False) -> Plan:
    """fft_level > 0: the far history of one BLOCKED trajectory by FFT convolution
    of dyadic block squares of level >= fft_level (sub-quadratic variant).
    adjoint_checkpoint: the adjoint calls keep block checkpoints and re-form the
    rows in the reverse pass instead of storing every row."""
    L = load()
    desc = _PlanDesc(_enum(system, SYSTEMS), int(dim), _enum(path, PATHS),
                     _enum(far_prec, FAR_PRECS), int(max_batch), int(max_steps),
                     int(max_total_steps), int(tile_L),
                     (FABM_PLAN_INITIAL_SLOPE if initial_slope else 0) |
                     (FABM_PLAN_PER_COMPONENT_ORDER if per_component_order else 0) |
                     (FABM_PLAN_ADJOINT_CHECKPOINT if adjoint_checkpoint else 0),
                     int(fft_level))
    h = C.c_void_p()
    ws = C.c_size_t()
    _check(L.fabm_plan(C.byref(desc), C.byref(h), C.byref(ws)), "fabm_plan")
    return Plan(h, int(ws.value), desc.system, desc.dim, fabm_n_params(desc.system, desc.dim),
                desc.path, bool(initial_slope), bool(per_component_order))


def fabm_workspace_size(plan: Plan, N) -> int:
    import numpy as np
    Ns = np.ascontiguousarray(np.atleast_1d(N), dtype=np.int64)
    out = C.c_size_t()
    _check(load().fabm_workspace_size(plan.handle, Ns.size, Ns.ctypes.data_as(_I64P),
                                      C.byref(out)), "fabm_workspace_size")
    return int(out.value)


def fabm_solve(plan: Plan, workspace, alpha: float, h: float, N: int, y0, params, y_out,
               status, stream=None):
    _check(load().fabm_solve(plan.handle, _ptr(workspace), workspace.numel() * workspace.element_size(),
                             float(alpha), float(h), int(N), _ptr(y0), _ptr(params), _ptr(y_out),
                             _ptr(status), _stream(stream)), "fabm_solve")


def fabm_solve_noalloc(plan: Plan, alpha: float, h: float, N: int, y0, params, y_out, status,
                       stream=None):
    """fabm_solve with the library's own device scratch array as the workspace
    (nothing is allocated by the call)."""
    _check(load().fabm_solve_noalloc(plan.handle, float(alpha), float(h), int(N), _ptr(y0),
                                     _ptr(params), _ptr(y_out), _ptr(status), _stream(stream)),
           "fabm_solve_noalloc")


def fabm_solve_batch(plan: Plan, workspace, alpha, h, N, y0, params, row_off, y_out, status,
                     stream=None):
    import numpy as np
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    hh = np.ascontiguousarray(h, dtype=np.float64)
    Ns = np.ascontiguousarray(N, dtype=np.int64)
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    _check(load().fabm_solve_batch(plan.handle, _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), Ns.size,
                                   al.ctypes.data_as(_DP), hh.ctypes.data_as(_DP),
                                   Ns.ctypes.data_as(_I64P), _ptr(y0), _ptr(params),
                                   ro.ctypes.data_as(_I64P), _ptr(y_out), _ptr(status),
                                   _stream(stream)), "fabm_solve_batch")


class _TuneReport(C.Structure):
    _fields_ = [("knob", C.c_int32), ("n", C.c_int32), ("value", C.c_int32 * 8),
                ("seconds", C.c_double * 8), ("chosen", C.c_int32)]


TUNE_KNOBS = ("none", "far_workgroups", "split_target", "source_group")


def fabm_tune(plan: Plan, workspace, alpha, h, N, y0, params, row_off, y_out, status,
              stream=None) -> dict:
    """Autotune the plan's launch shape on these inputs (see fabm.h); returns
    {"knob", "candidates", "seconds", "chosen"}, "chosen" being the index of
    the candidate the plan now uses (None when there was nothing to choose)."""
    import numpy as np
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    hh = np.ascontiguousarray(h, dtype=np.float64)
    Ns = np.ascontiguousarray(N, dtype=np.int64)
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    rep = _TuneReport()
    _check(load().fabm_tune(plan.handle, _ptr(workspace), workspace.numel() * workspace.element_size(),
                            Ns.size, al.ctypes.data_as(_DP), hh.ctypes.data_as(_DP),
                            Ns.ctypes.data_as(_I64P), _ptr(y0), _ptr(params),
                            ro.ctypes.data_as(_I64P), _ptr(y_out), _ptr(status), _stream(stream),
                            C.byref(rep)), "fabm_tune")
    n = rep.n
    return {"knob": TUNE_KNOBS[rep.knob], "candidates": list(rep.value[:n]),
            "seconds": list(rep.seconds[:n]), "chosen": rep.chosen if n else None}


class Graph:
    """A captured solve (fabm_graph_solve_batch); `launch(stream)` runs it."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep  # the device buffers the graph reads and writes

    def launch(self, stream=None):
        _check(load().fabm_graph_launch(self.handle, _stream(stream)), "fabm_graph_launch")

    def __del__(self):
        if self.handle and _lib is not None and not _exiting:
            _lib.fabm_graph_destroy(self.handle)
            self.handle = None


def fabm_graph_solve_batch(plan: Plan, workspace, alpha, h, N, y0, params, row_off, y_out,
                           status) -> Graph:
    import numpy as np
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    hh = np.ascontiguousarray(h, dtype=np.float64)
    Ns = np.ascontiguousarray(N, dtype=np.int64)
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    g = C.c_void_p()
    _check(load().fabm_graph_solve_batch(plan.handle, _ptr(workspace),
                                         workspace.numel() * workspace.element_size(), Ns.size,
                                         al.ctypes.data_as(_DP), hh.ctypes.data_as(_DP),
                                         Ns.ctypes.data_as(_I64P), _ptr(y0), _ptr(params),
                                         ro.ctypes.data_as(_I64P), _ptr(y_out), _ptr(status),
                                         C.byref(g)), "fabm_graph_solve_batch")
    return Graph(g, (plan, workspace, y0, params, y_out, status))


def fabm_adjoint_workspace_size(plan: Plan, N) -> int:
    import numpy as np
    Ns = np.ascontiguousarray(np.atleast_1d(N), dtype=np.int64)
    out = C.c_size_t()
    _check(load().fabm_adjoint_workspace_size(plan.handle, Ns.size, Ns.ctypes.data_as(_I64P),
                                              C.byref(out)), "fabm_adjoint_workspace_size")
    return int(out.value)


def fabm_adjoint(plan: Plan, workspace, alpha, h, N, y0, params, row_off, gy, gy0, gparams,
                 status, stream=None):
    import numpy as np
    al = np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64)
    hh = np.ascontiguousarray(np.atleast_1d(h), dtype=np.float64)
    Ns = np.ascontiguousarray(np.atleast_1d(N), dtype=np.int64)
    ro = np.ascontiguousarray(np.atleast_1d(row_off), dtype=np.int64)
    _check(load().fabm_adjoint(plan.handle, _ptr(workspace),
                               workspace.numel() * workspace.element_size(), Ns.size,
                               al.ctypes.data_as(_DP), hh.ctypes.data_as(_DP),
                               Ns.ctypes.data_as(_I64P), _ptr(y0), _ptr(params),
                               ro.ctypes.data_as(_I64P), _ptr(gy), _ptr(gy0), _ptr(gparams),
                               _ptr(status), _stream(stream)), "fabm_adjoint")


def _host_arrays(alpha, h, N, row_off):
    import numpy as np
    return (np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64),
            np.ascontiguousarray(np.atleast_1d(h), dtype=np.float64),
            np.ascontiguousarray(np.atleast_1d(N), dtype=np.int64),
            np.ascontiguousarray(np.atleast_1d(row_off), dtype=np.int64))


def fabm_adjoint_forward(plan: Plan, workspace, alpha, h, N, y0, params, row_off, y_out, status,
                         stream=None):
    al, hh, Ns, ro = _host_arrays(alpha, h, N, row_off)
    _check(load().fabm_adjoint_forward(plan.handle, _ptr(workspace),
                                       workspace.numel() * workspace.element_size(), Ns.size,
                                       al.ctypes.data_as(_DP), hh.ctypes.data_as(_DP),
                                       Ns.ctypes.data_as(_I64P), _ptr(y0), _ptr(params),
                                       ro.ctypes.data_as(_I64P), _ptr(y_out), _ptr(status),
                                       _stream(stream)), "fabm_adjoint_forward")


def fabm_adjoint_reverse(plan: Plan, workspace, alpha, h, N, y0, params, row_off, gy, gy0,
                         gparams, stream=None):
    al, hh, Ns, ro = _host_arrays(alpha, h, N, row_off)
    _check(load().fabm_adjoint_reverse(plan.handle, _ptr(workspace),
                                       workspace.numel() * workspace.element_size(), Ns.size,
                                       al.ctypes.data_as(_DP), hh.ctypes.data_as(_DP),
                                       Ns.ctypes.data_as(_I64P), _ptr(y0), _ptr(params),
                                       ro.ctypes.data_as(_I64P), _ptr(gy), _ptr(gy0),
                                       _ptr(gparams), _stream(stream)), "fabm_adjoint_reverse")


def fabm_plan_set_profiling(plan: Plan, enable: bool):
    _check(load().fabm_plan_set_profiling(plan.handle, int(bool(enable))),
           "fabm_plan_set_profiling")


def fabm_plan_kernel_times(plan: Plan):
    """{kernel class: (seconds, launches)} of the last profiled call."""
    n = len(KERNEL_CLASSES)
    sec = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(load().fabm_plan_kernel_times(plan.handle, sec, cnt), "fabm_plan_kernel_times")
    return {k: (float(sec[i]), int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}


def fabm_fft_far_schedule(NB: int, level: int, s: int):
    """(jend, skip_prev, square) of step launch s (host only)."""
    j, k, q = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().fabm_fft_far_schedule(int(NB), int(level), int(s), C.byref(j), C.byref(k),
                                        C.byref(q)), "fabm_fft_far_schedule")
    return int(j.value), bool(k.value), int(q.value)


def fabm_weights(alpha: float, n: int, b, a, c, stream=None):
    _check(load().fabm_weights(float(alpha), int(n), _ptr(b), _ptr(a), _ptr(c), _stream(stream)),
           "fabm_weights")


def fabm_history_workspace_size(N: int, dim: int) -> int:
    return int(load().fabm_history_workspace_size(int(N), int(dim)))


def fabm_history_sums(alpha: float, N: int, dim: int, f, P, Cs, path="auto", far_prec="fp64",
                      workspace=None, stream=None):
    _check(load().fabm_history_sums(float(alpha), int(N), int(dim), _ptr(f), _ptr(P), _ptr(Cs),
                                    _enum(path, PATHS), _enum(far_prec, FAR_PRECS),
                                    _ptr(workspace),
                                    0 if workspace is None else workspace.numel() * workspace.element_size(),
                                    _stream(stream)), "fabm_history_sums")


# ---------------------------------------------------------------------------
# Convenience wrappers: allocate outputs and workspace with torch, then call
# the ABI above. No arithmetic happens here.
# ---------------------------------------------------------------------------
def _dev(x):
    """float64 device tensor of x (a tensor, array or nested list)."""
    import numpy as np
    import torch
    if not isinstance(x, torch.Tensor):
        x = np.asarray(x, dtype=np.float64)
    return torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()


def _workspace(nbytes: int):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def _init_rows(y0, lead: int):
    """Initial values with `lead` leading dimensions: [..., d] (y(0)) or
    [..., 2, d] (y(0), y'(0)). Returns (device tensor, d, two_rows)."""
    y0 = _dev(y0)
    two = y0.dim() == lead + 2
    if two and y0.shape[-2] != 2:
        raise ValueError("initial values must be [..., d] or [..., 2, d]")
    return y0, int(y0.shape[-1]), two


def solve(system, theta, alpha: float, h: float, N: int, y0, path="auto", far_prec="fp64",
          plan: Plan | None = None, tile_L: int = 0, fft_level: int = 0):
    """One trajectory; returns (y [N+1, d] float64 device tensor, status int).
    fft_level > 0 (path "blocked"): far history by FFT squares of that level on.
    y0 is y(0) [d], or [2, d] holding y(0) and y'(0) (orders 1 < alpha <= 2).
    alpha may be one order per component ([d]): a batch of one on the DIRECT
    kernels (non-commensurate orders)."""
    import numpy as np
    import torch
    if np.ndim(alpha) == 1:
        y, _, st = solve_batch(system, np.reshape(theta, (1, -1)), np.reshape(alpha, (1, -1)),
                               [h], [N], _dev(y0)[None], path=path, far_prec=far_prec, plan=plan)
        return y, st
    y0, d, two = _init_rows(y0, 0)
    th = _dev(theta).reshape(-1)
    if plan is None:
        plan = fabm_plan(system, d, path, far_prec, 1, N, tile_L=tile_L, initial_slope=two,
                         fft_level=fft_level)
    ws = _workspace(fabm_workspace_size(plan, [N]))
    y = torch.empty((N + 1, d), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int64, device="cuda")
    fabm_solve(plan, ws, alpha, h, N, y0, th, y, st)
    return y, st


def solve_batch(system, thetas, alphas, hs, Ns, y0s, path="auto", far_prec="fp64",
                plan: Plan | None = None, tile_L: int = 0):
    """Ragged batch; returns (y_rows [sum(N+1), d], row_off numpy, status tensor).
    y0s is [B, d], or [B, 2, d] with y'(0) as the second row (orders above one);
    alphas is [B], or [B, d] for a separate order per component (DIRECT)."""
    import numpy as np
    import torch
    y0s, d, two = _init_rows(y0s, 1)
    B = int(y0s.shape[0])
    pc = np.ndim(alphas) == 2
    th = _dev(thetas).reshape(B, -1)
    Ns = np.ascontiguousarray(Ns, dtype=np.int64)
    row_off = np.zeros(B, dtype=np.int64)
    row_off[1:] = np.cumsum(Ns + 1)[:-1]
    if plan is None:
        plan = fabm_plan(system, d, path, far_prec, B, int(Ns.max()), int(Ns.sum()),
                         tile_L=tile_L, initial_slope=two, per_component_order=pc)
    ws = _workspace(fabm_workspace_size(plan, Ns))
    y = torch.empty((int((Ns + 1).sum()), d), dtype=torch.float64, device="cuda")
    st = torch.zeros(B, dtype=torch.int64, device="cuda")
    fabm_solve_batch(plan, ws, alphas, hs, Ns, y0s, th, row_off, y, st)
    return y, row_off, st


def adjoint_batch(system, thetas, alphas, hs, Ns, y0s, gy, plan: Plan | None = None,
                  checkpoint: bool = False):
    """Gradients of sum <gy, y> for a ragged batch (gy rows placed as solve_batch
    returns y); returns (gy0 shaped like y0s, gtheta [B, n_params], status)
    device tensors (with [B, 2, d] initial values gy0 holds dL/dy(0), dL/dy'(0))."""
    import numpy as np
    import torch
    y0s, d, two = _init_rows(y0s, 1)
    B = int(y0s.shape[0])
    pc = np.ndim(alphas) == 2
    th = _dev(thetas).reshape(B, -1)
    gy = _dev(gy)
    Ns = np.ascontiguousarray(Ns, dtype=np.int64)
    row_off = np.zeros(B, dtype=np.int64)
    row_off[1:] = np.cumsum(Ns + 1)[:-1]
    if plan is None:
        plan = fabm_plan(system, d, "blocked", "fp64", B, int(Ns.max()), int(Ns.sum()),
                         initial_slope=two, per_component_order=pc,
                         adjoint_checkpoint=checkpoint)
    ws = _workspace(fabm_adjoint_workspace_size(plan, Ns))
    gy0 = torch.empty_like(y0s)
    gth = torch.empty_like(th)
    st = torch.zeros(B, dtype=torch.int64, device="cuda")
    fabm_adjoint(plan, ws, alphas, hs, Ns, y0s, th, row_off, gy, gy0, gth, st)
    return gy0, gth, st


def _solve_function():
    import torch

    class FabmSolveBatch(torch.autograd.Function):
        """y = solve_batch(...) as a differentiable function of y0 [B, d] (or
        [B, 2, d] with y'(0), orders above one) and theta [B, n_params];
        backward runs the blocked reverse pass.
        Rows of y are the instances' trajectories concatenated (row_off as in
        solve_batch)."""

        @staticmethod
        def forward(ctx, y0s, thetas, system, alphas, hs, Ns, checkpoint=False):
            # the forward pass of the adjoint: the workspace it leaves (rows,
            # predictor rows, history) is kept for the backward pass
            import numpy as np
            import torch
            y0d, d, two = _init_rows(y0s.detach(), 1)
            B = int(y0d.shape[0])
            th = _dev(thetas.detach()).reshape(B, -1).contiguous()
            al = np.asarray(alphas, dtype=np.float64)
            hh = np.asarray(hs, dtype=np.float64)
            Ns = np.ascontiguousarray(Ns, dtype=np.int64)
            row_off = np.zeros(B, dtype=np.int64)
            row_off[1:] = np.cumsum(Ns + 1)[:-1]
            plan = fabm_plan(system, d, "blocked", "fp64", B, int(Ns.max()), int(Ns.sum()),
                             initial_slope=two, per_component_order=al.ndim == 2,
                             adjoint_checkpoint=bool(checkpoint))
            ws = _workspace(fabm_adjoint_workspace_size(plan, Ns))
            y = torch.empty((int((Ns + 1).sum()), d), dtype=torch.float64, device="cuda")
            st = torch.zeros(B, dtype=torch.int64, device="cuda")
            fabm_adjoint_forward(plan, ws, al, hh, Ns, y0d, th, row_off, y, st)
            ctx.save_for_backward(y0d, th)
            ctx.meta = (plan, ws, al, hh, Ns, row_off)
            return y

        @staticmethod
        def backward(ctx, gy):
            import torch
            y0d, th = ctx.saved_tensors
            plan, ws, al, hh, Ns, row_off = ctx.meta
            gy0 = torch.empty_like(y0d)
            gth = torch.empty_like(th)
            fabm_adjoint_reverse(plan, ws, al, hh, Ns, y0d, th, row_off,
                                 _dev(gy).contiguous(), gy0, gth)
            ctx.meta = None  # release the workspace
            return gy0, gth, None, None, None, None, None

    return FabmSolveBatch


def solve_batch_autograd(y0s, thetas, system, alphas, hs, Ns, checkpoint: bool = False):
    """Differentiable batched solve (torch autograd; see FabmSolveBatch).
    checkpoint: block checkpoints in the adjoint (FABM_PLAN_ADJOINT_CHECKPOINT)."""
    return _solve_function().apply(y0s, thetas, system, alphas, hs, Ns, checkpoint)
