"""Python face of the CPU oracle (``fabm_oracle.c``).

TEST INFRASTRUCTURE. The oracle is the plain, slow, FP64 (binary128 weights,
long-double history sums) statement of the fractional Adams-Bashforth-Moulton
PECE scheme of Section 2 of arXiv:1611.08678. Only ``tests/``, the package
smoke check and the CPU-baseline leg of ``bench.py`` may import this module.
It never imports the GPU package and the GPU package never imports it.

``build()`` compiles ``liboracle.so`` next to this file with gcc (no fast-math,
no FMA contraction); ``lib()`` loads it, building on first use.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fabm_oracle.c")
SO = os.path.join(HERE, "liboracle.so")

# Own numbering of the right-hand sides (see fabm_oracle.c).
LINEAR, CHEN, ROSSLER, VDP, FINANCIAL, HINDMARSH_ROSE = 0, 1, 2, 3, 4, 5

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc; returns its path."""
    if not force and os.path.exists(SO) and os.path.getmtime(SO) >= os.path.getmtime(SRC):
        return SO
    tmp = SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", tmp, SRC, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
RHS_CB = C.CFUNCTYPE(None, C.c_double, _D, _D, C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(SO)
        L.oracle_weights.argtypes = [C.c_double, C.c_int64, _D, _D, _D]
        L.oracle_solve.argtypes = [C.c_int, C.c_int, _D, C.c_double, C.c_double, C.c_int64,
                                   _D, _D, _D, _D, _D, _D, _D]
        L.oracle_solve.restype = C.c_int64
        L.oracle_solve_cb.argtypes = [RHS_CB, C.c_void_p, C.c_int, C.c_double, C.c_double,
                                      C.c_int64, _D, _D, _D, _D]
        L.oracle_solve_cb.restype = C.c_int64
        L.oracle_solve_batch.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, _D, _D,
                                         _I64,
                                         _D, _D, _I64, _D, _D, _D, _I64]
        L.oracle_history_sums.argtypes = [C.c_double, C.c_int64, C.c_int, _D, _D, _D, _D, _D]
        L.oracle_history_sums_rows.argtypes = [C.c_double, C.c_int64, C.c_int, _D, C.c_int64,
                                               _I64, _D, _D, _D, _D]
        L.oracle_solve_orders.argtypes = [C.c_int, C.c_int, _D, _D, C.c_double, C.c_int64, _D,
                                          C.c_int, _D, _D, _D]
        L.oracle_solve_orders.restype = C.c_int64
        L.oracle_solve_orders_cb.argtypes = [RHS_CB, C.c_void_p, C.c_int, _D, C.c_double,
                                             C.c_int64, _D, C.c_int, _D, _D, _D]
        L.oracle_solve_orders_cb.restype = C.c_int64
        L.oracle_solve_orders_batch.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                                _D, _D, _I64, _D, _D, _I64, _D, _I64]
        L.oracle_adjoint_orders.argtypes = [C.c_int, C.c_int, _D, _D, C.c_double, C.c_int64,
                                            _D, C.c_int, _D, _D, _D]
        L.oracle_adjoint_orders.restype = C.c_int64
        L.oracle_adjoint.argtypes = [C.c_int, C.c_int, _D, C.c_double, C.c_double, C.c_int64,
                                     _D, _D, _D, _D]
        L.oracle_adjoint.restype = C.c_int64
        L.oracle_rhs.argtypes = [C.c_int, C.c_int, _D, C.c_double, _D, _D]
        L.oracle_threads.restype = C.c_int
        L.oracle_rhs_rows.argtypes = [C.c_int, C.c_int, _D, C.c_double, C.c_int64, _D, _D]
        L.oracle_step_from_history.argtypes = [C.c_int, C.c_int, _D, C.c_double, C.c_double,
                                               C.c_int64, _D, _D, _D, _D, _D, _D, _D]
        L.oracle_n_params.argtypes = [C.c_int, C.c_int]
        L.oracle_n_params.restype = C.c_int
        L.oracle_dim.argtypes = [C.c_int, C.c_int]
        L.oracle_dim.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def n_params(system: int, d: int) -> int:
    return lib().oracle_n_params(system, d)


def dim(system: int, d_linear: int = 0) -> int:
    return lib().oracle_dim(system, d_linear)


def weights(alpha: float, n: int):
    """b_m, a_m, c_m for m = 0..n-1 (Section 2 weight definitions)."""
    b, a, c = (np.empty(n) for _ in range(3))
    lib().oracle_weights(float(alpha), int(n), _p(b), _p(a), _p(c))
    return b, a, c


def rhs(system: int, theta, t: float, y):
    y = _f64(y)
    th = _f64(theta)
    f = np.empty_like(y)
    lib().oracle_rhs(system, y.size, _p(th), float(t), _p(y), _p(f))
    return f


def rhs_rows(system: int, theta, h: float, y):
    """f(t_k, y_k) for every row k of y ([n, d]), t_k = k h."""
    y = _f64(y)
    f = np.empty_like(y)
    lib().oracle_rhs_rows(system, y.shape[1], _p(_f64(theta).ravel()), float(h), y.shape[0],
                          _p(y), _p(f))
    return f


def _init(y0, alpha):
    """Initial values as [ceil(alpha)][d] rows (y(0), then y'(0) for alpha > 1):
    y0 is [d] or [1|2][d]. Returns (flat array, d, rows given)."""
    y0 = _f64(y0)
    rows = 1 if y0.ndim == 1 else y0.shape[0]
    d = y0.shape[-1]
    assert rows in (1, 2) and (alpha <= 1.0 or rows == 2), "alpha > 1 needs y(0) and y'(0)"
    return np.ascontiguousarray(y0.reshape(rows * d)), d, rows


def step_from_history(system: int, theta, alpha: float, h: float, t: int, y0, f_hist,
                      weights_bac):
    """Teacher-forced step: y_t from the history rows f_0..f_{t-1} (f_hist has
    at least t rows), with weight tables of length >= t. Returns (y_t, mag)
    where mag is h^alpha times the sum of the magnitudes of the history terms."""
    y0, d, _ = _init(y0, alpha)
    f = _f64(f_hist)
    assert f.shape[0] >= t and f.shape[1] == d
    wb, wa, wc = (_f64(w) for w in weights_bac)
    assert min(wb.size, wa.size, wc.size) >= t
    y, mag = np.empty(d), np.empty(d)
    lib().oracle_step_from_history(system, d, _p(_f64(theta).ravel()), float(alpha), float(h),
                                   int(t), _p(y0), _p(f), _p(wb), _p(wa), _p(wc), _p(y), _p(mag))
    return y, mag


def solve(system: int, theta, alpha: float, h: float, N: int, y0, weights_bac=None):
    """One trajectory. y0 is y(0) [d], or [2][d] holding y(0) and y'(0) (needed
    for 1 < alpha <= 2). Returns (y [N+1,d], yP [N+1,d], f [N+1,d], status)."""
    y0, d, _ = _init(y0, alpha)
    th = _f64(theta).ravel()
    y = np.empty((N + 1, d))
    yp = np.empty((N + 1, d))
    f = np.empty((N + 1, d))
    wb = wa = wc = None
    if weights_bac is not None:
        wb, wa, wc = (_f64(w) for w in weights_bac)
    st = lib().oracle_solve(system, d, _p(th), float(alpha), float(h), int(N), _p(y0),
                            _p(wb), _p(wa), _p(wc), _p(y), _p(yp), _p(f))
    return y, yp, f, int(st)


def solve_callback(fn, alpha: float, h: float, N: int, y0):
    """One trajectory with a Python right-hand side fn(t, y) -> f (small N only);
    y0 as in solve()."""
    y0, d, _ = _init(y0, alpha)

    def _cb(t, yptr, fptr, _user):
        yy = np.ctypeslib.as_array(yptr, shape=(d,)).copy()
        out = np.asarray(fn(t, yy), dtype=np.float64)
        for i in range(d):
            fptr[i] = float(out[i])

    cb = RHS_CB(_cb)
    y = np.empty((N + 1, d))
    yp = np.empty((N + 1, d))
    f = np.empty((N + 1, d))
    st = lib().oracle_solve_cb(cb, None, d, float(alpha), float(h), int(N), _p(y0), _p(y),
                               _p(yp), _p(f))
    return y, yp, f, int(st)


def solve_batch(system: int, thetas, alphas, hs, Ns, y0s, want_f: bool = False):
    """Ragged batch. y0s is [B][d], or [B][2][d] with y'(0) as the second row
    (used by instances with alpha > 1). Returns (y_rows, row_off, status[,
    f_rows]); instance i occupies rows row_off[i] .. row_off[i] + N_i of y_rows."""
    y0s = _f64(y0s)
    B, d = y0s.shape[0], y0s.shape[-1]
    n_init = 1 if y0s.ndim == 2 else y0s.shape[1]
    assert n_init in (1, 2) and (n_init == 2 or np.all(_f64(alphas) <= 1.0))
    y0s = np.ascontiguousarray(y0s.reshape(B * n_init * d))
    th = _f64(thetas).reshape(B, -1)
    al = _f64(alphas).ravel()
    hh = _f64(hs).ravel()
    Nn = np.ascontiguousarray(Ns, dtype=np.int64).ravel()
    off = np.zeros(B, dtype=np.int64)
    off[1:] = np.cumsum(Nn + 1)[:-1]
    rows = int((Nn + 1).sum())
    y = np.empty((rows, d))
    f = np.empty((rows, d)) if want_f else None
    st = np.zeros(B, dtype=np.int64)
    lib().oracle_solve_batch(system, d, th.shape[1], n_init, B, _p(al), _p(hh),
                             Nn.ctypes.data_as(_I64), _p(y0s), _p(th),
                             off.ctypes.data_as(_I64), _p(y), None, _p(f),
                             st.ctypes.data_as(_I64))
    if want_f:
        return y, off, st, f
    return y, off, st


def _orders_init(y0, alphas):
    """Initial values [n_init][d] for per-component orders (y'(0) needed when
    any component's order exceeds one)."""
    y0 = _f64(y0)
    rows = 1 if y0.ndim == 1 else y0.shape[0]
    assert rows in (1, 2) and (np.all(_f64(alphas) <= 1.0) or rows == 2)
    return np.ascontiguousarray(y0.reshape(-1)), y0.shape[-1], rows


def solve_orders(system: int, theta, alphas, h: float, N: int, y0):
    """One trajectory with a separate order per component (alphas [d]); y0 is
    [d] or [2][d] as in solve(). Returns (y, yP, f, status)."""
    al = np.ascontiguousarray(_f64(alphas).ravel())
    init, d, rows = _orders_init(y0, al)
    assert al.size == d
    y, yp, f = (np.empty((N + 1, d)) for _ in range(3))
    st = lib().oracle_solve_orders(system, d, _p(_f64(theta).ravel()), _p(al), float(h), int(N),
                                   _p(init), rows, _p(y), _p(yp), _p(f))
    return y, yp, f, int(st)


def solve_orders_callback(fn, alphas, h: float, N: int, y0):
    """Per-component orders with a Python right-hand side (small N only)."""
    al = np.ascontiguousarray(_f64(alphas).ravel())
    init, d, rows = _orders_init(y0, al)

    def _cb(t, yptr, fptr, _user):
        out = np.asarray(fn(t, np.ctypeslib.as_array(yptr, shape=(d,)).copy()), dtype=np.float64)
        for i in range(d):
            fptr[i] = float(out[i])

    cb = RHS_CB(_cb)
    y, yp, f = (np.empty((N + 1, d)) for _ in range(3))
    st = lib().oracle_solve_orders_cb(cb, None, d, _p(al), float(h), int(N), _p(init), rows,
                                      _p(y), _p(yp), _p(f))
    return y, yp, f, int(st)


def solve_orders_batch(system: int, thetas, alphas, hs, Ns, y0s):
    """Ragged batch with per-component orders: alphas [B][d], y0s [B][d] or
    [B][2][d]. Returns (y_rows, row_off, status) as solve_batch."""
    y0s = _f64(y0s)
    B, d = y0s.shape[0], y0s.shape[-1]
    n_init = 1 if y0s.ndim == 2 else y0s.shape[1]
    al = np.ascontiguousarray(_f64(alphas).reshape(B, d))
    assert n_init == 2 or np.all(al <= 1.0)
    th = _f64(thetas).reshape(B, -1)
    Nn = np.ascontiguousarray(Ns, dtype=np.int64).ravel()
    off = np.zeros(B, dtype=np.int64)
    off[1:] = np.cumsum(Nn + 1)[:-1]
    y = np.empty((int((Nn + 1).sum()), d))
    st = np.zeros(B, dtype=np.int64)
    lib().oracle_solve_orders_batch(system, d, th.shape[1], n_init, B, _p(al),
                                    _p(_f64(hs).ravel()), Nn.ctypes.data_as(_I64),
                                    _p(np.ascontiguousarray(y0s.reshape(-1))), _p(th),
                                    off.ctypes.data_as(_I64), _p(y), st.ctypes.data_as(_I64))
    return y, off, st


def adjoint_orders(system: int, theta, alphas, h: float, N: int, y0, gy):
    """Discrete adjoint of solve_orders for L = sum_n <gy[n], y[n]>. Returns
    (gy0 shaped like y0, gtheta, status)."""
    al = np.ascontiguousarray(_f64(alphas).ravel())
    shape = np.shape(y0)
    init, d, rows = _orders_init(y0, al)
    th = _f64(theta).ravel()
    g = _f64(gy).reshape(N + 1, d)
    gy0 = np.zeros(rows * d)
    gth = np.empty(max(th.size, 1))
    st = lib().oracle_adjoint_orders(system, d, _p(th), _p(al), float(h), int(N), _p(init), rows,
                                     _p(g), _p(gy0), _p(gth))
    return gy0.reshape(shape), gth[: th.size], int(st)


def history_sums(alpha: float, f_hist):
    """Teacher-forced sums P_t, C_t (t = 1..N) for history rows f_0..f_{N-1},
    with their magnitude sums. Returns (P, C, Pabs, Cabs), each [N, d]."""
    f = _f64(f_hist)
    if f.ndim == 1:
        f = f[:, None]
    N, d = f.shape
    P, Cc, Pa, Ca = (np.empty((N, d)) for _ in range(4))
    lib().oracle_history_sums(float(alpha), int(N), int(d), _p(f), _p(P), _p(Cc), _p(Pa), _p(Ca))
    return P, Cc, Pa, Ca


def history_sums_rows(alpha: float, f_hist, rows):
    """history_sums for the targets in `rows` only (1 <= t <= N, N = len(f_hist)).
    Returns (P, C, Pabs, Cabs), each [len(rows), d]."""
    f = _f64(f_hist)
    if f.ndim == 1:
        f = f[:, None]
    N, d = f.shape
    r = np.ascontiguousarray(rows, dtype=np.int64).ravel()
    assert r.size == 0 or (r.min() >= 1 and r.max() <= N)
    P, Cc, Pa, Ca = (np.empty((r.size, d)) for _ in range(4))
    lib().oracle_history_sums_rows(float(alpha), int(N), int(d), _p(f), int(r.size),
                                   r.ctypes.data_as(_I64), _p(P), _p(Cc), _p(Pa), _p(Ca))
    return P, Cc, Pa, Ca


def adjoint(system: int, theta, alpha: float, h: float, N: int, y0, gy):
    """Discrete adjoint for L = sum_n <gy[n], y[n]>. Returns (gy0, gtheta, status);
    gy0 has the shape of y0 ([d], or [2][d] with the gradient with respect to
    y'(0) in the second row, zero for alpha <= 1)."""
    shape = np.shape(y0)
    y0, d, rows = _init(y0, alpha)
    th = _f64(theta).ravel()
    g = _f64(gy).reshape(N + 1, d)
    gy0 = np.zeros(rows * d)
    gth = np.empty(max(th.size, 1))
    st = lib().oracle_adjoint(system, d, _p(th), float(alpha), float(h), int(N), _p(y0), _p(g),
                              _p(gy0), _p(gth))
    return gy0.reshape(shape), gth[: th.size], int(st)


def threads() -> int:
    """OpenMP threads of the oracle's parallel loops (batches, history sums)."""
    return int(lib().oracle_threads())
