"""Bounds of the reduced-precision parity tests (binary32 and split binary16
far tiles of the BLOCKED paths).

Per test case the bound is twice the normwise error against the FP64 oracle
measured on MI355X for that case (`MEASURED`). Beside it stands the a-priori
model of one far sum: binary32 windows round every operand once and sum the
64 products of a window (16 lags x 4) in binary32, so a far sum is off by at
most (2 + 64) u32 of its magnitude sum |w| |f| (u32 = 2^-24); split binary16
operands carry 22 significant bits (hi + lo, the lo*lo product dropped,
2^-22 relative) and one block of 64 source rows is summed in binary32, so
(2 + 1 + 64) u32. Propagated through the stable dynamics of these tests, and
scaled by h^alpha, that is far above what the tests measure (the per-term
errors are not all of one sign); the model is reported with each case
(`model_bound`), the measured x 2 is what is asserted. The test of the
teacher-forced contraction (tests/test_gpu_history.py) asserts the model
itself per far sum.

Running the GPU tests with FABM_MEASURE_REDUCED=1 prints the error of every
case (`MEASURED <case> <error>`) and skips these assertions: that is how the
table below was taken."""
from __future__ import annotations

import os

U32 = 2.0 ** -24
MODEL_FP32 = (2 + 64) * U32       # one far sum, relative to its magnitude
MODEL_FP16X2 = (2 + 1 + 64) * U32

# normwise error vs the FP64 oracle measured for each case on MI355X
MEASURED = {
    "blocked_fp32_batch": 1.345e-06,
    "blocked_fp32_single": 5.573e-06,
    "fft_far_fp32_windows": 3.343e-06,
    "orders_fp32_hindmarsh_rose": 1.564e-06,
    "orders_fp32_linear3": 4.875e-07,
    "orders_fp32_vdp": 1.488e-06,
    "rossler_full_fp32_prefix": 1.236e-06,
    "rossler_full_fp32_reformed": 3.962e-08,   # relative to the history magnitude
    "slope_mixed_fp32_sys0_d3": 7.335e-06,
    "slope_mixed_fp32_sys3_d2": 6.692e-06,
    "slope_mixed_fp32_sys4_d3": 3.883e-05,
    "slope_shared_grid_fp16x2": 1.137e-06,
    "slope_shared_grid_fp32": 1.335e-06,
    "wide_alpha0.05_fp16x2": 2.677e-08,
    "wide_alpha1.0_fp16x2": 2.426e-08,
    "wide_blowup_fp16x2": 2.974e-07,
    "wide_fp32_blowup": 1.204e-14,             # two blocks: no far windows run
    "wide_linear64_fp16x2_prefix": 2.005e-07,
    "wide_linear64_fp16x2_reformed": 6.574e-08,
    "wide_linear64_fp32_prefix": 3.163e-07,
    "wide_linear64_fp32_reformed": 7.356e-08,
    "wide_magnitudes_fp16x2": 1.824e-07,
    "wide_magnitudes_fp32": 2.684e-07,
    "wide_reduced_fp16x2": 1.930e-07,
    "wide_reduced_fp32": 2.417e-07,
}


def measuring() -> bool:
    return os.environ.get("FABM_MEASURE_REDUCED", "") not in ("", "0")


def bound(case: str) -> float:
    return 2.0 * MEASURED[case]


def check(case: str, err: float, cap: float) -> None:
    """Assert err <= 2 x the measured error of `case` (and never above `cap`,
    the a-priori sanity bound of the test); print it in measuring mode."""
    if measuring():
        print(f"MEASURED {case} {err:.3e}", flush=True)
        assert err <= cap, (case, err, cap)
        return
    assert case in MEASURED, f"no measured error for {case}"
    assert err <= min(bound(case), cap), (case, err, MEASURED[case], cap)
