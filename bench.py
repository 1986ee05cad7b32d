"""Benchmark of the fractional ABM hot path on one MI355X.

Workload: the single fractional Chen trajectory (a, b, c) = (35, 3, 28),
alpha = 0.95, y0 = (-9, -5, 14), h = 0.001, N = 2^20 steps (d = 3). One
bench "step" is one complete solve (weight generation, history contraction,
predictor/corrector updates, output) with inputs already in device memory.

Prints one JSON line: steps*states/s of the headline (BLOCKED) path as
`value`, history GFLOP/s (2 d N (N+1) flops per trajectory), the per-path
breakdown (DIRECT vs BLOCKED), the roofline of the dominant kernel from HIP
events recorded by the library on the kernel's own stream, and the CPU oracle
timed on a bounded sample of the same trajectory.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a
# reference copy kernel (profiles/k_step_chen_N2p20_pmc.md), valid only for
# the kernel source it was measured on (sha256 prefix of blocked.hip).
MEASURED_TRAFFIC = {"k_step": (59.12e6, "66c96f50e43922b2")}
FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
FP16_MFMA_PEAK_TFLOPS = 2500.0  # dense binary16 matrix rate
HBM_PEAK_GBPS = 8000.0
BAND_CYCLES_PER_ROW = 587  # band-dominated last launches of the trace (profiles/k_step_chen_N2p20_kernel_stats.md)
CLOCK_HZ = 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--paths", default="blocked,direct", help="comma list of blocked,direct")
    ap.add_argument("--direct-steps", type=int, default=1,
                    help="timed solves of the (slow) direct comparison path")
    ap.add_argument("--cpu-sample", type=int, default=1 << 15,
                    help="steps of the oracle sample for cpu_baseline (0 disables)")
    ap.add_argument("--no-kernel-times", action="store_true",
                    help="skip the instrumented solve that measures per-kernel time")
    ap.add_argument("--workload", default="chen",
                    choices=["chen", "rossler_batch", "vdp_batch", "vdp_adjoint",
                             "linear64_batch", "hr_table2"],
                    help="chen: the headline single trajectory; the batch workloads are "
                         "additional measurements of the batched BLOCKED path; hr_table2: "
                         "one Hindmarsh-Rose trajectory swept over the step counts of the "
                         "paper's Section 4 timing table")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before the benchmark "
                         "(untimed; a reference kernel of known traffic for hardware counters)")
    ap.add_argument("--batch-path", default="blocked", choices=["blocked", "direct"],
                    help="batch workloads: the path to time (direct: one workgroup per "
                         "instance, HBM-bound)")
    ap.add_argument("--tune", action="store_true",
                    help="batch workloads: run fabm_tune on the plan before timing (untimed)")
    ap.add_argument("--per-component-orders", action="store_true",
                    help="batch workloads: a separate order per state component, alpha ~ "
                         "U[0.8, 1] (non-commensurate system; DIRECT, or BLOCKED with FP64 "
                         "far windows)")
    ap.add_argument("--alpha", type=float, default=None,
                    help="batch workloads: one order for every instance (1 < alpha <= 2 "
                         "needs --slope)")
    ap.add_argument("--slope", action="store_true",
                    help="batch workloads: pass y'(0) ~ 0.5 N(0, 1) as a second initial "
                         "row (orders above one, eq. (1))")
    ap.add_argument("--fft-level", type=int, default=0,
                    help="chen / hr_table2: far history of block squares of this level and "
                         "above by FFT convolution (sub-quadratic variant; 0 = off)")
    ap.add_argument("--sweep-N", default=None,
                    help="hr_table2: comma list of step counts (default: all of the table's)")
    ap.add_argument("--far-prec", default=None, choices=["fp64", "fp32", "fp16x2"],
                    help="far-window arithmetic (default: fp64; rossler_batch: fp32; "
                         "fp16x2 only for linear64_batch)")
    return ap.parse_args()


def setup(F, w, path, fft_level=0):
    import torch
    N = int(w["N"][0])
    d = w["d"]
    plan = F.fabm_plan(w["system"], d, path, "fp64", 1, N,
                       fft_level=fft_level if path == "blocked" else 0)
    ws = torch.empty(F.fabm_workspace_size(plan, [N]), dtype=torch.uint8, device="cuda")
    y0 = torch.as_tensor(w["y0"][0], device="cuda").contiguous()
    th = torch.as_tensor(w["theta"][0], device="cuda").contiguous()
    y = torch.empty((N + 1, d), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int64, device="cuda")
    return plan, (plan, ws, float(w["alpha"][0]), float(w["h"][0]), N, y0, th, y, st), y, st


def time_path(F, w, path: str, steps: int, warmup: int, kernel_times: bool, fft_level: int = 0):
    import torch
    plan, args, y, st = setup(F, w, path, fft_level)
    for _ in range(warmup):
        F.fabm_solve(*args)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        F.fabm_solve(*args)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) / 1e3 for a, b in evs]
    out = dict(path=path, wall_s=wall, solve_s=per, y=y.cpu().numpy(), status=int(st.item()))
    if kernel_times:
        # one extra, instrumented solve: the library records an event pair on
        # each kernel's own stream around every launch
        F.fabm_plan_set_profiling(plan, True)
        F.fabm_solve(*args)
        torch.cuda.synchronize()
        out["kernel_times"] = F.fabm_plan_kernel_times(plan)
        F.fabm_plan_set_profiling(plan, False)
    return out


def cpu_baseline(w, n_sample: int, N: int):
    """Oracle (single trajectory, one thread) on the first n_sample steps of the
    same trajectory, scaled to the full N by the N(N+1) cost of the history sums."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    yref, _, _, st = O.solve(w["system"], w["theta"][0], float(w["alpha"][0]),
                             float(w["h"][0]), n_sample, w["y0"][0])
    dt = time.perf_counter() - t0
    scale = (N * (N + 1)) / (n_sample * (n_sample + 1))
    t_full = dt * scale
    return yref, dict(value=N * w["d"] / t_full, unit="steps*states/s", cores=1, kind="oracle",
                      sample=(f"first {n_sample} steps of the same trajectory, {dt:.2f} s on 1 "
                              f"host thread, extrapolated by N(N+1) to N={N}"),
                      sample_seconds=dt)


def measured_traffic(kernel: str):
    """Counter-measured HBM bytes per launch, or None if the kernel source has
    changed since the counters were taken."""
    import hashlib
    val, sha = MEASURED_TRAFFIC.get(kernel, (None, None))
    if val is None:
        return None
    src = os.path.join(ROOT, "paper_1611_08678_amd", "csrc", "blocked.hip")
    with open(src, "rb") as f:
        cur = hashlib.sha256(f.read()).hexdigest()[:16]
    return val if cur == sha else None


def roofline(kt: dict, N: int, d: int, fft_level: int = 0):
    """Roofline object of the dominant kernel of the headline path, from the
    library's per-launch HIP events (recorded on the kernel's own stream).
    With the FFT variant the flops are direct-equivalent: the 2 d N (N + 1) of
    the plain sums, of which the variant performs O(N log^2 N)."""
    if not kt:
        return None
    dom = max(kt, key=lambda k: kt[k][0])
    secs, launches = kt[dom]
    flops = 2.0 * d * N * (N + 1)  # algorithmic history flops of one solve
    if dom == "blocked_step" and fft_level > 0:
        band_floor = N * BAND_CYCLES_PER_ROW / CLOCK_HZ
        fsecs, fl = kt.get("fft_far", (0.0, 0))
        ach = flops / secs / 1e12
        return dict(bound="mfma", achieved=ach, peak=FP64_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP64_MFMA_PEAK_TFLOPS, traffic=None, kernel="k_step",
                    flops_basis="direct-equivalent 2 d N (N + 1) (sub-quadratic variant)",
                    launches=launches, avg_launch_s=secs / launches,
                    fft_far=dict(seconds=fsecs, launches=fl),
                    sequential_floor=dict(s=band_floor, frac=band_floor / (secs + fsecs),
                                          basis=f"N rows x {BAND_CYCLES_PER_ROW} cycles per row "
                                                f"of the band walk at {CLOCK_HZ / 1e9:.1f} GHz"))
    if dom == "blocked_step":
        # every history flop of the BLOCKED path is done inside the step
        # kernels (MFMA near/far windows plus the sequential band)
        ach = flops / secs / 1e12
        # the band forms one row after another: N rows at the walk's measured
        # cycles per row (2.4 GHz) bound the solve from below whatever the
        # matrix cores do
        band_floor = N * BAND_CYCLES_PER_ROW / CLOCK_HZ
        return dict(bound="mfma", achieved=ach, peak=FP64_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP64_MFMA_PEAK_TFLOPS, traffic=measured_traffic("k_step"),
                    kernel="k_step",
                    launches=launches, avg_launch_s=secs / launches,
                    algorithmic_flops_per_launch=flops / launches,
                    sequential_floor=dict(s=band_floor, frac=band_floor / secs,
                                          basis=f"N rows x {BAND_CYCLES_PER_ROW} cycles per row "
                                                f"of the band walk at {CLOCK_HZ / 1e9:.1f} GHz"))
    if dom == "direct_grid":
        alg_bytes = 4.0 * N * (N + 1) * (d + 2)  # sum_t 8 t (d + 2): history row + two weights
        ach = alg_bytes / secs / 1e9
        return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None, kernel="k_direct_grid",
                    launches=launches, avg_launch_s=secs / launches,
                    algorithmic_bytes_per_launch=alg_bytes / launches)
    return dict(bound="unknown", kernel=dom, seconds=secs)


def bench_batch(F, W, args):
    """Batched BLOCKED solve of a batch workload: Rossler (4096 instances,
    N uniform in [2^14, 2^17], per-instance alpha, FP32 far windows), the
    Van der Pol forward pass (1024 instances, N = 2^15), or the linear d = 64
    batch (512 instances sharing alpha = 0.8, h = 0.01, N = 2^16: the
    shared-grid form, far tiles FP64, FP32 or FP16X2)."""
    import numpy as np
    import torch
    w = {"rossler_batch": W.rossler_batch, "linear64_batch": W.linear64_batch}.get(
        args.workload, W.vdp_adjoint)()
    pc = args.per_component_orders
    if pc:
        if args.batch_path == "blocked" and (args.far_prec or "fp64") != "fp64":
            sys.exit("--per-component-orders on the BLOCKED path takes FP64 far windows")
        # the workload's own order range: Rossler's [0.9, 1], else [0.8, 1]
        w = W.per_component_orders(w, lo=0.9 if args.workload == "rossler_batch" else 0.8)
    prec = args.far_prec or ("fp32" if args.workload == "rossler_batch" and not pc else "fp64")
    Ns = np.asarray(w["N"], dtype=np.int64)
    B, d = len(Ns), w["d"]
    if args.alpha is not None:
        w = dict(w, alpha=np.full(w["alpha"].shape, args.alpha))
    if args.slope:
        slope = 0.5 * np.random.Generator(np.random.PCG64(7)).standard_normal((B, d))
        w = dict(w, y0=np.stack([w["y0"], slope], axis=1))
    plan = F.fabm_plan(w["system"], d, args.batch_path, prec, B, int(Ns.max()), int(Ns.sum()),
                       per_component_order=pc, initial_slope=args.slope)
    ws = torch.empty(F.fabm_workspace_size(plan, Ns), dtype=torch.uint8, device="cuda")
    y0 = torch.as_tensor(w["y0"], dtype=torch.float64, device="cuda").contiguous()
    th = torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda").contiguous()
    row_off = np.zeros(B, dtype=np.int64)
    row_off[1:] = np.cumsum(Ns + 1)[:-1]
    y = torch.empty((int((Ns + 1).sum()), d), dtype=torch.float64, device="cuda")
    st = torch.zeros(B, dtype=torch.int64, device="cuda")
    call = lambda: F.fabm_solve_batch(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, y, st)
    tune = None
    if args.tune:
        tune = F.fabm_tune(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, y, st)
        print(f"# tune: {tune}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        call()
        b.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) / 1e3 for a, b in evs]
    print(f"# {args.workload}: solve times {['%.4f' % t for t in per]} s", file=sys.stderr,
          flush=True)
    kt = {}
    if not args.no_kernel_times:
        F.fabm_plan_set_profiling(plan, True)
        call()
        torch.cuda.synchronize()
        kt = {k: v for k, v in F.fabm_plan_kernel_times(plan).items() if v[1]}
    t = float(np.mean(per))
    # an instance whose state leaves every bounded set stops at its status
    # step (later rows NaN, its remaining windows skipped): count the rows
    # actually formed
    stv = st.cpu().numpy()
    Neff = np.where(stv > 0, stv - 1, Ns).astype(np.float64)
    flops = float((2.0 * d * Neff * (Neff + 1)).sum())
    out = {"metric": "steps*states/s (history GFLOP/s alongside), batched blocked",
           "value": float(Neff.sum()) * d / t, "unit": "steps*states/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp64": "f64", "fp32": "f64 band, f32 far windows",
                     "fp16x2": "f64 band, fp16 hi+lo far tiles (f32 sums)"}[prec],
           "data": "synthetic",
           "config": {"workload": w["name"], "batch": B, "N_min": int(Ns.min()),
                      "N_max": int(Ns.max()), "path": args.batch_path,
                      "far_prec": prec if args.batch_path == "blocked" else None,
                      "orders": (f"per component, U[{float(np.min(w['alpha'])):.2f}.., 1]"
                                 if pc else "one per instance"),
                      "alpha": args.alpha, "initial_slope": args.slope},
           "history_gflops": flops / t / 1e9,
           "status_nonzero": int((stv != 0).sum()),
           "rows_counted": "rows formed: N_i, or status_i - 1 for instances that left every "
                           "bounded set",
           "tune": tune,
           "kernel_times_s": {k: v[0] for k, v in kt.items()},
           "kernel_launches": {k: v[1] for k, v in kt.items()}}
    if "blocked_step" in kt:
        secs, launches = kt["blocked_step"]
        peak = FP32_MFMA_PEAK_TFLOPS if prec == "fp32" else FP64_MFMA_PEAK_TFLOPS
        ach = flops / secs / 1e12
        out["roofline"] = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                               frac=ach / peak, traffic=None, kernel="k_step_batch",
                               launches=launches, avg_launch_s=secs / launches,
                               algorithmic_flops_per_launch=flops / launches)
    if "direct_wg" in kt:
        secs, launches = kt["direct_wg"]
        # every step reads the history (d values per row) and the weight rows
        # b, a: one pair per instance, or one per component with per-component orders
        by = float((4.0 * Neff * (Neff + 1) * (3 * d if pc else d + 2)).sum())
        out["roofline"] = dict(bound="hbm", achieved=by / secs / 1e9, peak=HBM_PEAK_GBPS,
                               unit="GB/s", frac=by / secs / 1e9 / HBM_PEAK_GBPS, traffic=None,
                               kernel="k_direct_wg", launches=launches,
                               avg_launch_s=secs / launches, algorithmic_bytes_per_launch=by)
    if "wide_far" in kt:
        # far sums of the shared grid: every target row t takes the 64 * (t // 64)
        # source rows of earlier blocks, both tables, every column
        secs, launches = kt["wide_far"]
        t_rows = np.arange(int(Neff.max()) + 1, dtype=np.float64)
        far_flops = float((4.0 * B * d * 64.0 * np.floor(t_rows / 64.0)).sum())
        hw = 3.0 if prec == "fp16x2" else 1.0  # hi*hi + hi*lo + lo*hi products
        peak = {"fp64": FP64_MFMA_PEAK_TFLOPS, "fp32": FP32_MFMA_PEAK_TFLOPS,
                "fp16x2": FP16_MFMA_PEAK_TFLOPS}[prec]
        ach = hw * far_flops / secs / 1e12
        # history read by the far launches: every earlier row, every column,
        # once per workgroup column tile (8, 4 or 2 + 2 bytes per value)
        eb = {"fp64": 8.0, "fp32": 4.0, "fp16x2": 4.0}[prec]
        hist = float((64.0 * np.floor(t_rows[::64] / 64.0)).sum()) * B * d * eb
        if prec == "fp16x2":
            # 64 flop per history byte: 512 TFLOP/s at 8 TB/s, below the
            # 833 TFLOP/s of algorithmic work the binary16 matrix cores give at
            # three products per term, so HBM bounds this kernel
            out["roofline"] = dict(bound="hbm", achieved=hist / secs / 1e9, peak=HBM_PEAK_GBPS,
                                   unit="GB/s", frac=hist / secs / 1e9 / HBM_PEAK_GBPS,
                                   traffic=None, kernel="k_wide_far", launches=launches,
                                   avg_launch_s=secs / launches,
                                   algorithmic_bytes_per_launch=hist / launches,
                                   mfma_tflops=ach, mfma_frac=ach / peak,
                                   mfma_flops_per_algorithmic_flop=hw)
        else:
            out["roofline"] = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                                   frac=ach / peak, traffic=None, kernel="k_wide_far",
                                   launches=launches, avg_launch_s=secs / launches,
                                   algorithmic_flops_per_launch=far_flops / launches,
                                   history_gbps=hist / secs / 1e9)
    if args.cpu_sample > 0 and args.workload == "linear64_batch":
        # oracle check of the first 1000 steps of the first and last instance
        from oracle import oracle as O
        errs = []
        for i in (0, B - 1):
            ref, _, _, _ = O.solve(w["system"], w["theta"][i], float(w["alpha"][i]),
                                   float(w["h"][i]), 1000, w["y0"][i])
            g = y[int(row_off[i]):int(row_off[i]) + 1001].cpu().numpy()
            errs.append(float(np.abs(g - ref).max() / np.abs(ref).max()))
        out["rel_err_first_1000_steps"] = errs
    elif args.cpu_sample > 0:
        # oracle check of the three shortest instances
        from oracle import oracle as O
        yy = y.cpu().numpy()
        errs = []
        for i in np.argsort(Ns)[:3]:
            if pc:
                ref, _, _, _ = O.solve_orders(w["system"], w["theta"][i], w["alpha"][i],
                                              float(w["h"][i]), int(Ns[i]), w["y0"][i])
            else:
                ref, _, _, _ = O.solve(w["system"], w["theta"][i], float(w["alpha"][i]),
                                       float(w["h"][i]), int(Ns[i]), w["y0"][i])
            g = yy[row_off[i]:row_off[i] + Ns[i] + 1]
            errs.append(float(np.abs(g - ref).max() / np.abs(ref).max()))
        out["rel_err_shortest_3"] = errs
    print(json.dumps(out), flush=True)


def bench_adjoint(F, W, args):
    """Van der Pol x1024, N = 2^15: forward solve, MSE loss against targets from
    mu + N(0, 0.05) (computed once by the same forward pass, untimed) and the
    adjoint for d/dmu and d/dy0. Timed: forward + backward, as a training step
    does it: fabm_adjoint_forward (trajectory and the adjoint's workspace),
    loss gradient, fabm_adjoint_reverse. The one-call fabm_adjoint (which
    recomputes the forward) after a plain solve is timed beside it."""
    import numpy as np
    import torch
    w = W.vdp_adjoint()
    Ns = np.asarray(w["N"], dtype=np.int64)
    B, d = len(Ns), w["d"]
    plan = F.fabm_plan(w["system"], d, "blocked", "fp64", B, int(Ns.max()), int(Ns.sum()))
    ws = torch.empty(max(F.fabm_workspace_size(plan, Ns), F.fabm_adjoint_workspace_size(plan, Ns)),
                     dtype=torch.uint8, device="cuda")
    y0 = torch.as_tensor(w["y0"], dtype=torch.float64, device="cuda").contiguous()
    th = torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda").contiguous()
    tht = torch.as_tensor(w["theta_target"], dtype=torch.float64, device="cuda").contiguous()
    row_off = np.zeros(B, dtype=np.int64)
    row_off[1:] = np.cumsum(Ns + 1)[:-1]
    rows = int((Ns + 1).sum())
    y = torch.empty((rows, d), dtype=torch.float64, device="cuda")
    yt = torch.empty_like(y)
    st = torch.zeros(B, dtype=torch.int64, device="cuda")
    gy0 = torch.empty((B, d), dtype=torch.float64, device="cuda")
    gth = torch.empty_like(th)
    F.fabm_solve_batch(plan, ws, w["alpha"], w["h"], Ns, y0, tht, row_off, yt, st)
    scale = 2.0 / (rows * d)  # d/dy of the mean of squared differences

    def step():
        F.fabm_adjoint_forward(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, y, st)
        gy = (y - yt) * scale
        F.fabm_adjoint_reverse(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, gy, gy0, gth)
        return gy

    def step_one_call():
        F.fabm_solve_batch(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, y, st)
        gy = (y - yt) * scale
        F.fabm_adjoint(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, gy, gy0, gth, st)
        return gy

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        gy = step()
        b.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) / 1e3 for a, b in evs]
    print(f"# vdp_adjoint: forward+backward times {['%.4f' % t for t in per]} s", file=sys.stderr,
          flush=True)
    step_one_call()
    a, b = evs[0]
    a.record(stream)
    step_one_call()
    b.record(stream)
    torch.cuda.synchronize()
    one_call = a.elapsed_time(b) / 1e3
    step()  # leave the split path's gradients in gy0, gth
    F.fabm_plan_set_profiling(plan, True)
    F.fabm_adjoint(plan, ws, w["alpha"], w["h"], Ns, y0, th, row_off, gy, gy0, gth, st)
    torch.cuda.synchronize()
    kt = {k: v for k, v in F.fabm_plan_kernel_times(plan).items() if v[1]}
    t = float(np.mean(per))
    flops = float((2.0 * d * Ns * (Ns + 1)).sum())
    out = {"metric": "forward + backward (adjoint) time of a batched solve, d/dmu and d/dy0",
           "value": t, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": w["name"], "batch": B, "N": int(Ns.max())},
           "history_gflops_fwd_plus_bwd": 2.0 * flops / t / 1e9,
           "solve_then_one_call_adjoint_s": one_call,
           "adjoint_kernel_times_s": {k: v[0] for k, v in kt.items()},
           "adjoint_kernel_launches": {k: v[1] for k, v in kt.items()}}
    if args.cpu_sample > 0:
        from oracle import oracle as O
        i = 0
        g = gy.cpu().numpy()[row_off[i]:row_off[i] + Ns[i] + 1]
        t0 = time.perf_counter()
        rg0, rgt, _ = O.adjoint(w["system"], w["theta"][i], float(w["alpha"][i]), float(w["h"][i]),
                                int(Ns[i]), w["y0"][i], g)
        dt = time.perf_counter() - t0
        ref = np.concatenate([rg0, rgt])
        got = np.concatenate([gy0.cpu().numpy()[i], gth.cpu().numpy()[i]])
        out["grad_rel_err_vs_oracle_instance0"] = float(np.abs(got - ref).max() / np.abs(ref).max())
        out["oracle_adjoint_seconds_one_instance"] = dt
    print(json.dumps(out), flush=True)


# Average seconds the paper reports for its Hindmarsh-Rose runs (Section 4,
# Table 2) on a BlueGene/P partition and on a CUDA GPU, neither named further;
# model parameters, alpha, h and precision of those runs are not given, so
# these are context for the shape of the sweep, not a baseline of this workload.
PAPER_TABLE2_S = {100_000: (170.75, 169.06), 500_000: (1592.66, 1276.42),
                  1_000_000: (4621.25, 2670.56), 1_500_000: (9162.33, 4450.09),
                  2_000_000: (14931.16, 6639.45), 2_500_000: (22697.66, 9229.66),
                  3_000_000: (31659.66, 12226.39)}


def bench_table2(F, W, args):
    """One Hindmarsh-Rose trajectory (d = 3) solved by the BLOCKED path at each
    step count of the paper's timing table. `value` is the whole sweep's
    steps*states over its summed solve time; each N is also reported alone."""
    import numpy as np
    rows, tot_states, tot_t = [], 0.0, 0.0
    head = None
    Ns = [int(n) for n in args.sweep_N.split(",")] if args.sweep_N else list(W.TABLE2_N)
    for N in Ns:
        w = W.hindmarsh_rose(N=N)
        print(f"# hr_table2: N={N} blocked, {args.warmup} warmup + {args.steps} timed",
              file=sys.stderr, flush=True)
        r = time_path(F, w, "blocked", args.steps, args.warmup,
                      kernel_times=not args.no_kernel_times, fft_level=args.fft_level)
        t = float(np.mean(r["solve_s"]))
        y = r["y"]
        hpc, cuda = PAPER_TABLE2_S.get(N, (None, None))
        rows.append(dict(N=N, solve_s=t, steps_states_per_s=N * 3 / t,
                         history_gflops=2.0 * 3 * N * (N + 1) / t / 1e9, status=r["status"],
                         finite=bool(np.all(np.isfinite(y))),
                         x_range=[float(y[:, 0].min()), float(y[:, 0].max())],
                         paper_cuda_s=cuda, paper_hpc_s=hpc,
                         ratio_paper_cuda_over_this=cuda / t if cuda else None))
        print(f"# hr_table2: N={N} solve {t:.4f} s", file=sys.stderr, flush=True)
        tot_states += N * 3
        tot_t += t
        head = (N, r)
    N, r = head
    value = tot_states / tot_t
    out = {
        "metric": "steps*states/s (history GFLOP/s alongside), blocked path, N sweep",
        "value": value, "unit": "steps*states/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tot_t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": ("fractional Hindmarsh-Rose (a,b,c,d,r,s,xr,I)=(1,3,1,5,0.006,4,"
                                "-1.6,3.25), alpha=0.95, h=0.01, y0=(-1.6,-10,2), d=3, one "
                                "trajectory per N, N in " + ",".join(str(n) for n in Ns)),
                   "path": "blocked", "far_prec": "fp64", "fft_level": args.fft_level},
        "sweep": rows,
        "paper_context": ("paper Table 2: average seconds on a BlueGene/P partition and an "
                          "unnamed CUDA GPU for Hindmarsh-Rose runs of unstated parameters, "
                          "step size and precision; ratios are context, not a baseline"),
    }
    kt = r.get("kernel_times")
    if kt:
        out["kernel_times_s_at_largest_N"] = {k: v[0] for k, v in kt.items() if v[1]}
    out["roofline"] = roofline({k: v for k, v in (kt or {}).items() if v[1]}, N, 3,
                               args.fft_level)
    if out["roofline"]:
        out["roofline"]["at_N"] = N
    if args.cpu_sample > 0:
        w = W.hindmarsh_rose(N=N)
        yref, cpu = cpu_baseline(w, min(args.cpu_sample, N), N)
        n = yref.shape[0]
        out["cpu_baseline"] = cpu
        scale = np.abs(yref).max()
        out["rel_err_sample_prefix"] = float((np.abs(r["y"][:n] - yref).max(axis=1) /
                                              scale).max())
    print(json.dumps(out), flush=True)


def copy_reference(mib: int):
    """One device-to-device copy of `mib` MiB (reads and writes that many bytes)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"# copy reference: {mib} MiB read + {mib} MiB written", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_mib > 0:
        copy_reference(args.copy_mib)
    if args.workload != "chen":
        import paper_1611_08678_amd as F
        from paper_1611_08678_amd import workloads as W
        F.load()
        if args.workload == "vdp_adjoint":
            return bench_adjoint(F, W, args)
        if args.workload == "hr_table2":
            return bench_table2(F, W, args)
        return bench_batch(F, W, args)
    import numpy as np
    import paper_1611_08678_amd as F
    from paper_1611_08678_amd import workloads as W

    F.load()
    w = W.chen(N=args.N)
    N, d = int(w["N"][0]), w["d"]
    flops = 2.0 * d * N * (N + 1)
    results = {}
    paths = [p for p in args.paths.split(",") if p]
    for path in paths:
        head_path = path == "blocked" or "blocked" not in paths
        r = time_path(F, w, path, args.steps if head_path else args.direct_steps,
                      args.warmup if head_path else 0,
                      kernel_times=head_path and not args.no_kernel_times,
                      fft_level=args.fft_level)
        results[path] = r
        print(f"# {path}: solve times {['%.4f' % s for s in r['solve_s']]} s", file=sys.stderr,
              flush=True)
    head = "blocked" if "blocked" in results else "direct"
    r = results[head]
    t = float(np.mean(r["solve_s"]))
    value = N * d / t

    out = {
        "metric": "steps*states/s (history GFLOP/s alongside), blocked vs direct, at stated rel err",
        "value": value, "unit": "steps*states/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"fractional Chen (35,3,28), alpha=0.95, y0=(-9,-5,14), "
                               f"h=0.001, N={N}, d=3, single trajectory",
                   "path": head, "far_prec": "fp64", "fft_level": args.fft_level},
        "history_gflops": flops / t / 1e9,
        "paths": {k: {"solve_s": float(np.mean(v["solve_s"])),
                      "steps_states_per_s": N * d / float(np.mean(v["solve_s"])),
                      "history_gflops": flops / float(np.mean(v["solve_s"])) / 1e9,
                      "status": v["status"]} for k, v in results.items()},
    }
    kt = r.get("kernel_times")
    if kt:
        out["kernel_times_s"] = {k: v[0] for k, v in kt.items() if v[1]}
        out["kernel_launches"] = {k: v[1] for k, v in kt.items() if v[1]}
    out["roofline"] = roofline({k: v for k, v in (kt or {}).items() if v[1]}, N, d,
                               args.fft_level)
    if "direct" in results:
        # DIRECT reads both weight rows and the history at every step:
        # sum_t 8 t (d + 2) B = 4 N (N + 1) (d + 2) B (algorithmic)
        by = 4.0 * N * (N + 1) * (d + 2)
        td = float(np.mean(results["direct"]["solve_s"]))
        out["paths"]["direct"]["algorithmic_hbm_gbps"] = by / td / 1e9
        out["paths"]["direct"]["hbm_frac"] = by / td / 1e9 / HBM_PEAK_GBPS
    if "direct" in results and "blocked" in results:
        out["blocked_speedup_over_direct"] = (np.mean(results["direct"]["solve_s"]) /
                                              np.mean(results["blocked"]["solve_s"]))
    if args.cpu_sample > 0:
        yref, cpu = cpu_baseline(w, min(args.cpu_sample, N), N)
        out["cpu_baseline"] = cpu
        n = yref.shape[0]
        scale = np.abs(yref).max()
        for k, v in results.items():
            e = np.abs(v["y"][:n] - yref).max(axis=1) / scale
            out["paths"][k]["rel_err_first_4096"] = float(e[:4097].max())
            out["paths"][k]["rel_err_sample_prefix"] = float(e.max())
        out["rel_err_note"] = ("chaotic system: normwise error vs the FP64 oracle is stated on "
                               "the first 4096 steps (before rounding differences amplify) and on "
                               "the whole sampled prefix")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
