"""Benchmark of the fractional ABM hot path on one MI355X.

Workload: the single fractional Chen trajectory (a, b, c) = (35, 3, 28),
alpha = 0.95, y0 = (-9, -5, 14), h = 0.001, N = 2^20 steps (d = 3). One
bench "step" is one complete solve (weight generation, history contraction,
predictor/corrector updates, output) with inputs already in device memory.

Prints one JSON line: steps*states/s of the headline path (`value`), history
GFLOP/s (2 d N (N+1) flops per trajectory), the per-path breakdown (direct vs
blocked), the roofline of the dominant kernel and the CPU oracle timed on a
bounded sample of the same trajectory.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--paths", default="blocked,direct", help="comma list of blocked,direct")
    ap.add_argument("--direct-steps", type=int, default=1,
                    help="timed solves of the (slow) direct comparison path")
    ap.add_argument("--cpu-sample", type=int, default=1 << 15,
                    help="steps of the oracle sample for cpu_baseline (0 disables)")
    return ap.parse_args()


def time_path(F, w, path: str, steps: int, warmup: int):
    import torch
    N = int(w["N"][0])
    d = w["d"]
    plan = F.fabm_plan(w["system"], d, path, "fp64", 1, N)
    ws = torch.empty(F.fabm_workspace_size(plan, [N]), dtype=torch.uint8, device="cuda")
    y0 = torch.as_tensor(w["y0"][0], device="cuda").contiguous()
    th = torch.as_tensor(w["theta"][0], device="cuda").contiguous()
    y = torch.empty((N + 1, d), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int64, device="cuda")
    args = (plan, ws, float(w["alpha"][0]), float(w["h"][0]), N, y0, th, y, st)
    for _ in range(warmup):
        F.fabm_solve(*args)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        F.fabm_solve(*args)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) / 1e3 for a, b in evs]
    return dict(path=path, wall_s=wall, solve_s=per, y=y.cpu().numpy(), status=int(st.item()))


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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1611_08678_amd as F
    from paper_1611_08678_amd import workloads as W

    F.load()
    w = W.chen(N=args.N)
    N, d = int(w["N"][0]), w["d"]
    flops = 2.0 * d * N * (N + 1)
    results = {}
    for path in [p for p in args.paths.split(",") if p]:
        head_path = path == "blocked" or "blocked" not in args.paths
        r = time_path(F, w, path, args.steps if head_path else args.direct_steps,
                      args.warmup if head_path else 0)
        results[path] = r
        print(f"# {path}: solve times {['%.4f' % s for s in r['solve_s']]} s", file=sys.stderr,
              flush=True)
    head = "blocked" if "blocked" in results else "direct"
    r = results[head]
    t = float(np.mean(r["solve_s"]))
    value = N * d / t

    # roofline of the dominant kernel of the headline path
    if head == "direct":
        alg_bytes = 4.0 * N * (N + 1) * (d + 2)  # sum_t 8 t (d + 2): history row + two weights
        achieved = alg_bytes / t / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=None, kernel="k_direct_grid",
                    algorithmic_bytes=alg_bytes)
    else:
        achieved = flops / t / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=78.6, unit="TFLOP/s",
                    frac=achieved / 78.6, traffic=None, kernel="k_blocked")

    out = {
        "metric": "steps*states/s (history GFLOP/s alongside), blocked vs direct, at stated rel err",
        "value": value, "unit": "steps*states/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"fractional Chen (35,3,28), alpha=0.95, y0=(-9,-5,14), "
                               f"h=0.001, N={N}, d=3, single trajectory",
                   "path": head, "far_prec": "fp64"},
        "history_gflops": flops / t / 1e9,
        "paths": {k: {"solve_s": float(np.mean(v["solve_s"])),
                      "steps_states_per_s": N * d / float(np.mean(v["solve_s"])),
                      "history_gflops": flops / float(np.mean(v["solve_s"])) / 1e9,
                      "status": v["status"]} for k, v in results.items()},
        "roofline": roof,
    }
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
