#!/usr/bin/env python3
"""Benchmark: immersed-boundary time steps per second on one MI355X.

Workload (default): the helix256 configuration -- a 256^3 periodic grid and
1.5M markers (a 1200 x 500 basilar-membrane strip plus a 1800 x 500 tethered
tube wall), dt = 2.5e-5, 1 kHz window drive; synthetic inputs from the seeded
generator.  A "step" is one full time step: binning, force, spreading with
advection/RHS, FFT Navier-Stokes solve, interpolation and move.

The timed region runs ``--steps`` steps of the mixed-precision step (FP32
fluid, FP64 markers) after ``--warmup`` untimed steps, bracketed by
synchronisations; ``value`` is steps/s.  The same steps are then run with an
FP64 fluid for comparison, and the maximum relative velocity difference
between the two is reported.  Per-phase HIP-event timers give the dominant
kernel's average duration, from which the roofline fraction follows.  The
oracle (plain FP64 CPU) is timed on a bounded sample for ``cpu_baseline``.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure


def phase_bytes(phase: str, N: int, M: int, b: int, touched_tiles: int) -> float:
    """Algorithmic HBM bytes per launch of each phase (the per-unit figures of the design notes)."""
    G = N ** 3
    spec = 3 * (N // 2 + 1) * N * N * 2 * b
    grid = 3 * G * b
    return {
        "fft_x": grid + spec,
        "fft_y": 2 * spec,
        "fft_z_solve": 2 * spec,
        "fft_y_inv": 2 * spec,
        "fft_x_inv": spec + grid,
        "rhs": 2 * grid + touched_tiles * 512 * 3 * b,
        "spread": M * (4 + 6 * b) + touched_tiles * 512 * 3 * b,
        "interp": M * (4 + 4 + 3 * b + 48),
        "bin": M * (24 + 8) + 3 * M * 20,
        "force": M * (24 + 24 + 8 + 8 + 8 + 24),
        "prep": M * (4 + 24 + 24 + 6 * b),
    }.get(phase, float("nan"))


def run_gpu(wl, precision, steps, warmup, timers=False):
    import torch
    from paper_math_0301321_amd import ib
    ctx = ib.Context(wl, precision)
    X = torch.as_tensor(wl.X0, dtype=torch.float64, device="cuda").contiguous()
    u = ctx.new_grid()
    n = 0
    for _ in range(warmup):
        ctx.step(X, u, n * wl.dt)
        n += 1
    torch.cuda.synchronize()
    if timers:
        ctx.timers_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        ctx.step(X, u, n * wl.dt)
        n += 1
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    ph = ctx.timers_read() if timers else {}
    if timers:
        ctx.timers_enable(False)
    return dict(ctx=ctx, X=X, u=u, wall=wall, ev_ms=ev_ms, phases=ph)


def cpu_baseline(wl, sample_steps: int):
    import numpy as np
    import oracle
    model = oracle.Model(wl)
    X = wl.X0.copy()
    u = np.zeros((3, wl.N, wl.N, wl.N))
    t0 = time.perf_counter()
    for n in range(sample_steps):
        X, u = oracle.step(model, wl, X, u, n * wl.dt)
    dt = time.perf_counter() - t0
    return {"value": sample_steps / dt, "unit": "steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{sample_steps} full FP64 oracle step(s) of {wl.name} ({wl.N}^3 grid, {wl.M} markers), "
                      f"{dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=None, help="steps of the FP64 comparison run (default: --steps)")
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_math_0301321_amd import workloads as W

    wl = W.config3(N=args.grid)
    print(f"[bench] workload {wl.name}: N={wl.N} M={wl.M}", file=sys.stderr, flush=True)
    mixed = run_gpu(wl, "fp32", args.steps, args.warmup, timers=True)
    ms_per_step = mixed["ev_ms"] / args.steps
    value = args.steps / (mixed["ev_ms"] / 1e3)
    print(f"[bench] mixed: {ms_per_step:.4f} ms/step ({value:.1f} steps/s), wall {mixed['wall']:.3f} s",
          file=sys.stderr, flush=True)

    # dominant kernel and its roofline
    ph = mixed["phases"]
    phases = {k: {"ms_avg": v[0] / v[1], "launches": v[1]} for k, v in ph.items()}
    dom = max(ph.items(), key=lambda kv: kv[1][0])[0] if ph else None
    roof = None
    if dom:
        avg_ms = ph[dom][0] / ph[dom][1]
        nbytes = phase_bytes(dom, wl.N, wl.M, 4, 0)
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": nbytes, "avg_ms": round(avg_ms, 5)}
    step_bytes = sum(phase_bytes(k, wl.N, wl.M, 4, 0) * v[1] for k, v in ph.items()) / max(1, args.steps)

    extra = {}
    if not args.no_fp64:
        k64 = args.fp64_steps or args.steps
        fp64 = run_gpu(wl, "fp64", k64, args.warmup)
        v64 = k64 / (fp64["ev_ms"] / 1e3)
        extra["fp64_steps_per_s"] = round(v64, 2)
        extra["mixed_speedup_vs_fp64"] = round(value / v64, 3)
        if k64 == args.steps:
            um, u64 = mixed["u"].double(), fp64["u"]
            extra["mixed_vs_fp64_rel_u"] = float((um - u64).abs().max() / u64.abs().max())
            dX64 = fp64["X"] - torch.as_tensor(wl.X0, device="cuda")
            dXm = mixed["X"] - torch.as_tensor(wl.X0, device="cuda")
            extra["mixed_vs_fp64_rel_dX"] = float((dXm - dX64).abs().max() / dX64.abs().max())
        print(f"[bench] fp64: {v64:.1f} steps/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_sample_steps)

    out = {
        "metric": "IB steps/s at 256^3 grid + 1.5M markers; mixed vs FP64 at stated error",
        "value": round(value, 2), "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.N}^3 periodic grid, {wl.M} markers (BM 1200x500 + wall 1800x500), "
                               f"dt {wl.dt}, {wl.drive_freq:g} Hz drive", "grid": wl.N, "markers": wl.M,
                   "precision": "FP32 fluid, FP64 markers and forces", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phases_ms": {k: round(v["ms_avg"], 5) for k, v in phases.items()},
        "model_bytes_per_step": step_bytes,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
