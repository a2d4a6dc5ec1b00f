#!/usr/bin/env python3
"""Benchmark of the multi-tracer PLIC-VoF hot path on one MI355X.

Workload (default): a 512^3 tri-periodic box with 8 FP64 tracer fields
holding ~5508 drops of diameter 24 cells (+-10%) at volume fraction 0.3,
placed by random sequential addition with a 1-cell gap, and a frozen random
solenoidal velocity (modes 1 <= |k| <= 8, E(k) ~ k^-5/3, rms 0.2 cells per
step, rise 0.1). All inputs are synthetic and seeded.

A step is one direction-split advection step of all tracers (three sweep
launches). `value` is the whole-job advection throughput in tracer-cell-steps
per second with the fields resident in HBM, timed with HIP events on the
stream the kernels run on. The line also carries the HBM roofline of the
sweep kernel and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "VoF cell-updates/s per tracer (FP64) at % HBM roofline; learned vs HF curvature cells/s"


def sweep_bytes(n3: int, ntr: int) -> float:
    """Algorithmic HBM bytes of one sweep launch: read and write every tracer
    field (16 B per tracer-cell), read the face velocity once for all tracers
    (8 B per cell) and one c > 0.5 bit per tracer-cell (written by the first
    sweep of a step, read by the other two)."""
    return n3 * ntr * 16.0 + n3 * 8.0 + n3 * ntr / 8.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="box size (cells per side)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-tracers", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 2:
        args.steps += 1  # an even number of steps leaves the result in place (no final copy)

    import numpy as np
    import torch

    from paper_2407_07463_amd import synth, vofmt

    n = args.n
    t0 = time.time()
    w = synth.random_drops(n, 8, 0.3, 24.0, 0.1, 1.0, seed=synth.workload_seed(2), order=8, workers=16)
    ntr = w["ntracers"]
    log(f"workload generated in {time.time() - t0:.1f}s: {len(w['radii'])} drops, rms {w['rms']:.3f}")
    dev = torch.device("cuda:0")
    c = torch.from_numpy(w["c"]).to(dev)
    s = [torch.from_numpy(w[k]).to(dev) for k in ("sx", "sy", "sz")]
    ctx = vofmt.Context(0)
    smax = ctx.check_courant(*s)
    stream = torch.cuda.current_stream()
    n3 = n**3

    # warmup
    ctx.advect(c, *s, step0=0, nsteps=max(args.warmup, 1) * 2)
    torch.cuda.synchronize()
    log("warmup done")

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    ctx.advect(c, *s, step0=0, nsteps=args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ms_step = ms / args.steps
    value = n3 * ntr * args.steps / (ms / 1e3)
    nsweeps = 3 * args.steps
    per_launch_s = ms / 1e3 / nsweeps
    achieved = sweep_bytes(n3, ntr) / per_launch_s / 1e9
    log(f"advection: {ms_step:.3f} ms/step, {value:.3e} tracer-cell-steps/s, {achieved:.0f} GB/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tracer-cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"drops{n}: {n}^3 tri-periodic box, {ntr} FP64 tracers, {len(w['radii'])} drops of "
                        f"diameter 24+-10% at phi=0.3 (RSA, gap 1), random solenoidal velocity (|k|<=8, "
                        f"k^-5/3, rms {w['rms']:.3f}, rise 0.1, max|s| {smax:.3f})",
            "grid": [n, n, n],
            "tracers": ntr,
        },
        "per_tracer_cell_steps_per_s": value / ntr,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_sweep<D> (one launch = one sweep of all tracers)",
            "bytes_per_launch": sweep_bytes(n3, ntr),
        },
    }

    if not args.no_cpu_baseline:
        import oracle

        k = args.cpu_sample_tracers
        host_c = w["c"][:k]
        log(f"cpu baseline: oracle, {k} tracers of the same field, 1 step")
        t1 = time.time()
        oracle.advect(host_c, w["sx"], w["sy"], w["sz"], 0, 1)
        dt = time.time() - t1
        out["cpu_baseline"] = {
            "value": n3 * k / dt,
            "unit": "tracer-cell-steps/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle advection of {k} of the {ntr} tracer fields of the same {n}^3 workload, "
                      f"1 step ({dt:.1f} s)",
        }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
