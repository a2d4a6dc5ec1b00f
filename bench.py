#!/usr/bin/env python3
"""Benchmark of the multi-tracer PLIC-VoF hot path on one MI355X.

Workload (default): a 512^3 tri-periodic box with 8 FP64 tracer fields
holding ~5508 drops of diameter 24 cells (+-10%) at volume fraction 0.3,
placed by random sequential addition with a 1-cell gap, and a frozen random
solenoidal velocity (modes 1 <= |k| <= 8, E(k) ~ k^-5/3, rms 0.2 cells per
step, rise 0.1). All inputs are synthetic and seeded.

A step is one direction-split advection step of all tracers (three sweeps,
each a PLIC pass over the mixed cells and streaming passes over the fields;
--sweeps paired runs two sweeps per streaming pass instead). `value` is the
whole-job advection throughput in tracer-cell-steps per second with the
fields resident in HBM, timed with HIP events on the stream the kernels run
on. `roofline` is that of the dominant kernel, the streaming pass (k_stream;
k_pair when paired), from its own launches timed with HIP events in a second
timed region of the same K steps; `traffic` comes from the committed
rocprofv3 counter summary when the advection sources have not changed since.

The same line carries, under `rows`, the other steps of the path measured on
the advected field: drop labelling, moments, recolouring, pair statistics,
height-function and learned curvature (cells/s, matrix-core rate), network
training, and batched advection of 32 uneven boxes (graph launch vs plain
launches); and under `cpu_baseline` the CPU oracle timed on a bounded sample.

--pmc-pass: a short run for rocprofv3 counter collection: a plain copy of
1 GiB (the calibration kernel), 2 advection steps, then two surface-tension
force evaluations of the advected tracers; prints one line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix cores
METRIC = "VoF cell-updates/s per tracer (FP64) at % HBM roofline; learned vs HF curvature cells/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_k_pair_drops512.txt")
TRAFFIC_FILE_SINGLE = os.path.join(ROOT, "profiles", "hbm_traffic_k_stream_drops512.txt")
COPY_BYTES = 1 << 30


def stream_bytes(n3: int, g: int) -> float:
    """Algorithmic HBM bytes of one streaming pass over g tracers: read and
    write every field value (16 B per tracer-cell), read the face velocity
    (8 B per cell) and one c > 0.5 bit per tracer-cell."""
    return n3 * (16.0 * g + 8.0 + g / 8.0)


def pair_bytes(n3: int, ntr: int, candidates: bool) -> float:
    """Algorithmic HBM bytes of one paired streaming pass over all tracers:
    read and write every field value once (16 B per tracer-cell), read the
    face velocities of both sweeps (8 B per cell each) and, when it lists the
    candidates of the following sweep, that sweep's face velocity; one c > 0.5
    bit per tracer-cell."""
    return n3 * (16.0 * ntr + 8.0 * (3 if candidates else 2) + ntr / 8.0)


def step_model_bytes(n3: int, ntr: int) -> float:
    """Per-step model of the method: three sweeps, each reading and writing
    every field once, reading the velocity once for all tracers and the
    c > 0.5 bits (51.5 B per tracer-cell-step at 8 tracers)."""
    return 3.0 * (n3 * ntr * 16.0 + n3 * 8.0 + n3 * ntr / 8.0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(torch, stream, fn):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    r = fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b), r


def rows_bench(torch, np, ctx, stream, c, w, n, ntr):
    """Timings of the other steps of the path on the advected field."""
    from paper_2407_07463_amd import synth, training

    dev = c.device
    rows = {}
    n3 = n ** 3
    # ---- labelling and moments
    lab = torch.zeros(c.shape, dtype=torch.int32, device=dev)
    ctx.label_drops(c, lab)  # warm
    ms, nd = timed(torch, stream, lambda: ctx.label_drops(c, lab))
    D = int(nd.sum())
    rows["label_drops"] = dict(ms=ms, drops=D, cells_per_s=n3 * ntr / (ms / 1e3))
    log(f"label_drops: {ms:.2f} ms, {D} drops")
    vol = torch.zeros(D, dtype=torch.float64, device=dev)
    xyz = torch.zeros((D, 3), dtype=torch.float64, device=dev)
    ctx.drop_moments(c, lab, nd, vol, xyz)
    ms, _ = timed(torch, stream, lambda: ctx.drop_moments(c, lab, nd, vol, xyz))
    rows["drop_moments"] = dict(ms=ms)
    log(f"drop_moments: {ms:.2f} ms")
    # ---- drop shapes: inertia tensors, aspect ratios and mean velocities
    sv = [torch.from_numpy(w[k]).to(dev) for k in ("sx", "sy", "sz")]
    inertia = torch.zeros((D, 6), dtype=torch.float64, device=dev)
    chi = torch.zeros(D, dtype=torch.float64, device=dev)
    velo = torch.zeros((D, 3), dtype=torch.float64, device=dev)
    ctx.drop_shapes(c, lab, nd, inertia, chi, sv, velo)
    ms, _ = timed(torch, stream, lambda: ctx.drop_shapes(c, lab, nd, inertia, chi, sv, velo))
    rows["drop_shapes"] = dict(ms=ms, drops=D, chi_mean=float(chi.mean().item()),
                               chi_max=float(chi.max().item()))
    log(f"drop_shapes: {ms:.2f} ms, mean aspect ratio {rows['drop_shapes']['chi_mean']:.4f}")
    del sv, inertia, chi, velo
    # ---- recolouring (on a copy with room for 2N tracers)
    cap = 2 * ntr
    cr = torch.zeros((cap,) + tuple(c.shape[1:]), dtype=torch.float64, device=dev)
    newt = torch.zeros(max(D, 1), dtype=torch.int32, device=dev)
    # one untimed call first (it sizes the scratch buffers), then the timed
    # call on a fresh copy of the same fields
    for _ in range(2):
        cr.zero_()
        cr[:ntr].copy_(c)
        ms, (ntr2, moved) = timed(torch, stream, lambda: ctx.recolor_tracers(cr, ntr, lab, nd, 1.5, newt))
    rows["recolor_tracers"] = dict(ms=ms, tracers_after=ntr2, drops_moved=moved, gap_cells=1.5)
    log(f"recolor_tracers: {ms:.2f} ms, {moved} drops moved, {ntr2} tracers")
    del cr, newt
    # ---- nearest-particle pair statistics, 64 x 32 histogram
    nr, nth = 64, 32
    r2e = (np.arange(nr + 1) * (4 * 24.0 / nr)) ** 2
    ce = np.linspace(1.0, -1.0, nth + 1)
    idx = torch.zeros(D, dtype=torch.int32, device=dev)
    ties = torch.zeros(D, dtype=torch.int32, device=dev)
    hist = torch.zeros(nr * nth + 1, dtype=torch.int64, device=dev)
    M = torch.zeros(3, dtype=torch.float64, device=dev)
    R = torch.zeros(9, dtype=torch.float64, device=dev)
    box = [float(n)] * 3
    ctx.nearest_pair_stats(xyz, box, 2, r2e, ce, idx, ties, hist, M, R)
    ms, _ = timed(torch, stream, lambda: ctx.nearest_pair_stats(xyz, box, 2, r2e, ce, idx, ties, hist, M, R))
    rows["nearest_pair_stats"] = dict(ms=ms, drops=D, histogram=[nr, nth])
    log(f"nearest_pair_stats: {ms:.2f} ms")
    del lab
    # ---- curvature of one tracer: height functions vs network + fallback
    P, meta = training.load_weights()
    Pd = torch.from_numpy(P).to(dev)
    c0 = c[0].contiguous()
    kap = torch.zeros(c0.shape, dtype=torch.float64, device=dev)
    st = torch.zeros(c0.shape, dtype=torch.uint8, device=dev)
    nmix = int(((c0 > 0) & (c0 < 1)).sum().item())
    # both methods' first pass (the ordered list of mixed cells, NaN elsewhere) is the same
    ctx.curvature_hf(c0, kap, st)
    ctx.profile_start()
    ms_hf, _ = timed(torch, stream, lambda: ctx.curvature_hf(c0, kap, st))
    prof_hf = ctx.profile_stop()
    ctx.curvature_mlp(c0, Pd, meta["kappa_lo"], kap, st)
    ctx.profile_start()
    ms_comb, _ = timed(torch, stream, lambda: ctx.curvature_mlp(c0, Pd, meta["kappa_lo"], kap, st))
    prof = ctx.profile_stop()
    hf_kernel_ms = prof_hf["k_curv_hf_list"][1]
    mlp_kernel_ms = prof["k_curv_fused"][1] + prof.get("k_curv_fallback", (1, 0.0))[1]
    # the network alone on the canonical stencils of the mixed cells
    xs = torch.zeros((nmix, 27), dtype=torch.float32, device=dev)
    cell = torch.zeros(nmix, dtype=torch.int32, device=dev)
    sg = torch.zeros(nmix, dtype=torch.int8, device=dev)
    ctx.mlp_stencils(c0, xs, cell, sg)
    y = torch.zeros(nmix, dtype=torch.float32, device=dev)
    ctx.mlp_forward(Pd, xs, y)
    ctx.profile_start()
    for _ in range(5):
        ctx.mlp_forward(Pd, xs, y)
    fprof = ctx.profile_stop()
    nf, tf = fprof["k_mlp_infer"]
    fwd_ms = tf / nf
    # matrix-core work per sample: layer 1 as hi + lo (2 x 32 x 128), layer 2 (128 x 128), multiply-add = 2 flops
    mfma_flops = 2.0 * (2 * 32 * 128 + 128 * 128)
    alg_flops = 2.0 * (27 * 128 + 128 * 128 + 128)
    fwd_tflops = nmix * mfma_flops / (fwd_ms / 1e3) / 1e12
    rows["curvature"] = dict(
        tracer=0, mixed_cells=nmix,
        hf_ms=ms_hf, hf_mixed_cells_per_s=nmix / (ms_hf / 1e3),
        mlp_hf_ms=ms_comb, mlp_hf_mixed_cells_per_s=nmix / (ms_comb / 1e3),
        hf_kernel_ms=hf_kernel_ms, hf_kernel_cells_per_s=nmix / (hf_kernel_ms / 1e3),
        mlp_hf_kernel_ms=mlp_kernel_ms, mlp_hf_kernel_cells_per_s=nmix / (mlp_kernel_ms / 1e3),
        mlp_forward_ms=fwd_ms, mlp_forward_cells_per_s=nmix / (fwd_ms / 1e3),
        mlp_forward_mfma_tflops=fwd_tflops, mlp_forward_mfma_frac=fwd_tflops / BF16_PEAK_TFLOPS,
        mlp_forward_algorithmic_tflops=nmix * alg_flops / (fwd_ms / 1e3) / 1e12,
        kappa_lo=meta["kappa_lo"],
        kernels_ms={**{k: v[1] / v[0] for k, v in prof_hf.items()}, **{k: v[1] / v[0] for k, v in prof.items()}})
    log(f"curvature: HF {ms_hf:.2f} ms (kernel {hf_kernel_ms:.3f}), MLP+HF {ms_comb:.2f} ms (kernels "
        f"{mlp_kernel_ms:.3f}), forward alone {fwd_ms:.3f} ms ({fwd_tflops:.1f} TFLOP/s) on {nmix} mixed cells")
    del kap, st, xs, cell, sg, y
    # ---- surface-tension force of all tracers, curvature by height functions
    kap8 = torch.empty(c.shape, dtype=torch.float64, device=dev)
    st8 = torch.empty(c.shape, dtype=torch.uint8, device=dev)
    for t in range(ntr):
        ctx.curvature_hf(c[t], kap8[t], st8[t])
    del st8
    fxyz = [torch.empty(tuple(c.shape[1:]), dtype=torch.float64, device=dev) for _ in range(3)]
    ctx.csf_force(c, kap8, 1.0, *fxyz)
    ms, _ = timed(torch, stream, lambda: ctx.csf_force(c, kap8, 1.0, *fxyz))
    csf_bytes = n3 * (16.0 * ntr + 24.0)  # every tracer's c and kappa read once, three face arrays written
    rows["csf_force"] = dict(ms=ms, cells_per_s=n3 / (ms / 1e3), algorithmic_bytes=csf_bytes,
                             achieved_gbs=csf_bytes / (ms / 1e3) / 1e9,
                             hbm_frac=csf_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS)
    log(f"csf_force: {ms:.2f} ms, {rows['csf_force']['achieved_gbs']:.0f} GB/s of the method's bytes")
    del kap8, fxyz
    # ---- training step throughput (batch 4096)
    bsz = 4096
    rng = synth.Splitmix64(5)
    xt = torch.from_numpy(rng.uniform(bsz * 27).astype(np.float32).reshape(bsz, 27)).to(dev)
    tt = torch.from_numpy((rng.uniform(bsz) * 0.5).astype(np.float32)).to(dev)
    Pt = torch.from_numpy(training.init_params(3)).to(dev)
    Mt = torch.zeros_like(Pt)
    Vt = torch.zeros_like(Pt)
    for s in range(1, 6):
        ctx.mlp_train_step(Pt, Mt, Vt, s, 1e-3, xt, tt)
    nst = 200
    ms, _ = timed(torch, stream, lambda: [ctx.mlp_train_step(Pt, Mt, Vt, 5 + s, 1e-3, xt, tt)
                                          for s in range(1, nst + 1)])
    rows["mlp_train_step"] = dict(batch=bsz, ms_per_step=ms / nst, samples_per_s=bsz * nst / (ms / 1e3))
    log(f"mlp training: {ms / nst:.3f} ms per step of {bsz}")
    return rows


def batched_bench(torch, ctx, stream, nsteps=10):
    """32 uneven boxes: one graph launch vs 32 plain launches."""
    from paper_2407_07463_amd import synth

    t0 = time.time()
    bb = synth.batch_boxes(32, workers=16)
    log(f"batched workload generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    boxes = [tuple(torch.from_numpy(b[k]).to(dev) for k in ("c", "sx", "sy", "sz")) for b in bb]
    cells = sum(b["c"].size for b in bb)
    tuning, tune_ms = ctx.autotune_batched(boxes, nsteps=1)
    ctx.advect_batched(boxes, step0=0, nsteps=nsteps, tuning=tuning)  # builds the graph
    ms_graph, _ = timed(torch, stream, lambda: ctx.advect_batched(boxes, step0=0, nsteps=nsteps, tuning=tuning))
    ms_plain, _ = timed(torch, stream, lambda: [ctx.advect(c, sx, sy, sz, step0=0, nsteps=nsteps)
                                                for c, sx, sy, sz in boxes])
    log(f"batched: graph {ms_graph / nsteps:.3f} ms/step, plain {ms_plain / nsteps:.3f} ms/step, tuning {tuning}")
    return dict(boxes=len(bb), tracer_cells=cells, steps=nsteps,
                sizes=[b["shape"][0] for b in bb], tracers=[b["ntracers"] for b in bb],
                tuning=dict(chunk=tuning[0], workgroups_per_cu=tuning[1]),
                graph_ms_per_step=ms_graph / nsteps, plain_ms_per_step=ms_plain / nsteps,
                graph_tracer_cell_steps_per_s=cells * nsteps / (ms_graph / 1e3),
                plain_tracer_cell_steps_per_s=cells * nsteps / (ms_plain / 1e3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="box size (cells per side)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="advection only")
    ap.add_argument("--cpu-sample-tracers", type=int, default=2)
    ap.add_argument("--pmc-pass", action="store_true", help="short run for rocprofv3 counters")
    ap.add_argument("--sweeps", choices=("single", "paired"), default="single",
                    help="run the sweeps one at a time (default, the faster form on this GPU) or in pairs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 2:
        args.steps += 1  # an even number of steps leaves the result in place (no final copy)

    import numpy as np
    import torch

    from paper_2407_07463_amd import profiling, synth, vofmt

    n = args.n
    t0 = time.time()
    w = synth.random_drops(n, 8, 0.3, 24.0, 0.1, 1.0, seed=synth.workload_seed(2), order=8, workers=16)
    ntr = w["ntracers"]
    log(f"workload generated in {time.time() - t0:.1f}s: {len(w['radii'])} drops, rms {w['rms']:.3f}")
    dev = torch.device("cuda:0")
    c = torch.from_numpy(w["c"]).to(dev)
    s = [torch.from_numpy(w[k]).to(dev) for k in ("sx", "sy", "sz")]
    ctx = vofmt.Context(0)
    ctx.set_advect_pairs(args.sweeps == "paired")
    smax = ctx.check_courant(*s)
    stream = torch.cuda.current_stream()
    n3 = n ** 3

    if args.pmc_pass:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # calibration: reads and writes COPY_BYTES
        ctx.advect(c, *s, step0=0, nsteps=2)
        # the surface-tension force of the advected tracers (curvature by height functions)
        kap8 = torch.empty(c.shape, dtype=torch.float64, device=dev)
        st8 = torch.empty(c.shape, dtype=torch.uint8, device=dev)
        for t in range(ntr):
            ctx.curvature_hf(c[t], kap8[t], st8[t])
        fxyz = [torch.empty(tuple(c.shape[1:]), dtype=torch.float64, device=dev) for _ in range(3)]
        for _ in range(2):
            ctx.csf_force(c, kap8, 1.0, *fxyz)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_pass": True, "copy_bytes": COPY_BYTES, "steps": 2, "csf_calls": 2}), flush=True)
        ctx.close()
        return

    # warmup
    ctx.advect(c, *s, step0=0, nsteps=max(args.warmup, 1) * 2)
    torch.cuda.synchronize()
    log("warmup done")

    # timed region 1: the throughput
    ms, _ = timed(torch, stream, lambda: ctx.advect(c, *s, step0=0, nsteps=args.steps))
    ms_step = ms / args.steps
    value = n3 * ntr * args.steps / (ms / 1e3)
    log(f"advection: {ms_step:.3f} ms/step, {value:.3e} tracer-cell-steps/s")

    # timed region 2: the same K steps with every launch timed by HIP events
    ctx.profile_start()
    ms2, _ = timed(torch, stream, lambda: ctx.advect(c, *s, step0=0, nsteps=args.steps))
    prof = ctx.profile_stop()
    kernels = {k: dict(launches=v[0], avg_ms=v[1] / v[0], total_ms=v[1]) for k, v in prof.items()}
    pair_names = [k for k in prof if k.startswith("k_pair<")]
    if pair_names:  # paired sweeps: the paired streaming pass over all tracers
        launches = sum(prof[k][0] for k in pair_names)
        total_ms = sum(prof[k][1] for k in pair_names)
        nbytes = sum(prof[k][0] * pair_bytes(n3, ntr, not k.endswith(",3>")) for k in pair_names)
        bytes_launch = nbytes / launches
        achieved = nbytes / (total_ms / 1e3) / 1e9
        kernel_desc = f"k_pair<A,B,N> (two sweeps of all {ntr} tracers in one pass; all axis pairs)"
        log(f"k_pair: {launches} launches, avg {total_ms / launches:.3f} ms, {achieved:.0f} GB/s "
            f"(profiled region {ms2 / args.steps:.3f} ms/step)")
        prefix, traffic_file = "k_pair<", TRAFFIC_FILE
    else:
        stream_names = [k for k in prof if k.startswith("k_stream<")]
        launches = sum(prof[k][0] for k in stream_names)
        total_ms = sum(prof[k][1] for k in stream_names)
        g = 4 if ntr >= 4 else ntr
        bytes_launch = stream_bytes(n3, g)
        achieved = bytes_launch / (total_ms / launches / 1e3) / 1e9
        kernel_desc = (f"k_stream<D,{g}> (streaming pass of {g} tracers; all axes; the x-sweep as "
                       f"k_stream_rows<{g}>); achieved counts the method's bytes per tracer-cell-sweep, "
                       f"actual_hbm_gbs the measured HBM bytes")
        log(f"k_stream: {launches} launches, avg {total_ms / launches:.3f} ms, {achieved:.0f} GB/s "
            f"(profiled region {ms2 / args.steps:.3f} ms/step)")
        prefix, traffic_file = ("k_stream<", "k_stream_rows<"), TRAFFIC_FILE_SINGLE

    traffic = None
    tr, sha = profiling.read_traffic(traffic_file)
    if tr and sha == profiling.advect_source_sha():
        vals = [v for k, v in tr.items() if k.startswith(prefix)]  # str.startswith takes a tuple too
        if vals:
            traffic = sum(vals) / len(vals)

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
        "step_model_gbs": step_model_bytes(n3, ntr) / (ms_step / 1e3) / 1e9,
        "step_model_frac": step_model_bytes(n3, ntr) / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "actual_hbm_gbs": (traffic / (total_ms / launches / 1e3) / 1e9) if traffic else None,
            "kernel": kernel_desc,
            "bytes_per_launch": bytes_launch,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
        "kernels": kernels,
    }

    if not args.no_rows:
        out["rows"] = rows_bench(torch, np, ctx, stream, c, w, n, ntr)
        del c, s
        torch.cuda.empty_cache()
        out["rows"]["batched_advection"] = batched_bench(torch, ctx, stream)

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
