#!/usr/bin/env python3
"""Benchmark of the multi-tracer PLIC-VoF hot path on one MI355X.

Workload (default): a 512^3 tri-periodic box with 8 FP64 tracer fields
holding ~5508 drops of diameter 24 cells (+-10%) at volume fraction 0.3,
placed by random sequential addition with a 1-cell gap, and a frozen random
solenoidal velocity (modes 1 <= |k| <= 8, E(k) ~ k^-5/3, rms 0.2 cells per
step, rise 0.1). All inputs are synthetic and seeded.

A step is one direction-split advection step of all tracers (three sweeps,
each a PLIC pass over the mixed cells and streaming passes over the fields).
After the warmup, K steps are timed `--runs` times with HIP events on the
stream the kernels run on, each run bracketed by device synchronisations;
`ms_per_step` and `value` come from the median run. `value` is the metric's
per-tracer rate: cell updates per second of one tracer field while all 8 are
advanced (n^3 * steps / t); the all-tracer rate is reported beside it.

`roofline` is that of the dominant kernel, the streaming pass (k_stream; the
x-sweep as k_stream_rows), from its launches timed with HIP events in a
further run of K steps: `achieved` = the method's bytes of one launch (17.17
B per tracer-cell-sweep at 8 tracers: read and write c, the face velocity
shared by the 8 tracers, 1/6 B of c > 0.5 bits) times the tracer-cells of the
launch, divided by its mean duration. `traffic` is the launch's HBM bytes
from the committed rocprofv3 counter summary when the advection sources have
not changed since. The end-to-end step against the same model (51.5 B per
tracer-cell-step) is `step_model_frac`.

The same line carries, under `rows`, the other steps of the path measured on
the advected field (labelling, moments, shapes, recolouring in both
near-contact modes, pair statistics with M, R, A and the densities, height-
function and learned curvature of every tracer with their agreement, the
surface-tension force, network training, the tracer count N(t) over the
256^3 workload and batched advection of 32 uneven boxes; labelling, moments,
shapes, recolouring, pair statistics and the force are the median of 5 timed
calls, their times in `runs_ms`), and under
`cpu_baseline` the CPU oracle timed on a bounded sample, multi- and
single-threaded.

--pmc-pass advect: a short run for the traffic counters (a plain copy of
1 GiB, the calibration kernel; 2 advection steps; two surface-tension force
evaluations). --pmc-pass mlp: the network kernels a few times each (forward
on given stencils, fused curvature, training steps at batch 262144). Each
prints one line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix cores
METRIC = "VoF cell-updates/s per tracer (FP64) at % HBM roofline; learned vs HF curvature cells/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_k_stream_drops512.txt")
MFMA_FILE = os.path.join(ROOT, "profiles", "mfma_mlp_kernels_drops512.txt")
COPY_BYTES = 1 << 30


def sweep_model_bytes(ntr: int) -> float:
    """The method's HBM bytes per tracer-cell-sweep: read and write c (16 B),
    the face velocity shared by the ntr tracers (8/ntr B), 1/6 B of c > 0.5
    bits (17.17 B at 8 tracers)."""
    return 16.0 + 8.0 / ntr + 1.0 / 6.0


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


def timed_median(torch, stream, fn, runs=5, prepare=None):
    """Median over `runs` timed calls of fn (each after an untimed prepare(), if given), the
    list of times, and the last call's result."""
    ts, r = [], None
    for _ in range(runs):
        if prepare is not None:
            prepare()
        ms, r = timed(torch, stream, fn)
        ts.append(ms)
    return statistics.median(ts), ts, r


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(cpu_model=model, nproc=avail, cpu_count=os.cpu_count())


def read_mfma_summary(path=MFMA_FILE):
    """{kernel: {MfmaUtil, MfmaFlopsBF16, ...}} from the committed counter summary, or {}."""
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            if not line.startswith("kernel = "):
                continue
            parts = [p.strip() for p in line.split("|")]
            name = parts[0][len("kernel = "):]
            vals = {}
            for p in parts[1:]:
                if " = " in p:
                    k, v = p.split(" = ", 1)
                    try:
                        vals[k] = float(v)
                    except ValueError:
                        vals[k] = v
            out[name] = vals
    return out


# ------------------------------------------------------------------ rows

def rows_bench(torch, np, ctx, stream, c, w, n, ntr):
    """Timings of the other steps of the path on the advected field."""
    from paper_2407_07463_amd import training

    dev = c.device
    rows = {}
    n3 = n ** 3
    # ---- labelling and moments
    lab = torch.zeros(c.shape, dtype=torch.int32, device=dev)
    ctx.label_drops(c, lab)  # warm
    ms, runs, nd = timed_median(torch, stream, lambda: ctx.label_drops(c, lab))
    D = int(nd.sum())
    lab_bytes = n3 * ntr * (8.0 + 4.0)  # read c, write the label
    rows["label_drops"] = dict(ms=ms, runs_ms=runs, drops=D, cells_per_s=n3 * ntr / (ms / 1e3),
                               hbm_frac=lab_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS)
    log(f"label_drops: {ms:.2f} ms, {D} drops")
    vol = torch.zeros(D, dtype=torch.float64, device=dev)
    xyz = torch.zeros((D, 3), dtype=torch.float64, device=dev)
    ctx.drop_moments(c, lab, nd, vol, xyz)
    ms, runs, _ = timed_median(torch, stream, lambda: ctx.drop_moments(c, lab, nd, vol, xyz))
    rows["drop_moments"] = dict(ms=ms, runs_ms=runs)
    log(f"drop_moments: {ms:.2f} ms")
    # ---- drop shapes: inertia tensors, aspect ratios and mean velocities
    sv = [torch.from_numpy(w[k]).to(dev) for k in ("sx", "sy", "sz")]
    inertia = torch.zeros((D, 6), dtype=torch.float64, device=dev)
    chi = torch.zeros(D, dtype=torch.float64, device=dev)
    velo = torch.zeros((D, 3), dtype=torch.float64, device=dev)
    ctx.drop_shapes(c, lab, nd, inertia, chi, sv, velo)
    ms, runs, _ = timed_median(torch, stream, lambda: ctx.drop_shapes(c, lab, nd, inertia, chi, sv, velo))
    rows["drop_shapes"] = dict(ms=ms, runs_ms=runs, drops=D, chi_mean=float(chi.mean().item()),
                               chi_max=float(chi.max().item()))
    log(f"drop_shapes: {ms:.2f} ms, mean aspect ratio {rows['drop_shapes']['chi_mean']:.4f}")
    ctx.drop_moments_shapes(c, lab, nd, vol, xyz, inertia, chi, sv, velo)
    ms, runs, _ = timed_median(torch, stream,
                               lambda: ctx.drop_moments_shapes(c, lab, nd, vol, xyz, inertia, chi, sv, velo))
    rows["drop_moments_shapes"] = dict(ms=ms, runs_ms=runs, separate_ms=rows["drop_moments"]["ms"] + rows["drop_shapes"]["ms"])
    log(f"drop_moments_shapes: {ms:.2f} ms (separately {rows['drop_moments_shapes']['separate_ms']:.2f} ms)")
    del sv, inertia, chi, velo
    # ---- recolouring in both near-contact modes (each call on a fresh copy with room for 2N
    # tracers, made outside the timed region); one untimed call first (it sizes the scratch
    # buffers), then the timed calls
    cap = 2 * ntr
    cr = torch.zeros((cap,) + tuple(c.shape[1:]), dtype=torch.float64, device=dev)
    newt = torch.zeros(max(D, 1), dtype=torch.int32, device=dev)

    def fresh():
        cr.zero_()
        cr[:ntr].copy_(c)

    for mode in ("tau", "stencil"):
        if mode == "tau":
            fn = lambda: ctx.recolor_tracers(cr, ntr, lab, nd, 1.5, newt)
        else:
            fn = lambda: ctx.recolor_tracers_stencil(cr, ntr, lab, nd, newt)
        fresh()
        fn()
        ms, runs, (ntr2, moved) = timed_median(torch, stream, fn, prepare=fresh)
        key = "recolor_tracers" if mode == "tau" else "recolor_tracers_stencil"
        rows[key] = dict(ms=ms, runs_ms=runs, tracers_after=ntr2, drops_moved=moved,
                         criterion="distance gap 1.5 cells" if mode == "tau" else "5x5x5 stencil, Steps 1-3")
        log(f"{key}: {ms:.2f} ms, {moved} drops moved, {ntr2} tracers")
    del cr, newt
    # ---- nearest-particle pair statistics: 64 x 32 histogram over r < 4 d, M, R, A, densities
    nr, nth = 64, 32
    r_edges = np.arange(nr + 1) * (4 * 24.0 / nr)
    th_edges = np.arange(nth + 1) * (math.pi / nth)
    r2e, ce = r_edges ** 2, np.cos(th_edges)
    idx = torch.zeros(D, dtype=torch.int32, device=dev)
    ties = torch.zeros(D, dtype=torch.int32, device=dev)
    hist = torch.zeros(nr * nth + 1, dtype=torch.int64, device=dev)
    M = torch.zeros(3, dtype=torch.float64, device=dev)
    R = torch.zeros(9, dtype=torch.float64, device=dev)
    A = torch.zeros(9, dtype=torch.float64, device=dev)
    box = [float(n)] * 3
    ctx.nearest_pair_stats(xyz, box, 2, r2e, ce, idx, ties, hist, M, R, A)
    ms, _, _ = timed_median(torch, stream,
                            lambda: ctx.nearest_pair_stats(xyz, box, 2, r2e, ce, idx, ties, hist, M, R, A))
    P = torch.zeros(nr * nth, dtype=torch.float64, device=dev)
    Pr = torch.zeros(nr, dtype=torch.float64, device=dev)
    ms_pdf, _, _ = timed_median(torch, stream, lambda: ctx.pair_pdfs(r_edges, th_edges, hist, D, P, Pr))
    ms_na = None
    if D <= 8192:
        ctx.nearest_pair_stats_noalloc(xyz, box, 2, r2e, ce, idx, ties, hist, M, R, A)
        ms_na, _, _ = timed_median(
            torch, stream, lambda: ctx.nearest_pair_stats_noalloc(xyz, box, 2, r2e, ce, idx, ties, hist, M, R, A))
    Rh = R.cpu().numpy().reshape(3, 3)
    Ah = A.cpu().numpy().reshape(3, 3)
    Prh = Pr.cpu().numpy()
    rc = 0.5 * (r_edges[1:] + r_edges[:-1])
    rows["nearest_pair_stats"] = dict(
        ms=ms, pdfs_ms=ms_pdf, noalloc_ms=ms_na, drops=D, histogram=[nr, nth], vertical_axis="z",
        M=[float(v) for v in M.cpu().numpy()], R=[[float(v) for v in r] for r in Rh],
        A=[[float(v) for v in r] for r in Ah], trace_R=float(np.trace(Rh)),
        A_zz_over_trR=float(Ah[2, 2] / np.trace(Rh)),
        P_r_peak_r_over_d=float(rc[int(np.argmax(Prh))] / 24.0))
    log(f"nearest_pair_stats: {ms:.2f} ms (+ densities {ms_pdf:.3f} ms); tr R {np.trace(Rh):.1f}, "
        f"A_zz/tr R {Ah[2, 2] / np.trace(Rh):+.4f}")
    del lab
    # ---- curvature: height functions vs network + fallback, tracer 0 in detail, then every tracer
    P_w, meta = training.load_weights()
    Pd = torch.from_numpy(P_w).to(dev)
    c0 = c[0].contiguous()
    kap = torch.zeros(c0.shape, dtype=torch.float64, device=dev)
    st = torch.zeros(c0.shape, dtype=torch.uint8, device=dev)
    nmix = int(((c0 > 1e-12) & (c0 < 1 - 1e-12)).sum().item())  # interface cells
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
    alg_flops = 2.0 * (27 * 128 + 128 * 128 + 128)  # 41,216 per sample (the model's own product)
    mfma_flops = 2.0 * (2 * 32 * 128 + 128 * 128)   # issued: layer 1 as hi + lo over 32 padded inputs, layer 2
    fwd_alg_tflops = nmix * alg_flops / (fwd_ms / 1e3) / 1e12
    del xs, cell, sg, y
    # every tracer: mixed cells of the whole field, both estimators, their agreement where HF is valid
    tot_mixed = 0
    t_hf = t_mlp = 0.0
    diffs = []
    kh = torch.empty(c0.shape, dtype=torch.float64, device=dev)
    sh = torch.empty(c0.shape, dtype=torch.uint8, device=dev)
    for t in range(ntr):
        ct = c[t].contiguous()
        ms1, _ = timed(torch, stream, lambda: ctx.curvature_hf(ct, kh, sh))
        ms2, nm = timed(torch, stream, lambda: ctx.curvature_mlp(ct, Pd, meta["kappa_lo"], kap, st))
        t_hf += ms1
        t_mlp += ms2
        tot_mixed += nm
        valid = (sh >= 1) & (sh <= 3) & (st == 8)  # HF valid and the network's own value kept
        d = (kap[valid] - kh[valid]).abs() / kh[valid].abs().clamp_min(1e-3)
        diffs.append(d.cpu().numpy())
    diffs = np.concatenate(diffs) if diffs else np.zeros(1)
    rows["curvature"] = dict(
        tracer=0, mixed_cells=nmix,
        hf_ms=ms_hf, hf_mixed_cells_per_s=nmix / (ms_hf / 1e3),
        mlp_hf_ms=ms_comb, mlp_hf_mixed_cells_per_s=nmix / (ms_comb / 1e3),
        hf_kernel_ms=hf_kernel_ms, hf_kernel_cells_per_s=nmix / (hf_kernel_ms / 1e3),
        mlp_hf_kernel_ms=mlp_kernel_ms, mlp_hf_kernel_cells_per_s=nmix / (mlp_kernel_ms / 1e3),
        learned_over_hf_kernel_speedup=hf_kernel_ms / mlp_kernel_ms,
        mlp_forward_ms=fwd_ms, mlp_forward_cells_per_s=nmix / (fwd_ms / 1e3),
        mlp_forward_algorithmic_tflops=fwd_alg_tflops,
        mlp_forward_issued_mfma_tflops=nmix * mfma_flops / (fwd_ms / 1e3) / 1e12,
        mlp_forward_frac_of_bf16_peak=fwd_alg_tflops / BF16_PEAK_TFLOPS,
        kappa_lo=meta["kappa_lo"],
        kernels_ms={**{k: v[1] / v[0] for k, v in prof_hf.items()}, **{k: v[1] / v[0] for k, v in prof.items()}},
        all_tracers=dict(mixed_cells=tot_mixed, hf_ms=t_hf, mlp_hf_ms=t_mlp,
                         hf_mixed_cells_per_s=tot_mixed / (t_hf / 1e3),
                         mlp_hf_mixed_cells_per_s=tot_mixed / (t_mlp / 1e3),
                         cells_compared=int(diffs.size),
                         mlp_vs_hf_rel_diff_median=float(np.median(diffs)),
                         mlp_vs_hf_rel_diff_p90=float(np.percentile(diffs, 90)),
                         mlp_vs_hf_rel_diff_mean=float(np.mean(diffs))))
    mf = read_mfma_summary()
    if mf:
        rows["curvature"]["mfma_counters"] = mf
    log(f"curvature: HF {ms_hf:.2f} ms (kernel {hf_kernel_ms:.3f}), MLP+HF {ms_comb:.2f} ms (kernels "
        f"{mlp_kernel_ms:.3f}), forward alone {fwd_ms:.3f} ms ({fwd_alg_tflops:.1f} TFLOP/s) on {nmix} mixed cells; "
        f"all tracers {tot_mixed} mixed cells, MLP vs HF median rel. diff {np.median(diffs):.4f}")
    del kap, st, kh, sh
    # ---- surface-tension force of all tracers, curvature by height functions
    kap8 = torch.empty(c.shape, dtype=torch.float64, device=dev)
    st8 = torch.empty(c.shape, dtype=torch.uint8, device=dev)
    for t in range(ntr):
        ctx.curvature_hf(c[t], kap8[t], st8[t])
    del st8
    fxyz = [torch.empty(tuple(c.shape[1:]), dtype=torch.float64, device=dev) for _ in range(3)]
    ctx.csf_force(c, kap8, 1.0, *fxyz)
    ms, runs, _ = timed_median(torch, stream, lambda: ctx.csf_force(c, kap8, 1.0, *fxyz))
    csf_bytes = n3 * (16.0 * ntr + 24.0)  # every tracer's c and kappa read once, three face arrays written
    rows["csf_force"] = dict(ms=ms, runs_ms=runs, cells_per_s=n3 / (ms / 1e3), algorithmic_bytes=csf_bytes,
                             achieved_gbs=csf_bytes / (ms / 1e3) / 1e9,
                             hbm_frac=csf_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS)
    log(f"csf_force: {ms:.2f} ms, {rows['csf_force']['achieved_gbs']:.0f} GB/s of the method's bytes")
    del kap8, fxyz
    # ---- training step throughput (batch 4096)
    from paper_2407_07463_amd import synth

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


def tracer_count_bench(torch, ctx, stream):
    """N(t) over the 256^3 workload: 200 steps, reassignment every 10, both near-contact modes."""
    from paper_2407_07463_amd import synth, tracer_count

    t0 = time.time()
    w = synth.drops256(workers=16)
    log(f"drops256 generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ntr = int(w["c"].shape[0])
    s = [torch.from_numpy(w[k]).to(dev) for k in ("sx", "sy", "sz")]
    out = {}
    for mode in ("tau", "stencil"):
        c = torch.zeros((24,) + tuple(w["c"].shape[1:]), dtype=torch.float64, device=dev)
        c[:ntr].copy_(torch.from_numpy(w["c"]))
        ms, (N, recs) = timed(torch, stream, lambda: tracer_count.run(ctx, c, *s, ntr, 200, 10, mode, 1.5))
        out[mode] = dict(ms_total=ms, steps=200, every=10, n_of_t=[[r["step"], r["ntracers"]] for r in recs],
                         moved_total=int(sum(r["moved"] for r in recs)),
                         retired_total=int(sum(r["retired"] for r in recs)), final_ntracers=N)
        log(f"tracer count ({mode}): N from {recs[0]['ntracers']} to {N} in 200 steps, {ms:.0f} ms")
        del c
    return out


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


def cpu_baseline(w, n, ntr):
    """The oracle as it stands, on the GPU machine's host: the whole workload's 8 tracers for one
    step with every thread the process may use, then one tracer for one step on one thread."""
    import numpy as np

    import oracle

    info = cpu_info()
    threads = oracle.num_threads()
    log(f"cpu baseline: oracle, {ntr} tracers x 1 step on {threads} threads ({info['cpu_model']})")
    t1 = time.time()
    oracle.advect(w["c"], w["sx"], w["sy"], w["sz"], 0, 1)
    dt_multi = time.time() - t1
    log(f"cpu baseline: 1 tracer x 1 step on 1 thread")
    oracle.set_num_threads(1)
    t1 = time.time()
    oracle.advect(np.ascontiguousarray(w["c"][:1]), w["sx"], w["sy"], w["sz"], 0, 1)
    dt_single = time.time() - t1
    oracle.set_num_threads(threads)
    n3 = n ** 3
    # per-tracer rate: one tracer field's cell updates per second while all ntr are advanced
    return {
        "value": n3 * 1 / dt_multi,
        "unit": "cell-updates/s per tracer",
        "cores": threads,
        "kind": "oracle",
        "sample": f"oracle advection of all {ntr} tracer fields of the {n}^3 workload for 1 step "
                  f"({dt_multi:.1f} s on {threads} threads); single thread: 1 tracer, 1 step ({dt_single:.1f} s)",
        "single_thread_value": n3 / (dt_single * ntr),
        "single_thread_tracer_cell_steps_per_s": n3 / dt_single,
        "tracer_cell_steps_per_s": n3 * ntr / dt_multi,
        "c3_100_steps_extrapolated_s": dt_multi * 100,
        **info,
    }


def pmc_pass(torch, np, ctx, c, s, ntr, which):
    dev = c.device
    if which == "advect":
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # calibration: reads and writes COPY_BYTES
        ctx.advect(c, *s, step0=0, nsteps=2)
        kap8 = torch.empty(c.shape, dtype=torch.float64, device=dev)
        st8 = torch.empty(c.shape, dtype=torch.uint8, device=dev)
        for t in range(ntr):
            ctx.curvature_hf(c[t], kap8[t], st8[t])
        fxyz = [torch.empty(tuple(c.shape[1:]), dtype=torch.float64, device=dev) for _ in range(3)]
        for _ in range(2):
            ctx.csf_force(c, kap8, 1.0, *fxyz)
        torch.cuda.synchronize()
        return {"pmc_pass": "advect", "copy_bytes": COPY_BYTES, "steps": 2, "csf_calls": 2}
    from paper_2407_07463_amd import synth, training

    P_w, meta = training.load_weights()
    Pd = torch.from_numpy(P_w).to(dev)
    ctx.advect(c, *s, step0=0, nsteps=2)
    c0 = c[0].contiguous()
    nmix = int(((c0 > 1e-12) & (c0 < 1 - 1e-12)).sum().item())  # interface cells
    xs = torch.zeros((nmix, 27), dtype=torch.float32, device=dev)
    cell = torch.zeros(nmix, dtype=torch.int32, device=dev)
    sg = torch.zeros(nmix, dtype=torch.int8, device=dev)
    ctx.mlp_stencils(c0, xs, cell, sg)
    y = torch.zeros(nmix, dtype=torch.float32, device=dev)
    kap = torch.zeros(c0.shape, dtype=torch.float64, device=dev)
    st = torch.zeros(c0.shape, dtype=torch.uint8, device=dev)
    for _ in range(3):
        ctx.mlp_forward(Pd, xs, y)
        ctx.curvature_mlp(c0, Pd, meta["kappa_lo"], kap, st)
    bsz = 262144  # 4096 tiles: the training kernels fill the chip (the training row times batch 4096)
    rng = synth.Splitmix64(5)
    xt = torch.from_numpy(rng.uniform(bsz * 27).astype(np.float32).reshape(bsz, 27)).to(dev)
    tt = torch.from_numpy((rng.uniform(bsz) * 0.5).astype(np.float32)).to(dev)
    Pt = torch.from_numpy(training.init_params(3)).to(dev)
    Mt, Vt = torch.zeros_like(Pt), torch.zeros_like(Pt)
    for k in range(1, 4):
        ctx.mlp_train_step(Pt, Mt, Vt, k, 1e-3, xt, tt)
    torch.cuda.synchronize()
    return {"pmc_pass": "mlp", "mixed_cells": nmix, "forward_calls": 3, "fused_calls": 3, "train_steps": 3,
            "train_batch": bsz}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--runs", type=int, default=5, help="timed runs of --steps steps; the median is reported")
    ap.add_argument("--n", type=int, default=512, help="box size (cells per side)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="advection only")
    ap.add_argument("--pmc-pass", choices=("advect", "mlp"), default=None,
                    help="short run for rocprofv3 counters")
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
    smax = ctx.check_courant(*s)
    stream = torch.cuda.current_stream()
    n3 = n ** 3

    if args.pmc_pass:
        res = pmc_pass(torch, np, ctx, c, s, ntr, args.pmc_pass)
        print(json.dumps(res), flush=True)
        ctx.close()
        return

    # warmup
    ctx.advect(c, *s, step0=0, nsteps=max(args.warmup, 1))
    torch.cuda.synchronize()
    g = max(args.warmup, 1)
    log("warmup done")

    # timed runs: K steps each, bracketed by synchronisations; the median is reported
    run_ms = []
    for _ in range(args.runs):
        ms, _ = timed(torch, stream, lambda: ctx.advect(c, *s, step0=g, nsteps=args.steps))
        g += args.steps
        run_ms.append(ms)
    ms_med = statistics.median(run_ms)
    ms_step = ms_med / args.steps
    value = n3 * args.steps / (ms_med / 1e3)  # cell updates per second of one tracer field (all 8 advanced)
    log(f"advection: {ms_step:.3f} ms/step (runs {', '.join(f'{m / args.steps:.3f}' for m in run_ms)}), "
        f"{value:.3e} cell-updates/s per tracer")

    # one more run of K steps with every launch timed by HIP events
    ctx.profile_start()
    ms2, _ = timed(torch, stream, lambda: ctx.advect(c, *s, step0=g, nsteps=args.steps))
    prof = ctx.profile_stop()
    g += args.steps
    kernels = {k: dict(launches=v[0], avg_ms=v[1] / v[0], total_ms=v[1]) for k, v in prof.items()}
    stream_names = [k for k in prof if k.startswith("k_stream<")]
    launches = sum(prof[k][0] for k in stream_names)
    total_ms = sum(prof[k][1] for k in stream_names)
    # tracers per streaming launch: every full group of 4 in one launch
    gsz = 4 if ntr >= 4 else ntr  # tracers per group (template argument)
    tpl = 4 * (ntr // 4) if ntr >= 4 else ntr
    bytes_launch = sweep_model_bytes(ntr) * tpl * n3
    avg_launch_s = total_ms / launches / 1e3
    achieved = bytes_launch / avg_launch_s / 1e9
    log(f"k_stream: {launches} launches, avg {1e3 * avg_launch_s:.3f} ms, {achieved:.0f} GB/s of the method's "
        f"bytes (profiled run {ms2 / args.steps:.3f} ms/step)")
    traffic = None
    tr, sha = profiling.read_traffic(TRAFFIC_FILE)
    if tr and sha == profiling.advect_source_sha():
        vals = [v for k, v in tr.items() if k.startswith(("k_stream<", "k_stream_rows<"))]
        if vals:
            traffic = sum(vals) / len(vals)
    step_bytes = 3.0 * sweep_model_bytes(ntr) * ntr * n3  # 51.5 B per tracer-cell-step at 8 tracers

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s per tracer",
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
        "runs_ms_per_step": [m / args.steps for m in run_ms],
        "all_tracer_cell_steps_per_s": value * ntr,
        "step_model_bytes_per_tracer_cell_step": 3.0 * sweep_model_bytes(ntr),
        "step_model_gbs": step_bytes / (ms_step / 1e3) / 1e9,
        "step_model_frac": step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"k_stream<D,{gsz}> / k_stream_rows<{gsz}> (streaming pass of {tpl} tracers in groups of {gsz}, all axes)",
            "bytes_per_launch": bytes_launch,
            "bytes_model": f"{sweep_model_bytes(ntr):.3f} B per tracer-cell-sweep x {tpl} x n^3",
            "avg_launch_ms": 1e3 * avg_launch_s,
            "actual_hbm_gbs": (traffic / avg_launch_s / 1e9) if traffic else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
        "kernels": kernels,
    }

    if not args.no_rows:
        out["rows"] = rows_bench(torch, np, ctx, stream, c, w, n, ntr)
        del c, s
        torch.cuda.empty_cache()
        out["rows"]["tracer_count_drops256"] = tracer_count_bench(torch, ctx, stream)
        torch.cuda.empty_cache()
        out["rows"]["batched_advection"] = batched_bench(torch, ctx, stream)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, n, ntr)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
