"""The number of tracers in use over time, N(t), as the paper reports it
(section "The no-coalescence.h algorithm": the tracers needed for the runs,
at most 3 at phi = 0.01 and 7 at phi = 0.2).

A host driver over the C ABI (every step runs in the library's kernels): the
fields are advected, and every `every` steps the drops are labelled,
reassigned so that no two drops in near contact share a tracer (distance
threshold or the literal stencil criterion), and tracers left without a
drop are retired. Each block logs one record: the global step, N(t), the
number of drops, the drops moved, the tracers retired and the volume their
dust carried.

    python -m paper_2407_07463_amd.tracer_count --workload drops256 --steps 200 --every 10

prints one JSON line per record.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def reassign(ctx, c, ntracers: int, mode: str = "tau", gap: float = 1.5):
    """Label, recolour and compact c[:ntracers] in place (c holds capacity fields).
    Returns (ntracers after, record)."""
    import torch

    if mode not in ("tau", "stencil"):
        raise ValueError("mode is 'tau' or 'stencil'")
    dev = c.device
    shape = tuple(c.shape[1:])
    lab = torch.empty((ntracers,) + shape, dtype=torch.int32, device=dev)
    nd = ctx.label_drops(c[:ntracers], lab)
    D = int(nd.sum())
    newt = torch.zeros(max(D, 1), dtype=torch.int32, device=dev)
    if mode == "tau":
        n_after, moved = ctx.recolor_tracers(c, ntracers, lab, nd, gap, newt)
    else:
        n_after, moved = ctx.recolor_tracers_stencil(c, ntracers, lab, nd, newt)
    del lab
    # drops per tracer after the moves; tracers left with none are retired
    per = np.bincount(newt[:D].cpu().numpy(), minlength=n_after)[:n_after] if D else np.zeros(n_after, np.int64)
    kept, new_index, discarded = ctx.compact_tracers(c, n_after, per.astype(np.int32))
    rec = dict(drops=D, moved=int(moved), tracers_before_compaction=int(n_after), retired=int(n_after - kept),
               discarded_volume=float(discarded))
    return int(kept), rec


def run(ctx, c, sx, sy, sz, ntracers: int, steps: int, every: int, mode: str = "tau", gap: float = 1.5,
        step0: int = 0, emit=None):
    """Advance c[:N] by `steps` steps with a reassignment before the first step and after every
    `every` steps. c: [capacity][nz][ny][nx] float64 on the GPU, N grows up to capacity.
    Returns (N at the end, records)."""
    if every < 1 or steps < 0 or not 1 <= ntracers <= int(c.shape[0]):
        raise ValueError("tracer_count.run: bad arguments")
    records = []
    N = ntracers
    g = step0
    end = step0 + steps
    while True:
        N, rec = reassign(ctx, c, N, mode, gap)
        rec = dict(step=g, ntracers=N, **rec)
        records.append(rec)
        if emit is not None:
            emit(rec)
        if g >= end:
            break
        k = min(every, end - g)
        ctx.advect(c[:N], sx, sy, sz, step0=g, nsteps=k)
        g += k
    return N, records


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=("spheres64", "drops256", "drops512"), default="drops256")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--mode", choices=("tau", "stencil"), default="tau")
    ap.add_argument("--gap", type=float, default=1.5)
    ap.add_argument("--capacity", type=int, default=16)
    args = ap.parse_args(argv)

    import torch

    from . import synth, vofmt

    make = getattr(synth, args.workload)
    w = make() if args.workload == "spheres64" else make(workers=16)
    dev = torch.device("cuda:0")
    ntr = int(w["c"].shape[0])
    c = torch.zeros((max(args.capacity, ntr),) + tuple(w["c"].shape[1:]), dtype=torch.float64, device=dev)
    c[:ntr].copy_(torch.from_numpy(w["c"]))
    s = [torch.from_numpy(w[k]).to(dev) for k in ("sx", "sy", "sz")]
    ctx = vofmt.Context(0)
    run(ctx, c, *s, ntr, args.steps, args.every, args.mode, args.gap,
        emit=lambda r: print(json.dumps(dict(workload=args.workload, mode=args.mode, **r)), flush=True))
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
