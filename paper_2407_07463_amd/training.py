"""Training and evaluation of the learned curvature network (host driver).

The paper computes curvature with height functions; the network is an
addition of this package. This module prepares seeded training data and
drives the HIP kernels through the C ABI; every network computation (stencil
canonicalisation, forward, backward, Adam, combined curvature) runs on the GPU.

Data: bodies are ellipsoids (a share of them spheres) with smallest semi-axis
R log-uniform in [2, 40] cells, the other two R * U(1, 2), random rotation and
a sub-cell random centre, in their own periodic box; exact volume fractions
come from the seeded generator. Every interface cell -- a mixed cell with
min(c, 1 - c) >= 1e-6; the rest is round-off dust of the fraction quadrature
whose stencil holds no interface -- gives one sample: its
canonical 3x3x3 stencil and the target sign * kappa*Delta, where kappa is the
sum of the principal curvatures of the ellipsoid at the surface point closest
to the cell centre (positive for a convex body filled with c = 1). For the
ellipsoid {x : x^T Q x = 1} with Q = diag(1/a_i^2) in its principal frame,
   kappa(x) = (|Q x|^2 tr Q - x^T Q^3 x) / |Q x|^3,
and the closest point to p is x_i = a_i^2 p_i / (a_i^2 + lam), where lam is
the root of sum_i a_i^2 p_i^2 / (a_i^2 + lam)^2 = 1, found by bisection.

Usage: python -m paper_2407_07463_amd.training --out DIR
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import synth

NPARAMS = 20868
OFF = dict(W1=0, b1=4096, W2=4224, b2=20608, W3=20736, b3=20864)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "curvature_mlp")
C_EPS = 1e-6  # interface cells: min(c, 1 - c) >= C_EPS


# ------------------------------------------------------------------ geometry of the targets

def ellipsoid_closest_kappa(p, axes):
    """Mean-curvature sum at the surface point of the ellipsoid with semi-axes
    `axes` (principal frame, centred at 0) closest to each point p[n][3]."""
    p = np.asarray(p, dtype=np.float64)
    a2 = np.asarray(axes, dtype=np.float64) ** 2
    amin2 = a2.min()
    amax = math.sqrt(a2.max())

    def f(lam):
        return np.sum(a2 * p ** 2 / (a2 + lam[:, None]) ** 2, axis=1) - 1.0

    lo = np.full(len(p), -amin2 * (1.0 - 1e-15))
    hi = np.linalg.norm(p, axis=1) * amax + 1e-9
    # f decreases on (-amin^2, inf); a root below lo only for points at the centre (never mixed)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        pos = f(mid) > 0.0
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
    lam = 0.5 * (lo + hi)
    x = a2 * p / (a2 + lam[:, None])
    q = x / a2                    # Q x
    q2 = np.sum(q * q, axis=1)    # |Q x|^2
    trq = np.sum(1.0 / a2)
    xq3x = np.sum(x * x / a2 ** 3, axis=1)
    return (q2 * trq - xq3x) / q2 ** 1.5


# ------------------------------------------------------------------ data

def _body(rng, rmin, rmax, sphere_share):
    R = rmin * (rmax / rmin) ** rng.uniform(1)[0]
    if rng.uniform(1)[0] < sphere_share:
        axes = np.array([R, R, R])
        rot = np.eye(3)
    else:
        axes = np.array([R, R * (1.0 + rng.uniform(1)[0]), R * (1.0 + rng.uniform(1)[0])])
        rot = synth.random_rotation(rng)
    return axes, rot


def body_samples(ctx, axes, rot, rng, cap=None, dev="cuda:0"):
    """Canonical stencils, signs, cells and targets of every mixed cell of one body."""
    import torch

    L = int(2 * max(axes) + 8)
    ctr = np.array([L / 2.0] * 3) + rng.uniform(3)
    Q = synth.ellipsoid_matrix(axes, rot)
    c = synth.fill_ellipsoids((L, L, L), 1, ctr[None], Q[None], [0])[0]
    cd = torch.from_numpy(c).to(dev)
    nmix = int(((cd > 1e-12) & (cd < 1 - 1e-12)).sum().item())  # interface cells
    xs = torch.zeros((max(nmix, 1), 27), dtype=torch.float32, device=dev)
    cell = torch.zeros(max(nmix, 1), dtype=torch.int32, device=dev)
    sg = torch.zeros(max(nmix, 1), dtype=torch.int8, device=dev)
    n = ctx.mlp_stencils(cd, xs, cell, sg)
    assert n == nmix
    cell_all = cell[:n].cpu().numpy().astype(np.int64)
    cv = c.ravel()[cell_all]
    keep = np.flatnonzero(np.minimum(cv, 1.0 - cv) >= C_EPS)
    if cap is not None and len(keep) > cap:
        keep = np.sort(keep[np.argsort(rng.uniform(len(keep)))[:cap]])
    cell_h = cell_all[keep]
    sg_h = sg[:n].cpu().numpy().astype(np.float64)[keep]
    k, j, i = cell_h // (L * L), (cell_h // L) % L, cell_h % L
    p = np.stack([i + 0.5, j + 0.5, k + 0.5], axis=1) - ctr
    kap = ellipsoid_closest_kappa(p @ rot, axes)  # rotate into the principal frame
    return xs[:n][torch.from_numpy(keep).to(dev)], (sg_h * kap).astype(np.float32)


def make_dataset(ctx, nbodies, seed, rmin=2.0, rmax=40.0, sphere_share=0.3, cap=1500, log=None):
    import torch

    rng = synth.Splitmix64(seed)
    xs, ts = [], []
    for b in range(nbodies):
        axes, rot = _body(rng, rmin, rmax, sphere_share)
        x, t = body_samples(ctx, axes, rot, rng, cap)
        xs.append(x)
        ts.append(t)
        if log and (b + 1) % 200 == 0:
            log(f"data: {b + 1}/{nbodies} bodies, {sum(len(t) for t in ts)} samples")
    return torch.cat(xs), torch.from_numpy(np.concatenate(ts)).to(xs[0].device)


# ------------------------------------------------------------------ training

def init_params(seed):
    rng = synth.Splitmix64(seed)
    P = np.zeros(NPARAMS, dtype=np.float32)
    P[OFF["W1"]:OFF["W1"] + 27 * 128] = rng.normal(27 * 128) * math.sqrt(2.0 / 27)
    P[OFF["W2"]:OFF["b2"]] = rng.normal(128 * 128) * math.sqrt(2.0 / 128)
    P[OFF["W3"]:OFF["b3"]] = rng.normal(128) * math.sqrt(1.0 / 128)
    return P


def train(ctx, x, t, steps, batch=4096, lr=1e-3, seed=1, log=None, log_every=2000):
    """Adam with cosine-decayed learning rate over seeded shuffled batches."""
    import torch

    dev = x.device
    P = torch.from_numpy(init_params(seed)).to(dev)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    n = x.shape[0]
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    perm = torch.randperm(n, generator=gen).to(dev)
    pos = 0
    hist = []
    for s in range(1, steps + 1):
        if pos + batch > n:
            perm = torch.randperm(n, generator=gen).to(dev)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        lr_s = 0.5 * lr * (1.0 + math.cos(math.pi * (s - 1) / steps))
        loss = ctx.mlp_train_step(P, M, V, s, lr_s, x[idx].contiguous(), t[idx].contiguous())
        if log and (s % log_every == 0 or s == 1):
            log(f"step {s}: loss {loss:.5f} lr {lr_s:.2e}")
            hist.append((s, loss))
    return P, hist


# ------------------------------------------------------------------ evaluation on spheres

def sphere_errors(ctx, params, kappa_lo, radii, per_radius=4, seed=7, dev="cuda:0"):
    """Relative errors against 2/R on every interface cell of spheres of each radius:
    height functions alone (on the cells where they are valid), the network
    alone, and the combination."""
    import torch

    rng = synth.Splitmix64(seed)
    rows = []
    for R in radii:
        e_hf, e_net, e_comb, n_all, n_hf = [], [], [], 0, 0
        for _ in range(per_radius):
            L = int(2 * R + 8)
            ctr = np.array([L / 2.0] * 3) + rng.uniform(3)
            c = synth.fill_spheres((L, L, L), 1, ctr[None], [R], [0])[0]
            cd = torch.from_numpy(c).to(dev)
            k_hf = torch.zeros(c.shape, dtype=torch.float64, device=dev)
            s_hf = torch.zeros(c.shape, dtype=torch.uint8, device=dev)
            ctx.curvature_hf(cd, k_hf, s_hf)
            k_c = torch.zeros_like(k_hf)
            s_c = torch.zeros_like(s_hf)
            ctx.curvature_mlp(cd, params, kappa_lo, k_c, s_c)
            k_n = torch.zeros_like(k_hf)
            s_n = torch.zeros_like(s_hf)
            ctx.curvature_mlp(cd, params, 0.0, k_n, s_n)
            mixed = np.minimum(c, 1.0 - c) >= C_EPS
            want = 2.0 / R
            khf, shf = k_hf.cpu().numpy()[mixed], s_hf.cpu().numpy()[mixed]
            valid = (shf >= 1) & (shf <= 3)
            e_hf.append((khf[valid] - want) / want)
            e_net.append((k_n.cpu().numpy()[mixed] - want) / want)
            e_comb.append((k_c.cpu().numpy()[mixed] - want) / want)
            n_all += int(mixed.sum())
            n_hf += int(valid.sum())
        row = dict(R=R, cells=n_all, hf_valid=n_hf / max(n_all, 1))
        for name, e in (("hf", e_hf), ("net", e_net), ("comb", e_comb)):
            e = np.concatenate(e)
            row[f"{name}_l2"] = float(np.sqrt(np.mean(e * e))) if len(e) else float("nan")
            row[f"{name}_linf"] = float(np.max(np.abs(e))) if len(e) else float("nan")
        rows.append(row)
    return rows


def tune_kappa_lo(ctx, params, grid, radii=(4, 6, 8, 12, 20, 40), seed=99):
    """kappa_lo minimising the worst combined L2 error over held-out spheres."""
    best = None
    for klo in grid:
        rows = sphere_errors(ctx, params, klo, radii, per_radius=2, seed=seed)
        worst = max(r["comb_l2"] for r in rows)
        if best is None or worst < best[1]:
            best = (klo, worst)
    return best


def load_weights(path=WEIGHTS):
    """(params FP32 numpy, metadata dict) of a trained network."""
    P = np.load(path + ".npy", allow_pickle=False)
    with open(path + ".json") as f:
        meta = json.load(f)
    assert P.dtype == np.float32 and P.shape == (NPARAMS,)
    return P, meta


def main(argv=None):
    import torch

    from . import vofmt

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--bodies", type=int, default=2400)
    ap.add_argument("--cap", type=int, default=1500)
    ap.add_argument("--steps", type=int, default=120000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=20240710)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[train] {msg}", flush=True)

    ctx = vofmt.Context(0)
    t0 = time.time()
    x, t = make_dataset(ctx, a.bodies, a.seed, cap=a.cap, log=log)
    log(f"dataset: {len(t)} samples in {time.time() - t0:.1f} s")
    t0 = time.time()
    P, hist = train(ctx, x, t, a.steps, a.batch, a.lr, seed=a.seed + 1, log=log)
    torch.cuda.synchronize()
    log(f"trained {a.steps} steps in {time.time() - t0:.1f} s")
    klo, worst = tune_kappa_lo(ctx, P, [0.0, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.45, 0.5, 0.7, 1.0, 2.0])
    log(f"kappa_lo = {klo} (worst held-out combined L2 {worst:.4f})")
    rows = sphere_errors(ctx, P, klo, [2, 3, 4, 6, 8, 12, 20, 40])
    for r in rows:
        log(" ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}" for k, v in r.items()))
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.save(a.out + ".npy", P.cpu().numpy())
    meta = dict(kappa_lo=klo, samples=int(len(t)), bodies=a.bodies, cap=a.cap, steps=a.steps, batch=a.batch,
                lr=a.lr, seed=a.seed, loss_history=hist, sphere_errors=rows)
    with open(a.out + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
