"""Seeded inputs for the tests of the learned curvature (test code only)."""
import numpy as np

import oracle
from paper_2407_07463_amd import synth

OFF = oracle.MLP_OFF
NP = oracle.MLP_NPARAMS


def random_params(seed, scale=1.0):
    """He-style random weights, padding inputs of layer 1 zero."""
    rng = synth.Splitmix64(seed)
    P = np.zeros(NP, dtype=np.float32)
    P[OFF["W1"]:OFF["b1"]] = (rng.normal(32 * 128) * scale * np.sqrt(2.0 / 27)).astype(np.float32)
    P[OFF["W1"] + 27 * 128:OFF["b1"]] = 0.0
    P[OFF["b1"]:OFF["W2"]] = (rng.normal(128) * 0.1).astype(np.float32)
    P[OFF["W2"]:OFF["b2"]] = (rng.normal(128 * 128) * scale * np.sqrt(2.0 / 128)).astype(np.float32)
    P[OFF["b2"]:OFF["W3"]] = (rng.normal(128) * 0.1).astype(np.float32)
    P[OFF["W3"]:OFF["b3"]] = (rng.normal(128) * scale * np.sqrt(1.0 / 128)).astype(np.float32)
    P[OFF["b3"]] = 0.05
    return P


def random_inputs(seed, n):
    rng = synth.Splitmix64(seed)
    return rng.uniform(n * 27).astype(np.float32).reshape(n, 27)


def sphere_field(R, seed, drop=True):
    """One sphere of radius R cells at a random sub-cell centre in a periodic box
    (a bubble, c -> 1 - c, when drop is False)."""
    rng = synth.Splitmix64(seed)
    L = int(2 * R + 8)
    ctr = np.array([L / 2.0] * 3) + rng.uniform(3)
    c = synth.fill_spheres((L, L, L), 1, ctr[None], [R], [0])[0]
    return c if drop else 1.0 - c


def block_at(c, k, j, i):
    return np.take(np.take(np.take(c, range(k - 1, k + 2), 0, mode="wrap"), range(j - 1, j + 2), 1, mode="wrap"),
                   range(i - 1, i + 2), 2, mode="wrap")


def canonical_inputs(c):
    """Oracle canonical stencils of every interface cell of c (more than 1e-12 inside (0, 1)), in
    linear cell order."""
    mixed = np.flatnonzero((c > 1e-12) & (c < 1.0 - 1e-12))
    nz, ny, nx = c.shape
    xs = np.zeros((len(mixed), 27), dtype=np.float32)
    sg = np.zeros(len(mixed), dtype=np.int8)
    for q, p in enumerate(mixed):
        k, j, i = p // (nx * ny), (p // nx) % ny, p % nx
        xs[q], sg[q] = oracle.canonical_stencil(block_at(c, k, j, i))
    return mixed.astype(np.int32), xs, sg
