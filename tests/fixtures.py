"""Shared test fixtures built from the paper's figures and from seeded inputs (test code only)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def near_contact_panels():
    """The two panels of the near-contact figure as character grids, row 0 first."""
    panels = {}
    cur = None
    with open(os.path.join(GOLDEN, "near_contact_figure.txt")) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                panels[cur] = []
            else:
                panels[cur].append(line)
    return panels


def panel_fields(rows, pad=(0, 0), nz=5):
    """Extrude a panel into periodic 3-D fields: (c_i, c_j), shape [2][nz][ny][nx].

    Occupied cells get 1.0. '1', '2', '*' belong to tracer i; 'j', '*' to tracer j.
    `pad` adds empty cells along x and y so that the periodic wrap does not join
    regions that the drawing separates."""
    nrow, ncol = len(rows), len(rows[0])
    ny, nx = nrow + pad[1], ncol + pad[0]
    c = np.zeros((2, nz, ny, nx))
    for r, line in enumerate(rows):
        for q, ch in enumerate(line):
            if ch in "12*":
                c[0, :, r, q] = 1.0
            if ch in "j*":
                c[1, :, r, q] = 1.0
    return c


def random_blobs(rng, shape, ntr, nblobs, rmin=1.0, rmax=2.5, value_noise=True):
    """Random ellipsoidal-ish blobs of occupied cells for labelling/recolouring tests."""
    nz, ny, nx = shape
    c = np.zeros((ntr,) + shape)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for _ in range(nblobs):
        t = rng.integers(ntr)
        ctr = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
        r = rng.uniform(rmin, rmax)
        dx = (xx - ctr[0] + nx / 2) % nx - nx / 2
        dy = (yy - ctr[1] + ny / 2) % ny - ny / 2
        dz = (zz - ctr[2] + nz / 2) % nz - nz / 2
        inside = dx * dx + dy * dy + dz * dz < r * r
        val = rng.uniform(0.05, 1.0, shape) if value_noise else np.ones(shape)
        c[t] = np.where(inside, np.maximum(c[t], val), c[t])
    return c
