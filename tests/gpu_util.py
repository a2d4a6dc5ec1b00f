"""Helpers for the GPU tests (test code only)."""
import os
import sys

import pytest


def require_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_07463_amd import vofmt

    if not os.path.exists(vofmt.LIB_PATH):
        raise RuntimeError("libvofmt.so is not built: the GPU tests need the HIP library")
    return torch


def note(msg):
    """Print (flushed) what the next GPU step is, so a failing run names its case."""
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def periodic_box(a, centre, half):
    """Extract a periodic sub-box a[..., z-half:z+half+1, y..., x...] around centre=(i,j,k)."""
    import numpy as np

    i, j, k = centre
    nz, ny, nx = a.shape[-3:]
    zi = (np.arange(k - half, k + half + 1)) % nz
    yi = (np.arange(j - half, j + half + 1)) % ny
    xi = (np.arange(i - half, i + half + 1)) % nx
    return a[..., zi[:, None, None], yi[None, :, None], xi[None, None, :]]
