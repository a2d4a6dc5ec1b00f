"""GPU parity of the multi-tracer surface-tension force on the cell faces
against the CPU FP64 oracle.

Bar: bit-exact. Both sides take every face term in the same operations and
order (difference, curvature mean or the defined side, product; tracers
summed in increasing order, then times gamma), so any difference is a bug.
"""
import numpy as np
import pytest

import oracle
from gpu_util import note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    from paper_2407_07463_amd import vofmt

    c = vofmt.Context(0)
    yield c
    c.close()
    del torch


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _inputs(shape, ntr, seed):
    rng = np.random.default_rng(seed)
    full = (ntr,) + tuple(shape)
    u = rng.uniform(size=full)
    c = np.where(u < 0.35, 0.0, np.where(u < 0.6, 1.0, rng.uniform(size=full)))
    kap = np.where(rng.uniform(size=full) < 0.5, rng.normal(size=full), np.nan)
    return c, kap


def _gpu_force(ctx, c, kap, gamma):
    import torch

    shape = c.shape[-3:]
    f = [torch.full(shape, float("nan"), dtype=torch.float64, device="cuda:0") for _ in range(3)]
    ctx.csf_force(_dev(c), _dev(kap), gamma, *f)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in f]


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.mark.parametrize("shape,ntr", [((5, 7, 9), 1), ((17, 33, 130), 3), ((20, 6, 64), 8), ((9, 13, 70), 9),
                                       ((6, 5, 129), 13), ((1, 1, 5), 2), ((16, 1, 70), 4), ((3, 40, 1), 5)])
def test_random_fields(ctx, shape, ntr):
    c, kap = _inputs(shape, ntr, sum(shape) * 31 + ntr)
    gamma = 0.73
    note(f"csf force shape={shape} ntr={ntr}")
    g = _gpu_force(ctx, c, kap, gamma)
    o = oracle.csf_force(c, kap, gamma)
    for d in range(3):
        assert np.array_equal(_bits(g[d]), _bits(o[d])), d


def test_sphere_with_height_function_curvature(ctx):
    from paper_2407_07463_amd import synth

    c = synth.fill_spheres((40, 40, 40), 2, [(20.3, 19.6, 20.2), (5.0, 31.0, 9.5)], [9.0, 4.0], [0, 1], order=8)
    kap = np.stack([oracle.curvature_hf(c[t])[0] for t in range(2)])
    note("csf force spheres with oracle curvature")
    g = _gpu_force(ctx, c, kap, 1.0)
    o = oracle.csf_force(c, kap, 1.0)
    for d in range(3):
        assert np.array_equal(_bits(g[d]), _bits(o[d])), d


def test_no_tracers_and_errors(ctx):
    import torch
    from paper_2407_07463_amd import vofmt

    note("csf force, no tracers and bad arguments")
    shape = (4, 5, 6)
    f = [torch.full(shape, float("nan"), dtype=torch.float64, device="cuda:0") for _ in range(3)]
    L = vofmt.load()
    rc = L.vofmt_csf_force(ctx.h, 6, 5, 4, 0, None, None, 2.0, *[vofmt._ptr(a) for a in f], vofmt._stream())
    torch.cuda.synchronize()
    assert rc == 0
    for a in f:
        assert np.array_equal(a.cpu().numpy(), np.zeros(shape))
    c, kap = _inputs(shape, 2, 1)
    tc, tk = _dev(c), _dev(kap)
    rc = L.vofmt_csf_force(ctx.h, 6, 5, 4, 2, vofmt._ptr(tc), vofmt._ptr(tk), float("inf"),
                           *[vofmt._ptr(a) for a in f], vofmt._stream())
    assert rc == vofmt.E_ARG
    rc = L.vofmt_csf_force(ctx.h, 6, 5, 4, 2, vofmt._ptr(tc), None, 1.0, *[vofmt._ptr(a) for a in f],
                           vofmt._stream())
    assert rc == vofmt.E_ARG
    rc = L.vofmt_csf_force(ctx.h, 0, 5, 4, 2, vofmt._ptr(tc), vofmt._ptr(tk), 1.0, *[vofmt._ptr(a) for a in f],
                           vofmt._stream())
    assert rc == vofmt.E_ARG
    with pytest.raises(ValueError):
        ctx.csf_force(tc, tk[:1], 1.0, *f)
