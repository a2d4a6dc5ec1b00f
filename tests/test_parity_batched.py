"""Batched advection: bit-identity with one plain vofmt_advect call per box
(itself checked against the CPU oracle), for every tuning, through the C ABI.

Boxes are uneven: edges not multiples of 64 or 4, 1-8 tracers (groups of 4,
2 and 1), odd and even sweep counts (the result copied back or not), several
step offsets (sweep orders), graph reuse on a repeated call, and 32 boxes of
the batched workload's size mix scaled down.
"""
import numpy as np
import pytest

import oracle
from gpu_util import note, require_gpu
from paper_2407_07463_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [((20, 24, 16), 3), ((17, 33, 70), 1), ((64, 64, 64), 5), ((36, 52, 40), 8), ((65, 9, 17), 2),
          ((20, 16, 129), 4), ((12, 10, 600), 2)]  # the last one splits its x-rows at chunk 8


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    from paper_2407_07463_amd import vofmt

    c = vofmt.Context(0)
    yield c
    c.close()
    del torch


def _box(shape, ntr, seed):
    nz, ny, nx = shape
    rng = synth.Splitmix64(seed)
    ndrops = 2 * ntr + 2
    R = 0.22 * min(shape)
    centres = rng.uniform(3 * ndrops).reshape(ndrops, 3) * np.array([nx, ny, nz])
    radii = R * (0.6 + 0.4 * rng.uniform(ndrops))
    c = synth.fill_spheres(shape, ntr, centres, radii, np.arange(ndrops) % ntr)
    np.minimum(c, 1.0, out=c)
    sx, sy, sz, _ = synth.fourier_velocity(shape, seed + 1, kmax=4, rms=0.15, rise=0.08)
    return c, sx, sy, sz


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _plain(ctx, boxes, step0, nsteps, calls=1):
    out = []
    for c, sx, sy, sz in boxes:
        t = _dev(c)
        for _ in range(calls):
            ctx.advect(t, _dev(sx), _dev(sy), _dev(sz), step0=step0, nsteps=nsteps)
        out.append(t)
    return out


@pytest.fixture(scope="module")
def boxes():
    return [_box(shape, ntr, 300 + i) for i, (shape, ntr) in enumerate(SHAPES)]


@pytest.mark.parametrize("tuning", [None, (16, 2), (64, 16), (8, 1), (32, 4)])
@pytest.mark.parametrize("step0,nsteps", [(0, 1), (1, 2), (5, 3)])
def test_bit_identical_to_plain(ctx, boxes, tuning, step0, nsteps):
    import torch

    note(f"batched tuning={tuning} step0={step0} nsteps={nsteps}")
    ref = _plain(ctx, boxes, step0, nsteps)
    dev = [(_dev(c), _dev(sx), _dev(sy), _dev(sz)) for c, sx, sy, sz in boxes]
    ctx.advect_batched(dev, step0=step0, nsteps=nsteps, tuning=tuning)
    torch.cuda.synchronize()
    for i, ((c, _, _, _), r) in enumerate(zip(dev, ref)):
        assert torch.equal(c, r), (i, SHAPES[i], float((c - r).abs().max()))


def test_matches_oracle(ctx, boxes):
    import torch

    dev = [(_dev(c), _dev(sx), _dev(sy), _dev(sz)) for c, sx, sy, sz in boxes[:3]]
    ctx.advect_batched(dev, step0=2, nsteps=2)
    torch.cuda.synchronize()
    for (c0, sx, sy, sz), (c, _, _, _) in zip(boxes[:3], dev):
        ref = oracle.advect(c0, sx, sy, sz, 2, 2)
        assert float(np.abs(c.cpu().numpy() - ref).max()) <= 1e-12


def test_long_rows_split_between_wavefronts(ctx):
    """x-rows longer than 64 * chunk cells are walked by several wavefronts."""
    box = _box((4, 6, 2113), 1, 404)
    note("plain advection 2113 x 6 x 4")
    c, sx, sy, sz = box
    t = _dev(c)
    ctx.advect(t, _dev(sx), _dev(sy), _dev(sz), step0=0, nsteps=2)
    ref = oracle.advect(c, sx, sy, sz, 0, 2)
    assert float(np.abs(t.cpu().numpy() - ref).max()) <= 1e-12


def test_graph_reuse(ctx, boxes):
    import torch

    note("batched graph reuse")
    ref = _plain(ctx, boxes, 4, 1, calls=3)
    dev = [(_dev(c), _dev(sx), _dev(sy), _dev(sz)) for c, sx, sy, sz in boxes]
    for _ in range(3):
        ctx.advect_batched(dev, step0=4, nsteps=1, tuning=(16, 4))
        torch.cuda.synchronize()  # eager work between replays
        _ = dev[0][0].sum().item()
    for (c, _, _, _), r in zip(dev, ref):
        assert torch.equal(c, r)


def test_empty_and_bad_arguments(ctx, boxes):
    from paper_2407_07463_amd import vofmt

    ctx.advect_batched([], nsteps=3)
    c, sx, sy, sz = boxes[0]
    dev = [(_dev(c), _dev(sx), _dev(sy), _dev(sz))]
    with pytest.raises(vofmt.VofmtError):
        ctx.advect_batched(dev, nsteps=1, tuning=(12, 4))
    with pytest.raises(vofmt.VofmtError):
        ctx.advect_batched(dev, nsteps=1, tuning=(32, 0))


def test_autotuner_leaves_fields_untouched(ctx, boxes):
    import torch

    dev = [(_dev(c), _dev(sx), _dev(sy), _dev(sz)) for c, sx, sy, sz in boxes]
    before = [c.clone() for c, _, _, _ in dev]
    (chunk, wg), ms = ctx.autotune_batched(dev, nsteps=1)
    torch.cuda.synchronize()
    assert chunk in (16, 32, 64) and wg in (2, 4, 8, 16) and ms > 0.0
    for (c, _, _, _), b in zip(dev, before):
        assert torch.equal(c, b)


def test_thirty_two_uneven_boxes(ctx):
    import torch

    bb = synth.batch_boxes(32, sizes=(16, 24, 32, 40, 48), seed=77, diameter=8.0, phi_range=(0.05, 0.2))
    boxes = [(b["c"], b["sx"], b["sy"], b["sz"]) for b in bb]
    note("batched 32 boxes " + ",".join(f"{b['shape'][0]}x{b['ntracers']}" for b in bb))
    ref = _plain(ctx, boxes, 0, 2)
    dev = [(_dev(c), _dev(sx), _dev(sy), _dev(sz)) for c, sx, sy, sz in boxes]
    ctx.advect_batched(dev, step0=0, nsteps=2)
    torch.cuda.synchronize()
    for (c, _, _, _), r in zip(dev, ref):
        assert torch.equal(c, r)
