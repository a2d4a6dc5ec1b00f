"""The no-allocation entry point against the one it mirrors.

vofmt_nearest_pair_stats_noalloc (fixed device scratch, edges as a kernel
argument) must give exactly what vofmt_nearest_pair_stats gives (same
kernels, same order): indices, tie counts, histograms, M, R and A bit for
bit, on two calls in a row, the second smaller than the first (the fixed
array keeps the first call's contents), and refuse sizes beyond its limits.
"""
import math

import numpy as np
import pytest

from gpu_util import note, require_gpu
from paper_2407_07463_amd import synth

pytestmark = pytest.mark.gpu


def _outputs(torch, n, nr, nth):
    z = lambda k, dt: torch.zeros(k, dtype=dt, device="cuda:0")  # noqa: E731
    return dict(idx=z(n, torch.int32), ties=z(n, torch.int32), hist=z(nr * nth + 1, torch.int64),
                M=z(3, torch.float64), R=z(9, torch.float64), A=z(9, torch.float64))


def _call(ctx, fn, xyz, box, r2e, ce, o):
    fn(xyz, box, 2, r2e, ce, o["idx"], o["ties"], o["hist"], o["M"], o["R"], o["A"])


def test_noalloc_matches_the_allocating_entry_point():
    torch = require_gpu()
    from paper_2407_07463_amd import vofmt

    ctx = vofmt.Context(0)
    try:
        box = np.array([512.0, 512.0, 512.0])
        nr, nth = 64, 32
        r2e = (np.arange(nr + 1) * (96.0 / nr)) ** 2
        ce = np.cos(np.arange(nth + 1) * math.pi / nth)
        for call, n in enumerate((8192, 1500)):
            rng = synth.Splitmix64(70 + call)
            xyz = torch.from_numpy(rng.uniform(3 * n).reshape(n, 3) * box).to("cuda:0")
            note(f"no-alloc pair stats call {call} n={n}")
            a = _outputs(torch, n, nr, nth)
            b = _outputs(torch, n, nr, nth)
            _call(ctx, ctx.nearest_pair_stats, xyz, box, r2e, ce, a)
            _call(ctx, ctx.nearest_pair_stats_noalloc, xyz, box, r2e, ce, b)
            torch.cuda.synchronize()
            for k in a:
                assert torch.equal(a[k], b[k]), (call, k)
            assert int(b["hist"].sum().item()) == 720720 * n
        # sizes beyond the fixed scratch are refused before anything runs
        n = 8193
        xyz = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
        o = _outputs(torch, n, nr, nth)
        with pytest.raises(vofmt.VofmtError) as e:
            _call(ctx, ctx.nearest_pair_stats_noalloc, xyz, box, r2e, ce, o)
        assert e.value.code == vofmt.E_ARG
        n = 100
        xyz = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
        big_r = np.arange(400.0) ** 2  # 399 + 32 + 2 = 433 edges > 384
        o = _outputs(torch, n, 399, nth)
        with pytest.raises(vofmt.VofmtError) as e:
            _call(ctx, ctx.nearest_pair_stats_noalloc, xyz, box, big_r, ce, o)
        assert e.value.code == vofmt.E_ARG
    finally:
        ctx.close()
