"""GPU parity of the drop-shape statistics (inertia tensor about the
centroid, aspect ratio chi = sqrt(I1/I2), mean drop velocity) against the
CPU FP64 oracle.

Bars. The GPU sums c r r^T about the centre of each drop's box and removes
the centroid's share (parallel axes); the oracle sums about the centroid
directly, so the two differ by rounding only: with n <= 2^17 cells per drop
and every term bounded by the tensor's trace, each component agrees within
n * eps * tr(I) <= 3e-11 tr(I) in the worst case (the cases below reach
~1e-15). The eigenvalues of a symmetric tensor move by at most the norm of
its perturbation (Weyl); the smallest one is at least V/6, which keeps chi's
relative error below 1e-10 for the drops here. Mean
velocities: within 1e-13 absolute (|u| <= 0.5, sums of c u over the drop).
"""
import numpy as np
import pytest

import oracle
from fixtures import random_blobs
from gpu_util import note, require_gpu
from paper_2407_07463_amd import synth

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


def _gpu_shapes(ctx, c, s=None):
    """Labels, drop counts, inertia, chi and velocity from the GPU."""
    import torch

    tc = _dev(c)
    lab = torch.zeros(tc.shape, dtype=torch.int32, device="cuda:0")
    nd = ctx.label_drops(tc, lab)
    D = int(nd.sum())
    inertia = torch.zeros((max(D, 1), 6), dtype=torch.float64, device="cuda:0")
    chi = torch.zeros(max(D, 1), dtype=torch.float64, device="cuda:0")
    vel = torch.zeros((max(D, 1), 3), dtype=torch.float64, device="cuda:0") if s is not None else None
    ctx.drop_shapes(tc, lab, nd, inertia, chi, [_dev(a) for a in s] if s is not None else None, vel)
    torch.cuda.synchronize()
    return (lab.cpu().numpy(), nd, inertia.cpu().numpy()[:D], chi.cpu().numpy()[:D],
            vel.cpu().numpy()[:D] if vel is not None else None)


def _oracle_shapes(c, labels, nd, s=None):
    I, V, X = [], [], []
    for t in range(c.shape[0]):
        k = int(nd[t])
        _, xyz, rc = oracle.drop_moments(c[t], labels[t], k)
        assert rc == 0
        inertia, vel, rc = oracle.drop_shapes(c[t], labels[t], k, xyz, s)
        assert rc == 0
        I.append(inertia)
        if vel is not None:
            V.append(vel)
    I = np.concatenate(I) if I else np.zeros((0, 6))
    _, chi = oracle.aspect_ratio(I)
    return I, chi, (np.concatenate(V) if V else None)


def _compare(c, gpu, s=None, ncells_max=1 << 17):
    lab, nd, gI, gchi, gvel = gpu
    oI, ochi, ovel = _oracle_shapes(c, lab, nd, s)
    assert len(gI) == len(oI)
    if len(oI) == 0:
        return
    tr = oI[:, :3].sum(axis=1) / 2.0  # trace of I over 2 = trace of J >= every |component|
    err = np.abs(gI - oI).max(axis=1) / tr
    assert err.max() <= ncells_max * 2.2e-16, err.max()
    assert np.all(np.abs(gchi / ochi - 1.0) <= 1e-10)
    if s is not None:
        assert np.abs(gvel - ovel).max() <= 1e-13
    return err.max()


def _velocity(shape, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-0.5, 0.5, shape) for _ in range(3)]


@pytest.mark.parametrize("seed", range(4))
def test_random_blobs(ctx, seed):
    rng = np.random.default_rng(40 + seed)
    while True:  # blobs that merge across half the box are out of the method's domain: draw again
        shape = tuple(int(v) for v in rng.integers(20, 61, 3))
        c = random_blobs(rng, shape, 3, 25, 1.0, 3.5)
        if all(oracle.drop_moments(c[t], *oracle.label(c[t]))[2] == 0 for t in range(3)):
            break
    s = _velocity(shape, seed) if seed % 2 == 0 else None
    note(f"drop shapes random blobs shape={shape} velocity={s is not None}")
    _compare(c, _gpu_shapes(ctx, c, s), s)


@pytest.mark.parametrize("shape,centre", [((48, 45, 47), (11.2, 44.1, 46.4)), ((64, 64, 64), (0.3, 63.8, 31.9)),
                                          ((50, 66, 70), (35.0, 33.0, 20.0))])
def test_rotated_ellipsoids(ctx, shape, centre):
    """One elongated ellipsoid per tracer, across the periodic boundaries in the
    first two cases, plus small spheres in a second tracer."""
    nz, ny, nx = shape
    R = synth.random_rotation(synth.Splitmix64(nx * ny + nz))
    Q = synth.ellipsoid_matrix([10.0, 5.0, 3.0], R)
    c = synth.fill_ellipsoids(shape, 2, [centre], [Q], [0], order=8)
    ctr = [((centre[0] + 14) % nx, (centre[1] + 7) % ny, (centre[2] + 9) % nz),
           ((centre[0] + 3) % nx, (centre[1] + 15) % ny, (centre[2] + 1) % nz)]
    synth.fill_spheres(shape, 2, ctr, [2.5, 4.0], [1, 1], order=8, out=c)
    s = _velocity(shape, 7)
    note(f"drop shapes ellipsoid shape={shape} centre={centre}")
    _compare(c, _gpu_shapes(ctx, c, s), s)


def test_spheres64(ctx):
    w = synth.spheres64(order=8)
    s = [w["sx"], w["sy"], w["sz"]]
    note("drop shapes spheres64")
    _compare(w["c"], _gpu_shapes(ctx, w["c"], s), s)


def test_single_cells_and_rods(ctx):
    """Degenerate drops: single cells (I = c/6 delta, chi = 1 exactly on both
    sides), two-cell pairs and one-cell-thick rods (two equal eigenvalues)."""
    c = np.zeros((1, 12, 20, 24))
    c[0, 1, 1, 1] = 0.7
    c[0, 5, 5, 5] = 1.0
    c[0, 5, 5, 6] = 0.25
    c[0, 9, 10, 2:10] = 1.0
    c[0, 3:9, 15, 20] = 0.5
    lab, nd, gI, gchi, gvel = _gpu_shapes(ctx, c)
    assert list(nd) == [4]
    assert gchi[0] == 1.0
    assert np.array_equal(gI[0], [0.7 / 6.0] * 3 + [0.0] * 3)
    _compare(c, (lab, nd, gI, gchi, gvel))


def test_empty_and_errors(ctx):
    import torch
    from paper_2407_07463_amd import vofmt

    c = np.zeros((2, 8, 9, 10))
    lab, nd, gI, gchi, _ = _gpu_shapes(ctx, c)
    assert list(nd) == [0, 0] and len(gI) == 0
    # labels that name a drop the counts do not have
    c[1, 2, 2, 2] = 1.0
    tc = _dev(c)
    labt = torch.zeros(tc.shape, dtype=torch.int32, device="cuda:0")
    nd = ctx.label_drops(tc, labt)
    inertia = torch.zeros((2, 6), dtype=torch.float64, device="cuda:0")
    chi = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    with pytest.raises(vofmt.VofmtError):
        ctx.drop_shapes(tc, labt, [0, 2], inertia, chi)
    # velocity output without velocity
    L = vofmt.load()
    ndh = np.array([0, 1], dtype=np.int32)
    rc = L.vofmt_drop_shapes(ctx.h, 10, 9, 8, 2, vofmt._ptr(tc), vofmt._ptr(labt), ndh.ctypes.data, None, None,
                             None, vofmt._ptr(inertia), vofmt._ptr(chi), vofmt._ptr(inertia), vofmt._stream())
    assert rc == vofmt.E_ARG
    # a drop spanning half the box along x: reported, outputs still written
    c = np.zeros((1, 6, 6, 16))
    c[0, 2, 2, 3:12] = 1.0
    tc = _dev(c)
    labt = torch.zeros(tc.shape, dtype=torch.int32, device="cuda:0")
    nd = ctx.label_drops(tc, labt)
    chi = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    rc = L.vofmt_drop_shapes(ctx.h, 16, 6, 6, 1, vofmt._ptr(tc), vofmt._ptr(labt), np.asarray(nd, np.int32).ctypes.data,
                             None, None, None, vofmt._ptr(inertia), vofmt._ptr(chi), None, vofmt._stream())
    assert rc == vofmt.E_EXTENT
    assert chi.cpu().numpy()[0] > 1.0
