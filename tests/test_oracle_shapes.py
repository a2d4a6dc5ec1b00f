"""Pins of the oracle's drop-shape statistics (appendix "Deformation of the
drops": inertia tensor about the centre of mass and the aspect ratio
chi = sqrt(I1/I2); plus the drop's mean velocity).

Each expected value comes from a closed form that is not the oracle's sum:
  - a rectangular block of full cells has the solid cuboid's tensor,
    V (b^2 + c^2) / 12 etc. with no products of inertia (textbook);
  - a rod of k full cells along the (1,1,0) diagonal: the positions along the
    rod have the variance (k^2 - 1)/12 of k consecutive integers, which gives
    Ixy = -k (k^2 - 1)/12 (the sign of a body stretched along x = y);
  - a rotated ellipsoid with semi-axes (a, b, c): I = (V/5) R diag(b^2 + c^2,
    a^2 + c^2, a^2 + b^2) R^T and chi = sqrt((a^2 + b^2)/(b^2 + c^2)), up to
    the grid's discretisation;
  - a periodic shift of the field leaves every tensor unchanged;
  - a uniform velocity is every drop's velocity exactly; a linear one is its
    value at the centroid.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2407_07463_amd import synth


def _shapes(c, s=None):
    lab, k = oracle.label(c)
    vol, xyz, rc = oracle.drop_moments(c, lab, k)
    assert rc == 0
    inertia, vel, rc = oracle.drop_shapes(c, lab, k, xyz, s)
    assert rc == 0
    return lab, k, vol, xyz, inertia, vel


def test_cuboid_across_the_periodic_boundary():
    nz, ny, nx = 20, 12, 16
    a, b, cz = 5, 3, 7  # cells along x, y, z
    c = np.zeros((nz, ny, nx))
    xs = [(13 + i) % nx for i in range(a)]
    ys = [(10 + i) % ny for i in range(b)]
    zs = [(17 + i) % nz for i in range(cz)]
    for value in (1.0, 0.5):
        c[:] = 0.0
        c[np.ix_(zs, ys, xs)] = value
        _, k, vol, _, inertia, _ = _shapes(c)
        assert k == 1
        V = value * a * b * cz
        want = V / 12.0 * np.array([b * b + cz * cz, a * a + cz * cz, a * a + b * b, 0, 0, 0])
        assert np.allclose(inertia[0], want, rtol=0, atol=1e-12 * V * 100)
        ev, chi = oracle.aspect_ratio(inertia)
        assert chi[0] == pytest.approx(math.sqrt((a * a + cz * cz) / (a * a + b * b)), rel=1e-13)


def test_diagonal_rod_products_of_inertia():
    k = 6
    nz, ny, nx = 4, 16, 16
    c = np.zeros((nz, ny, nx))
    lab = np.zeros(c.shape, dtype=np.int32)
    for i in range(k):
        c[1, i + 2, i + 2] = 1.0
        lab[1, i + 2, i + 2] = 1  # one drop by fiat: diagonal cells share no face
    vol, xyz, rc = oracle.drop_moments(c, lab, 1)
    assert rc == 0
    inertia, _, rc = oracle.drop_shapes(c, lab, 1, xyz)
    assert rc == 0
    var = k * (k * k - 1) / 12.0  # sum of squared deviations of 0..k-1
    want = [var + k / 6.0, var + k / 6.0, 2 * var + k / 6.0, -var, 0.0, 0.0]
    assert np.allclose(inertia[0], want, rtol=0, atol=1e-12)
    # principal moments: about the rod k/6, across it 2 var + k/6 (twice)
    ev, chi = oracle.aspect_ratio(inertia)
    assert np.allclose(ev[0], [k / 6.0, 2 * var + k / 6.0, 2 * var + k / 6.0], atol=1e-12)


def _rotation(z_deg, x_deg):
    a, b = math.radians(z_deg), math.radians(x_deg)
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    return Rz @ Rx


def _ellipsoid_error(scale, centre, n):
    axes = scale * np.array([9.0, 6.0, 4.0])
    R = _rotation(30.0, 20.0)
    Q = synth.ellipsoid_matrix(axes, R)
    c = synth.fill_ellipsoids((n, n, n), 1, [centre], [Q], [0], order=16)[0]
    _, k, vol, _, inertia, _ = _shapes(c)
    assert k == 1
    a, b, cc = axes
    T = vol[0] / 5.0 * R @ np.diag([b * b + cc * cc, a * a + cc * cc, a * a + b * b]) @ R.T
    want = np.array([T[0, 0], T[1, 1], T[2, 2], T[0, 1], T[0, 2], T[1, 2]])
    _, chi = oracle.aspect_ratio(inertia)
    chi_want = math.sqrt((a * a + b * b) / (b * b + cc * cc))
    return (inertia[0] - want) / np.trace(T), chi[0] / chi_want - 1.0


@pytest.mark.parametrize("scale,centre,n", [(1, (20.3, 19.7, 20.1), 40), (1, (1.2, 38.6, 0.4), 40),
                                            (2, (36.3, 35.7, 36.1), 72)])
def test_rotated_ellipsoid(scale, centre, n):
    """Products of inertia (which carry the rotation and its sign) to 1e-4 of
    the trace; the moments carry the grid's bias, which is second order in
    the cell size: the fluid of a cut cell sits at its centre (6e-3 of the
    trace at a smallest semi-axis of 4 cells)."""
    err, chi_err = _ellipsoid_error(scale, centre, n)
    assert np.abs(err[3:]).max() <= 1e-4
    assert np.abs(err[:3]).max() <= 1e-2 / scale**2
    assert abs(chi_err) <= 1e-2 / scale**2


def test_ellipsoid_converges_at_second_order():
    e1, c1 = _ellipsoid_error(1, (20.3, 19.7, 20.1), 40)
    e2, c2 = _ellipsoid_error(2, (36.3, 35.7, 36.1), 72)
    ratio = np.abs(e1[:3]).max() / np.abs(e2[:3]).max()
    assert 3.0 < ratio < 5.0
    assert 3.0 < abs(c1) / abs(c2) < 5.0


def test_sphere_is_round():
    Rr = 7.5
    c = synth.fill_spheres((32, 32, 32), 1, [(15.6, 16.3, 16.9)], [Rr], [0], order=16)[0]
    _, k, vol, _, inertia, _ = _shapes(c)
    ev, chi = oracle.aspect_ratio(inertia)
    assert abs(chi[0] - 1.0) < 2e-3
    # the cut cells' bias (second order, as for the ellipsoid): 1.5% at R = 7.5
    assert np.allclose(inertia[0][:3], 0.4 * vol[0] * Rr * Rr, rtol=1.0 / Rr**2)
    assert np.abs(inertia[0][3:]).max() <= 1e-4 * inertia[0][:3].sum()


def test_periodic_shift_invariance():
    Q = synth.ellipsoid_matrix([7.0, 5.0, 3.5], _rotation(-25.0, 40.0))
    c = synth.fill_ellipsoids((24, 28, 32), 1, [(30.5, 1.5, 22.8)], [Q], [0], order=8)[0]
    _, k, vol, _, I0, _ = _shapes(c)
    c2 = np.roll(c, (5, -9, 13), axis=(0, 1, 2))
    _, k2, vol2, _, I2, _ = _shapes(c2)
    assert k == k2 == 1
    assert np.abs(I0 - I2).max() <= 1e-12 * I0[0, :3].sum()


def test_velocity_uniform_and_linear():
    rng = np.random.default_rng(5)
    nz, ny, nx = 24, 24, 24
    c = synth.fill_spheres((nz, ny, nx), 1, [(7.3, 8.1, 9.4), (16.2, 15.5, 15.9)], [3.2, 4.1], [0, 0],
                           order=8)[0]
    c += (c > 0) * rng.uniform(-1e-3, 0, c.shape)  # uneven weights
    shape = c.shape
    # powers of two: every c u and their sums scale exactly
    s = [np.full(shape, 0.25), np.full(shape, -0.125), np.full(shape, 0.0625)]
    _, k, vol, xyz, _, vel = _shapes(c, s)
    assert k == 2
    assert np.array_equal(vel, np.tile([0.25, -0.125, 0.0625], (2, 1)))
    # linear fields, each along its own axis; s_d on the lower d-face of cell i sits at x_d = i
    al, be, ga = 0.01, -0.02, 0.015
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = [al * (xx - 3.0), be * (yy - 5.0), ga * (zz - 2.0)]
    _, _, _, xyz, _, vel = _shapes(c, s)
    want = np.stack([al * (xyz[:, 0] - 3.0), be * (xyz[:, 1] - 5.0), ga * (xyz[:, 2] - 2.0)], axis=1)
    assert np.abs(vel - want).max() <= 1e-14


def test_bad_labels():
    c = np.zeros((4, 4, 4))
    c[1, 1, 1] = 1.0
    lab = np.zeros(c.shape, dtype=np.int32)
    lab[1, 1, 1] = 2
    _, _, rc = oracle.drop_shapes(c, lab, 1, np.zeros((1, 3)))
    assert rc == oracle.E_ARG
