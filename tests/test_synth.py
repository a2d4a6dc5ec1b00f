"""The seeded input generators: accuracy of the drop fractions, placement and velocity fields."""
import math

import numpy as np
import pytest

from paper_2407_07463_amd import synth


def test_splitmix64_reference_values():
    # splitmix64 from seed 0: first outputs of the published generator
    rng = synth.Splitmix64(0)
    u = rng.uniform(3)
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert np.array_equal(u, np.array([(v >> 11) * 2.0**-53 for v in expect]))


def test_sphere_volumes_and_wrap():
    n = 32
    for centre, R in (((10.37, 11.91, 13.2), 6.3), ((0.3, 31.5, 1.2), 6.1)):
        c = synth.fill_spheres((n, n, n), 1, [centre], [R], [0])
        assert c.sum() == pytest.approx(4 / 3 * math.pi * R**3, rel=1e-12)
        assert c.min() >= 0 and c.max() <= 1


def test_rotated_ellipsoid_volume():
    rng = synth.Splitmix64(4)
    Q = synth.ellipsoid_matrix([5.0, 7.0, 9.3], synth.random_rotation(rng))
    c = synth.fill_ellipsoids((32, 32, 32), 1, [(16.2, 15.7, 14.9)], [Q], [0])
    assert c.sum() == pytest.approx(4 / 3 * math.pi * 5 * 7 * 9.3, rel=1e-12)


def test_cell_fraction_against_fine_sampling():
    centre = np.array([10.37, 11.91, 13.2])
    Q = np.eye(3) / 6.3**2
    m = 160
    g = (np.arange(m) + 0.5) / m
    for cell in [(6, 8, 9), (15, 10, 16), (12, 17, 8)]:
        v = synth.cell_fraction(centre, Q, cell)
        X, Y, Z = np.meshgrid(cell[0] + g, cell[1] + g, cell[2] + g, indexing="ij")
        mc = (((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) <= 6.3**2).mean()
        assert abs(v - mc) < 5e-4  # midpoint sampling error of the reference itself


def test_rsa_gap_and_count():
    rng = synth.Splitmix64(9)
    radii = np.full(60, 3.0)
    x = synth.rsa(rng, radii, (50.0, 50.0, 50.0), gap=2.0)
    for i in range(len(x)):
        d = x - x[i]
        d = (d + 25.0) % 50.0 - 25.0
        r = np.sqrt((d * d).sum(1))
        r[i] = np.inf
        assert r.min() >= 8.0


def test_fourier_velocity_solenoidal_and_bounded():
    sx, sy, sz, rms = synth.fourier_velocity((32, 24, 16), seed=3, kmax=5)
    div = (np.roll(sx, -1, 2) - sx) + (np.roll(sy, -1, 1) - sy) + (np.roll(sz, -1, 0) - sz)
    assert np.abs(div).max() < 1e-15
    assert max(np.abs(sx).max(), np.abs(sy).max(), np.abs(sz).max()) <= 0.45 + 1e-15
    assert sz.mean() == pytest.approx(0.1, abs=1e-12)
    assert 0 < rms <= 0.2 + 1e-12


def test_workload_spheres64_shape():
    w = synth.spheres64()
    assert w["c"].shape == (2, 64, 64, 64)
    assert w["c"].sum() == pytest.approx(8 * 4 / 3 * math.pi * 216, rel=1e-12)
