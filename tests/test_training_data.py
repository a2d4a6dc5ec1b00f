"""Pins of the training targets of the learned curvature: the curvature of an
ellipsoid at the surface point closest to a given point."""
import numpy as np

from paper_2407_07463_amd import synth
from paper_2407_07463_amd.training import ellipsoid_closest_kappa, init_params, NPARAMS


def _surface_points(axes, n, seed):
    rng = synth.Splitmix64(seed)
    u, v = rng.uniform(n), rng.uniform(n)
    th, ph = np.arccos(1 - 2 * u), 2 * np.pi * v
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    return d * np.asarray(axes)


def _kappa_closed_form(x, axes):
    """kappa1 + kappa2 of the ellipsoid at surface point x (classical closed form)."""
    a, b, c = axes
    r2 = np.sum(x * x, axis=1)
    s = x[:, 0] ** 2 / a ** 4 + x[:, 1] ** 2 / b ** 4 + x[:, 2] ** 2 / c ** 4
    return (a * a + b * b + c * c - r2) / ((a * b * c) ** 2 * s ** 1.5)


def test_sphere_gives_two_over_r():
    for R in (2.0, 5.5, 40.0):
        p = _surface_points((R, R, R), 50, 1) * (1.0 + 0.2 * (synth.Splitmix64(2).uniform(50)[:, None] - 0.5))
        assert np.allclose(ellipsoid_closest_kappa(p, (R, R, R)), 2.0 / R, rtol=1e-12)


def test_ellipsoid_vertices():
    a, b, c = 3.0, 5.0, 7.0
    p = np.array([[a + 0.3, 0, 0], [0, b - 0.4, 0], [0, 0, c + 0.2]])
    k = ellipsoid_closest_kappa(p, (a, b, c))
    assert np.allclose(k, [a / b ** 2 + a / c ** 2, b / a ** 2 + b / c ** 2, c / a ** 2 + c / b ** 2], rtol=1e-12)


def test_closest_point_along_the_normal():
    axes = np.array([4.0, 6.0, 7.5])
    x = _surface_points(axes, 200, 3)
    n = x / axes ** 2
    n /= np.linalg.norm(n, axis=1)[:, None]
    want = _kappa_closed_form(x, axes)
    for t in (-0.7, -0.2, 0.0, 0.3, 0.9):  # inside the focal distance (>= 4^2/7.5)
        got = ellipsoid_closest_kappa(x + t * n, axes)
        assert np.allclose(got, want, rtol=1e-9), t


def test_init_params_layout():
    P = init_params(5)
    assert P.shape == (NPARAMS,) and P.dtype == np.float32
    assert np.all(P[27 * 128:32 * 128] == 0.0) and np.all(P[4096:4224] == 0.0)
