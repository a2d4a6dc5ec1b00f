"""Pins of the oracle's multi-tracer surface-tension force (section "The
no-coalescence.h algorithm": the sum over tracers of gamma kappa_i grad C_i;
face-centred balanced-force form).

  - With one curvature value everywhere, the force on the lower faces is
    the discrete gradient of the potential gamma kappa sum_i C_i (the
    balanced-force property), and its sum over the box vanishes;
  - a five-cell profile whose face values are worked out by hand: a face
    between two defined curvatures, a face with one, a face with none and a
    face without a jump in C — along each axis in turn;
  - tracers add up: the force of two tracers is the sum of their forces;
  - a sphere with the exact curvature 2/R on its interface cells: the force
    through the central plane is gamma (2/R) times the plane's wetted area
    (the Laplace pressure jump), and there is no net force; with the
    oracle's own height-function curvature the net force vanishes by
    symmetry, up to the grid.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2407_07463_amd import synth


def test_uniform_curvature_is_a_discrete_gradient():
    rng = np.random.default_rng(3)
    shape = (7, 9, 11)
    c = rng.uniform(0, 1, (3,) + shape) * (rng.uniform(size=(3,) + shape) < 0.6)
    k0, gamma = 0.37, 1.75
    kap = np.full(c.shape, k0)
    fx, fy, fz = oracle.csf_force(c, kap, gamma)
    S = gamma * k0 * c.sum(axis=0)
    for f, ax in ((fx, 2), (fy, 1), (fz, 0)):
        want = S - np.roll(S, 1, axis=ax)  # value on the lower face of each cell
        assert np.allclose(f, want, rtol=0, atol=1e-14)
        assert abs(f.sum()) < 1e-12


NAN = float("nan")


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hand_worked_profile(axis):
    # cells 0..4 along one axis, periodic; every other axis has one cell
    C = [0.0, 0.3, 1.0, 0.6, 1.0]
    K = [NAN, 0.5, 0.3, 0.2, NAN]
    gamma = 2.0
    # lower face of cell i (between i-1 and i):
    # 0: C jumps 1 -> 0, no curvature on either side -> 0
    # 1: jump +0.3, only cell 1 defined (0.5)       -> 2 * 0.5 * 0.3 = 0.3
    # 2: jump +0.7, mean of 0.5 and 0.3 = 0.4        -> 2 * 0.4 * 0.7 = 0.56
    # 3: jump -0.4, mean of 0.3 and 0.2 = 0.25       -> 2 * 0.25 * -0.4 = -0.2
    # 4: jump +0.4, only cell 3 defined (0.2)        -> 2 * 0.2 * 0.4 = 0.16
    want = np.array([0.0, 0.3, 0.56, -0.2, 0.16])
    shape = [1, 1, 1]
    shape[axis] = 5
    c = np.array(C).reshape(shape)
    kap = np.array(K).reshape(shape)
    f = oracle.csf_force(c, kap, gamma)  # (fx, fy, fz)
    along = {2: 0, 1: 1, 0: 2}[axis]  # array axis -> force component
    assert np.allclose(f[along].ravel(), want, rtol=0, atol=1e-15)
    for d in range(3):
        if d != along:
            assert np.array_equal(f[d].ravel(), np.zeros(5))  # one cell: no jump


def test_tracers_add_up():
    rng = np.random.default_rng(8)
    shape = (6, 5, 7)
    c = rng.uniform(0, 1, (2,) + shape)
    kap = np.where(rng.uniform(size=c.shape) < 0.5, rng.normal(size=c.shape), np.nan)
    both = oracle.csf_force(c, kap, 0.8)
    one = oracle.csf_force(c[:1], kap[:1], 0.8)
    two = oracle.csf_force(c[1:], kap[1:], 0.8)
    for d in range(3):
        assert np.allclose(both[d], one[d] + two[d], rtol=0, atol=1e-15)


def test_sphere_pressure_jump():
    R, n = 9.0, 40
    ctr = (20.3, 19.6, 20.2)
    c = synth.fill_spheres((n, n, n), 1, [ctr], [R], [0], order=16)[0]
    gamma = 1.0
    scale = gamma * (2.0 / R) * math.pi * R * R
    # the exact curvature 2/R on the interface (mixed) cells only: every face
    # with a jump in C touches one, so the force through the plane below cell
    # 21 along x is gamma (2/R) times the wetted area of the slab [20, 21],
    # pi (R^2 - (20.5 - 20.3)^2) up to the slab's curvature (R^-2 small)
    mixed = (c > 0) & (c < 1)
    kap = np.where(mixed, 2.0 / R, np.nan)
    fx, fy, fz = oracle.csf_force(c, kap, gamma)
    for f in (fx, fy, fz):
        assert abs(f.sum()) < 1e-12 * scale  # telescoping: no net force
    through = fx[:, :, : int(ctr[0]) + 1].sum()
    area = math.pi * (R * R - (int(ctr[0]) + 0.5 - ctr[0]) ** 2)
    assert through == pytest.approx(gamma * (2.0 / R) * area, rel=5e-3)
    # the oracle's own height-function curvature: no net force by symmetry,
    # up to the grid (cells where the height function is invalid carry none)
    kap, st = oracle.curvature_hf(c)
    fx, fy, fz = oracle.csf_force(c, kap, gamma)
    for f in (fx, fy, fz):
        assert abs(f.sum()) < 0.02 * scale
