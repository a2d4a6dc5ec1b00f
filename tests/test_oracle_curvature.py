"""Pins of the oracle's height-function curvature.

The paper computes the curvature kappa_i of each tracer "as for a single
tracer" (section "The no-coalescence.h algorithm", citing Popinet's
surface-tension review); the oracle uses fixed 7-cell height columns. Pins:
kappa*Delta -> 2/R on spheres with second-order convergence, 0 on planes,
1/R on cylinders, sign independent of the side of the interface.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2407_07463_amd import synth


def sphere_kappa(R, centre, n=None):
    n = n or int(2 * R + 12)
    c = synth.fill_spheres((n, n, n), 1, [centre], [R], [0])[0]
    k, st = oracle.curvature_hf(c)
    ok = (st >= 1) & (st <= 3)
    return k[ok], st, c


@pytest.mark.parametrize("R", [4.0, 8.0, 16.0])
def test_sphere_curvature(R):
    vals, st, c = sphere_kappa(R, (R + 5.37, R + 6.11, R + 5.73))
    err = np.abs(vals * R / 2 - 1)
    assert ((st > 0).sum()) == ((c > 1e-12) & (c < 1 - 1e-12)).sum()  # every interface cell
    assert np.mean(err) < {4.0: 0.03, 8.0: 0.01, 16.0: 0.004}[R]


def test_sphere_convergence_second_order():
    errs = []
    for R in (5.0, 10.0, 20.0):
        vals, _, _ = sphere_kappa(R, (R + 5.21, R + 6.42, R + 5.9))
        errs.append(np.sqrt(np.mean((vals * R / 2 - 1) ** 2)))
    # halving the cell size relative to R divides the error by ~4 (allow 2.8)
    assert errs[0] / errs[1] > 2.8 and errs[1] / errs[2] > 2.8


def test_plane_zero_curvature():
    """Exact fractions of a periodic tilted slab (slopes 1/4, -1/4): kappa = 0."""
    from fractions import Fraction

    from exact_geometry import slab_fraction

    nx = ny = 64
    nz = 16
    t1, t2 = Fraction(1, 4), Fraction(-1, 4)
    n = (-t1, -t2, Fraction(1))
    lo, hi = Fraction(37, 10), Fraction(117, 10)
    cache = {}
    c = np.zeros((nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                off = (n[0] * i + n[1] * j + n[2] * k) % nz
                if off not in cache:
                    cache[off] = float(slab_fraction((0, 0, 0), n, lo - off, hi - off, shifts=(-nz, 0, nz)))
                c[k, j, i] = cache[off]
    k, st = oracle.curvature_hf(c)
    ok = (st >= 1) & (st <= 3)
    assert ok.sum() == ((c > 1e-12) & (c < 1 - 1e-12)).sum()
    assert np.abs(k[ok]).max() < 1e-12


def test_cylinder_curvature():
    R, n = 8.0, 32
    c = synth.fill_cylinders_z((8, n, n), 1, [(15.3, 16.2)], [R], [0])[0]
    k, st = oracle.curvature_hf(c)
    ok = (st >= 1) & (st <= 3)
    assert ok.sum() > 0
    assert np.mean(np.abs(k[ok] * R - 1)) < 0.01


def test_inverted_sphere_negative_curvature():
    """A spherical bubble (phase outside) has curvature -2/R: the sign follows the phase."""
    R = 8.0
    n = 28
    c = synth.fill_spheres((n, n, n), 1, [(14.3, 13.8, 14.1)], [R], [0])[0]
    k, st = oracle.curvature_hf(1.0 - c)
    ok = (st >= 1) & (st <= 3)
    assert np.mean(np.abs(k[ok] * R / 2 + 1)) < 0.01


def test_pure_cells_are_not_interface():
    c = np.zeros((8, 8, 8))
    c[:4] = 1.0
    k, st = oracle.curvature_hf(c)
    assert np.all(st == 0) and np.all(np.isnan(k))
