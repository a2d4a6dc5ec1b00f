"""Pins of the oracle's PLIC geometry: plane/cube volume, its inverse, MYC normals.

The paper names geometric PLIC VoF (section "Numerical method") without its
discrete form; the volume function is the Scardovelli-Zaleski plane/cube
volume and the normal is Mixed-Youngs-Centred (Aulisa et al. 2007). These
tests pin the oracle to closed forms, symmetries and exact rational
arithmetic, independent of the oracle's own formulas.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_geometry import cube_cut_volume


def test_volume_axis_aligned_is_clamped_alpha():
    for a in np.linspace(-0.5, 1.5, 41):
        assert oracle.plane_volume((0.0, 0.0, 1.0), a) == min(max(a, 0.0), 1.0)
        assert oracle.plane_volume((0.0, -1.0, 0.0), a) == min(max(a + 1.0, 0.0), 1.0)


def test_volume_half_at_centre_and_symmetry():
    rng = random.Random(7)
    for _ in range(2000):
        m = [rng.uniform(-1, 1) for _ in range(3)]
        M = sum(abs(v) for v in m)
        lo = sum(v for v in m if v < 0)
        assert oracle.plane_volume(m, lo + M / 2) == pytest.approx(0.5, abs=1e-15)
        a = lo + rng.uniform(0, M)
        v1 = oracle.plane_volume(m, a)
        v2 = oracle.plane_volume([-x for x in m], -a)  # complement region {m.x >= a}
        assert v1 + v2 == pytest.approx(1.0, abs=1e-15)


def test_volume_monotone_in_alpha():
    rng = random.Random(11)
    for _ in range(200):
        m = [rng.uniform(-1, 1) for _ in range(3)]
        lo = sum(v for v in m if v < 0)
        hi = sum(v for v in m if v > 0)
        a = np.linspace(lo - 0.1, hi + 0.1, 301)
        v = np.array([oracle.plane_volume(m, x) for x in a])
        assert np.all(np.diff(v) >= -1e-16)
        assert v[0] == 0.0 and v[-1] == 1.0


@pytest.mark.parametrize("seed", range(4))
def test_volume_matches_exact_inclusion_exclusion(seed):
    rng = random.Random(seed)
    worst = 0.0
    for _ in range(1500):
        m = [rng.uniform(-1, 1) for _ in range(3)]
        if min(abs(v) for v in m) < 1e-6:
            continue
        lo = sum(v for v in m if v < 0)
        a = lo + rng.uniform(0, sum(abs(v) for v in m))
        exact = float(cube_cut_volume([Fraction(v) for v in m], Fraction(a)))
        got = oracle.plane_volume(m, a)
        worst = max(worst, abs(got - exact))
    assert worst < 2e-13


def test_volume_degenerate_reductions():
    rng = random.Random(3)
    for _ in range(500):
        # 2-D: m3 = 0 reduces to the area cut from the unit square
        m = [rng.uniform(0.01, 1), rng.uniform(0.01, 1), 0.0]
        a = rng.uniform(0, m[0] + m[1])
        exact = float(cube_cut_volume([Fraction(m[0]), Fraction(m[1])], Fraction(a)))
        assert oracle.plane_volume(m, a) == pytest.approx(exact, abs=1e-14)
        # 1-D: only one component
        m1 = rng.uniform(0.01, 1)
        a1 = rng.uniform(-0.2, 1.2) * m1
        assert oracle.plane_volume((0.0, m1, 0.0), a1) == pytest.approx(min(max(a1 / m1, 0), 1), abs=1e-15)
    # the tetrahedral corner: alpha^3 / (6 m1 m2 m3)
    assert oracle.plane_volume((0.2, 0.3, 0.5), 0.1) == pytest.approx(0.1**3 / (6 * 0.2 * 0.3 * 0.5), rel=1e-15)


def test_alpha_round_trip():
    rng = random.Random(5)
    for _ in range(3000):
        m = np.array([rng.uniform(-1, 1) for _ in range(3)])
        m /= np.abs(m).sum()
        c = rng.uniform(1e-9, 1 - 1e-9) if rng.random() < 0.9 else rng.choice([1e-14, 1 - 1e-14, 0.5])
        a = oracle.plane_alpha(m, c)
        v = oracle.plane_volume(m, a)
        assert abs(v - c) <= 4 * np.spacing(max(c, 1e-300)) + 1e-300 or abs(v - c) <= 4.5e-16


def _plane_block(normal, alpha0):
    """Exact fractions of {n.x <= alpha0} (x relative to the centre cell's lower corner) in a 3x3x3 block."""
    b = np.zeros((3, 3, 3))
    n = [Fraction(v) for v in normal]
    for az in (-1, 0, 1):
        for ay in (-1, 0, 1):
            for ax in (-1, 0, 1):
                a = Fraction(alpha0) - (n[0] * ax + n[1] * ay + n[2] * az)
                b[az + 1, ay + 1, ax + 1] = float(cube_cut_volume(n, a))
    return b


def test_myc_exact_on_gentle_planes():
    """Slopes t relative to the dominant axis with 2|t1|+|t2| <= 1 and |t1|+2|t2| <= 1
    keep every 3-cell column unsaturated, so the centred-columns estimate is
    exact and the choice rule must select it: MYC returns the exact normal."""
    rng = random.Random(2024)
    checked = 0
    while checked < 400:
        t1 = Fraction(rng.randint(-64, 64), 128)
        t2 = Fraction(rng.randint(-64, 64), 128)
        if 2 * abs(t1) + abs(t2) > 1 or abs(t1) + 2 * abs(t2) > 1:
            continue
        d = rng.randrange(3)
        sgn = rng.choice([1, -1])
        n = [None, None, None]
        tr = [a for a in range(3) if a != d]
        n[d] = Fraction(sgn)
        n[tr[0]] = -t1
        n[tr[1]] = -t2
        # plane through the centre cell: choose alpha so that the centre is mixed
        L1 = sum(abs(v) for v in n)
        lo = sum(v for v in n if v < 0)
        alpha0 = lo + L1 * Fraction(rng.randint(1, 63), 64)
        b = _plane_block(n, alpha0)
        if not (0 < b[1, 1, 1] < 1):
            continue
        m, used_cs = oracle.myc_normal(b)
        exact = np.array([float(v / L1) for v in n])
        assert used_cs
        assert np.max(np.abs(m - exact)) < 1e-15, (n, m, exact)
        checked += 1


def test_myc_isolated_cell_fallback():
    b = np.zeros((3, 3, 3))
    b[1, 1, 1] = 0.3
    m, used_cs = oracle.myc_normal(b)
    assert used_cs and tuple(m) == (1.0, 0.0, 0.0)


def test_myc_sign_points_away_from_phase():
    # phase below a horizontal interface: outward normal is +z
    b = np.zeros((3, 3, 3))
    b[0] = 1.0
    b[1] = 0.4
    m, _ = oracle.myc_normal(b)
    assert m[2] == pytest.approx(1.0) and abs(m[0]) < 1e-15 and abs(m[1]) < 1e-15
    # phase on the +x side: outward normal is -x
    b = np.zeros((3, 3, 3))
    b[:, :, 2] = 1.0
    b[:, :, 1] = 0.7
    m, _ = oracle.myc_normal(b)
    assert m[0] == pytest.approx(-1.0)


def test_face_flux_matches_exact_subbox_volume():
    """Flux through a face = s times the exact phase volume of the donor's upwind sub-box."""
    rng = random.Random(99)
    for _ in range(200):
        t1 = Fraction(rng.randint(-30, 30), 128)
        t2 = Fraction(rng.randint(-30, 30), 128)
        n = [-t1, -t2, Fraction(1)]
        L1 = sum(abs(v) for v in n)
        lo = sum(v for v in n if v < 0)
        alpha0 = lo + L1 * Fraction(rng.randint(8, 56), 64)
        # 5x5x5 periodic-free field around the donor at (2,2,2): exact plane fractions
        f = np.zeros((5, 5, 5))
        for k in range(5):
            for j in range(5):
                for i in range(5):
                    a = alpha0 - (n[0] * (i - 2) + n[1] * (j - 2) + n[2] * (k - 2))
                    f[k, j, i] = float(cube_cut_volume(n, a))
        if not (0 < f[2, 2, 2] < 1):
            continue
        for d in range(3):
            s = Fraction(rng.choice([-1, 1]) * rng.randint(1, 63), 128)
            # face on the lower d-face of cell q; donor (2,2,2) is upwind
            q = [2, 2, 2]
            if s > 0:
                q[d] += 1
            sub_lo = [Fraction(0)] * 3
            sub_hi = [Fraction(1)] * 3
            if s > 0:
                sub_lo[d] = 1 - s
            else:
                sub_hi[d] = -s
            # exact volume of {n.x <= alpha0} inside the sub-box (affine map to the unit cube)
            width = [sub_hi[e] - sub_lo[e] for e in range(3)]
            ns = [n[e] * width[e] for e in range(3)]
            a_sub = alpha0 - sum(n[e] * sub_lo[e] for e in range(3))
            phi = cube_cut_volume(ns, a_sub)
            expect = float(s * phi)
            got = oracle.lib().orc_face_flux(np.ascontiguousarray(f).ctypes.data, 5, 5, 5, d, q[0], q[1], q[2],
                                             float(s))
            assert got == pytest.approx(expect, abs=2e-15)
