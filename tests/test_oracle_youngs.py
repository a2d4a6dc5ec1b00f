"""Pins of the Youngs branch of the oracle's Mixed-Youngs-Centred normal.

The paper names geometric PLIC VoF (section "Numerical method") without its
discrete normal; the oracle follows Aulisa et al. (2007): a centred-columns
candidate and a Youngs candidate -G/|G|_1, G the central differences of the
3x3x3 block weighted (1,2,1) across, with centred columns kept unless Youngs'
largest component beats the centred-columns quality. The gentle-plane pins
elsewhere always select centred columns; these select Youngs:

- planes at 45 degrees to two axes (and to all three), where the 3-cell
  columns saturate so the centred-columns estimate is biased, while Youngs is
  exact by the block's mirror symmetry (any symmetric weights would do, so the
  weights are pinned separately);
- one block whose gradient is worked out by hand from the (1,2,1) weights;
- the error of the normal over 6000 random planes with exact fractions, which
  separates the reading's choice rule (mean L-inf error 0.0013) from the
  opposite rule (0.020), from equal weights (0.0029) and from a wrong sign.
"""
import random
from fractions import Fraction

import numpy as np

import oracle
from exact_geometry import cube_cut_volume


def _block(n, alpha0):
    """Exact fractions of {n.x <= alpha0} (x from the centre cell's lower corner), b[az][ay][ax]."""
    b = np.zeros((3, 3, 3))
    for az in (-1, 0, 1):
        for ay in (-1, 0, 1):
            for ax in (-1, 0, 1):
                a = alpha0 - (n[0] * ax + n[1] * ay + n[2] * az)
                b[az + 1, ay + 1, ax + 1] = float(cube_cut_volume(n, a))
    return b


def test_youngs_exact_on_45_degree_planes():
    """n along (+-1, +-1, 0) in every axis pair: the block is symmetric under the swap of the
    two axes, so Youngs gives exactly (+-1/2, +-1/2, 0). The 3-cell columns saturate unless the
    plane passes through the centre cell's centre line, so centred columns overestimate their
    quality and the rule must pick Youngs."""
    checked = 0
    for pair in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                n = [Fraction(0)] * 3
                n[pair[0]] = Fraction(sa)
                n[pair[1]] = Fraction(sb)
                lo = sum(v for v in n if v < 0)
                for k in (1, 3, 5, 7, 9, 11, 13, 15):
                    if k == 8:
                        continue
                    alpha0 = lo + Fraction(2 * k, 16)
                    b = _block(n, alpha0)
                    assert 0 < b[1, 1, 1] < 1
                    m, used_cs = oracle.myc_normal(b)
                    assert not used_cs, (n, alpha0)
                    expect = np.array([float(v) / 2 for v in n])
                    assert np.array_equal(m, expect), (n, alpha0, m)
                    checked += 1
    assert checked == 96


def test_youngs_exact_on_body_diagonal_planes():
    """n along (+-1, +-1, +-1): the block is invariant under every permutation of the axes, so
    the three Youngs differences have the same magnitude and the normal is +-1/3 on every axis
    (up to rounding). Saturated columns again make the rule pick Youngs."""
    third = 1.0 / 3.0
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                n = [Fraction(sx), Fraction(sy), Fraction(sz)]
                lo = sum(v for v in n if v < 0)
                for k in (1, 2, 4, 5, 7, 8):
                    alpha0 = lo + Fraction(3 * k, 9)
                    b = _block(n, alpha0)
                    m, used_cs = oracle.myc_normal(b)
                    assert not used_cs, (n, alpha0)
                    # signs exact; magnitudes 1/3 up to the rounding of the sums (the reflections
                    # visit the same terms in another order)
                    assert np.array_equal(np.sign(m), np.array([sx, sy, sz], dtype=float)), (n, alpha0, m)
                    assert np.max(np.abs(np.abs(m) - third)) <= 4 * np.spacing(third), (n, alpha0, m)


def test_youngs_hand_worked_block():
    """A block with four non-zero cells, the gradient summed by hand.

    b(0,0,0) = 1/2 (centre), b(1,0,0) = 1/2, b(-1,1,1) = 1/4, b(0,-1,1) = 3/4 (offsets ax, ay, az).
    Weights are w(0) = 2, w(+-1) = 1 on the two transverse offsets:
      Gx = w(0)w(0)(1/2) - w(1)w(1)(1/4)                    = 2 - 1/4   = 7/4
      Gy = w(-1)w(1)(1/4) - w(0)w(1)(3/4)                   = 1/4 - 3/2 = -5/4
      Gz = w(-1)w(1)(1/4) + w(0)w(-1)(3/4)                  = 1/4 + 3/2 = 7/4
    |G|_1 = 19/4, Youngs = -G/|G|_1 = (-7/19, 5/19, -7/19), quality 7/19.
    Centred columns along x: every transverse column sum other than the centre's is 0, so the
    slopes vanish and the quality is 1 > 7/19: Youngs is chosen."""
    b = np.zeros((3, 3, 3))
    b[1, 1, 1] = 0.5
    b[1, 1, 2] = 0.5
    b[2, 2, 0] = 0.25
    b[2, 0, 1] = 0.75
    m, used_cs = oracle.myc_normal(b)
    assert not used_cs
    expect = np.array([-7.0 / 19.0, 5.0 / 19.0, -7.0 / 19.0])
    assert np.max(np.abs(m - expect)) <= 2 * np.spacing(0.5)


def test_myc_error_over_random_planes():
    """6000 planes with isotropic random normals (components rounded to 1/1024) through the
    centre cell, fractions exact. With the choice rule of the reading the mean L-inf error of
    the normal is 0.0013 and the largest 0.0106; the opposite rule gives 0.020, equal
    transverse weights 0.0029 (largest 0.019), and the centred-columns candidate is exact
    wherever it is chosen."""
    rng = random.Random(1)
    errs = []
    exact_cs = n_cs = 0
    while len(errs) < 6000:
        g = [rng.gauss(0.0, 1.0) for _ in range(3)]
        s = sum(abs(x) for x in g)
        n = [Fraction(round(x / s * 1024), 1024) for x in g]
        L1 = sum(abs(v) for v in n)
        if L1 == 0:
            continue
        lo = sum(v for v in n if v < 0)
        alpha0 = lo + L1 * Fraction(rng.randint(1, 1023), 1024)
        b = _block(n, alpha0)
        if not (0 < b[1, 1, 1] < 1):
            continue
        m, used_cs = oracle.myc_normal(b)
        err = float(np.max(np.abs(m - np.array([float(v / L1) for v in n]))))
        errs.append(err)
        if used_cs:
            n_cs += 1
            exact_cs += err < 1e-14
    errs = np.array(errs)
    assert errs.mean() <= 0.0015, errs.mean()
    assert errs.max() <= 0.011, errs.max()
    assert n_cs > 0 and exact_cs / n_cs > 0.65
