"""Pins of the second trigger of the height-function fallback: a 3x3x3 block
that holds two interfaces.

The reading: on the block as canonicalised (complemented when its centre
exceeds 1/2), MYC's centred-columns orientation sigma along the first axis
the height functions try (largest |m_d|, ties to the lower axis) disagrees
with the orientation the height functions take there (the full end on the
low side when m_d >= 0). A single planar interface gives the same side both
ways; a second interface in the block can turn the column sums against the
normal.
"""
import random
from fractions import Fraction

import numpy as np

import oracle
from exact_geometry import cube_cut_volume
from paper_2407_07463_amd import synth
from test_oracle_mlp import _apply, _symmetries


def _hand_block():
    """b[az][ay][ax]. Low layer (ax = -1): the centre row and its four edge neighbours full
    (Youngs weight 4 + 4 * 2 = 12, count 5). High layer (ax = +1): the rows ay = -1 and ay = +1
    full (weight 2 * (1 + 2 + 1) = 8, count 6). Middle layer: the centre 0.2 and (ay = +1,
    az = 0) 0.3."""
    b = np.zeros((3, 3, 3))
    for ay, az in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
        b[az + 1, ay + 1, 0] = 1.0
    for ay in (-1, 1):
        for az in (-1, 0, 1):
            b[az + 1, ay + 1, 2] = 1.0
    b[1, 1, 1] = 0.2
    b[1, 2, 1] = 0.3
    return b


def test_hand_worked_block_holds_two_interfaces():
    """Gx = 8 - 12 = -4; Gy = w(0)w(0)(0.3 - 0) = 1.2 (every other pair cancels); Gz = 0; so
    Youngs gives -G/|G|_1 = (10/13, -3/13, 0), quality 10/13. Centred columns along x: the
    transverse column sums are 2.3 and 2 along y, 1 and 1 along z, so D = 1.15 and the quality
    1/1.15 = 0.870 > 10/13 (along y D = 1.5, along z D = 2.65): Youngs is chosen. Its largest
    component is x, positive: full end on the low side. The column sums along x are 5 (low)
    and 6 (high): sigma_x = -1. The two disagree."""
    b = _hand_block()
    m, used_cs = oracle.myc_normal(b)
    assert not used_cs
    assert np.max(np.abs(m - np.array([10.0 / 13.0, -3.0 / 13.0, 0.0]))) <= 4 * np.spacing(1.0)
    assert oracle.two_interfaces(b)
    # the same block with the middle layer's off-centre value removed: Youngs is (1, 0, 0),
    # centred columns (quality 1) are kept with sigma_x = -1, so the normal itself points to the
    # fuller side and the orientations agree
    b2 = b.copy()
    b2[1, 2, 1] = 0.0
    m2, cs2 = oracle.myc_normal(b2)
    assert cs2 and m2[0] == -1.0
    assert not oracle.two_interfaces(b2)


def _plane_block(n, alpha0):
    b = np.zeros((3, 3, 3))
    for az in (-1, 0, 1):
        for ay in (-1, 0, 1):
            for ax in (-1, 0, 1):
                a = alpha0 - (n[0] * ax + n[1] * ay + n[2] * az)
                b[az + 1, ay + 1, ax + 1] = float(cube_cut_volume(n, a))
    return b


def test_single_planes_never_flag():
    """One planar interface with any normal and offset through the centre cell, exact
    fractions: the column sums along any axis with n_d != 0 are larger on the side the plane
    leaves full, and MYC's largest component has the sign of n there."""
    rng = random.Random(7)
    seen = 0
    while seen < 3000:
        g = [rng.gauss(0.0, 1.0) for _ in range(3)]
        s = sum(abs(x) for x in g)
        n = [Fraction(round(x / s * 1024), 1024) for x in g]
        L1 = sum(abs(v) for v in n)
        if L1 == 0:
            continue
        lo = sum(v for v in n if v < 0)
        b = _plane_block(n, lo + L1 * Fraction(rng.randint(1, 1023), 1024))
        if not (0 < b[1, 1, 1] < 1):
            continue
        assert not oracle.two_interfaces(b), n
        seen += 1


def _blocks_of(c, cells):
    out = []
    for k, j, i in cells:
        out.append(np.take(np.take(np.take(c, range(k - 1, k + 2), 0, mode="wrap"),
                                   range(j - 1, j + 2), 1, mode="wrap"), range(i - 1, i + 2), 2, mode="wrap"))
    return out


def test_spheres_and_close_sphere_pairs_never_flag():
    """Every interface cell of single spheres (R = 3..10) and of pairs of spheres (radii 2 to 12)
    whose surfaces are 0.2 to 2.5 cells apart: no flag. In the gap the low and high sides of
    the block both hold fluid, but the column sums and Youngs' weighted differences see the
    same imbalance; only blocks built for it, like the one above, turn them apart. (So the
    trigger seldom acts: measured 0 of 102,506 interface cells over 72 such pairs.)"""
    rng = synth.Splitmix64(11)
    for R in (3.0, 4.5, 6.0, 10.0):
        L = int(2 * R + 8)
        ctr = np.array([L / 2.0] * 3) + rng.uniform(3)
        c = synth.fill_spheres((L, L, L), 1, ctr[None], [R], [0])[0]
        cells = np.argwhere((c > 1e-12) & (c < 1 - 1e-12))
        assert not any(oracle.two_interfaces(b) for b in _blocks_of(c, cells)), R
    L = 32
    for R1, R2 in ((2.0, 6.0), (3.0, 3.0), (4.0, 12.0)):
        for gap in (0.2, 0.8, 1.8):
            a = np.array([16.0 - R1 - gap / 2, 16.3 + 0.7, 15.8])
            b_ = np.array([16.0 + R2 + gap / 2, 16.3, 15.8])
            c = synth.fill_spheres((L, L, L), 2, np.stack([a, b_]), [R1, R2], [0, 0])
            c = np.minimum(c[0] + c[1], 1.0)
            cells = np.argwhere((c > 1e-12) & (c < 1 - 1e-12))
            assert not any(oracle.two_interfaces(blk) for blk in _blocks_of(c, cells)), (R1, R2, gap)


def _perturbed_hand_blocks(n, seed):
    """The hand-worked block with every value moved by up to 0.05 (kept in [0, 1]): flagged and
    unflagged cases around the construction."""
    rng = np.random.default_rng(seed)
    out = []
    base = _hand_block()
    for _ in range(n):
        out.append(np.clip(base + rng.uniform(-0.05, 0.05, base.shape), 0.0, 1.0))
    return out


def test_flag_invariant_under_the_cube_group_and_the_phase_exchange():
    """The predicate is defined on the canonicalised block, so every symmetry of the cube and the
    exchange c -> 1 - c leave it unchanged (blocks with ties between the normal's components
    excluded)."""
    blocks = [_hand_block()] + _perturbed_hand_blocks(80, 3)
    rng = random.Random(5)
    while len(blocks) < 121:
        n = [Fraction(rng.randint(-64, 64), 64) for _ in range(3)]
        L1 = sum(abs(v) for v in n)
        if L1 == 0:
            continue
        b = _plane_block(n, sum(v for v in n if v < 0) + L1 * Fraction(rng.randint(1, 63), 64))
        if 0 < b[1, 1, 1] < 1:
            blocks.append(b)
    n_true = 0
    for b in blocks:
        m, _ = oracle.myc_normal(b)
        a = np.sort(np.abs(m))
        if a[2] - a[1] <= 1e-9 or abs(b[1, 1, 1] - 0.5) <= 1e-9:
            continue
        f = oracle.two_interfaces(b)
        n_true += f
        for perm, flips in _symmetries():
            assert oracle.two_interfaces(_apply(b, perm, flips)) == f
        assert oracle.two_interfaces(1.0 - b) == f
    assert 0 < n_true < len(blocks)
