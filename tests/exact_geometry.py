"""Exact rational geometry used to pin the oracle (test code only).

`cube_cut_volume` is the volume of {x in [0,1]^3 : m.x <= alpha} written as
the inclusion-exclusion sum over the cube's vertices, evaluated in exact
rational arithmetic. It is an independent route to the quantity the oracle
computes with a piecewise closed form, so a dropped term, a wrong sign or a
swapped index in the oracle shows up as a mismatch here.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction


def cube_cut_volume(m, alpha) -> Fraction:
    """Exact volume of {x in [0,1]^k : m.x <= alpha} for rational inputs."""
    m = [Fraction(v) for v in m]
    alpha = Fraction(alpha)
    # reflect negative components: x_i -> 1 - x_i
    for i, v in enumerate(m):
        if v < 0:
            alpha -= v
            m[i] = -v
    pos = [v for v in m if v != 0]
    k = len(pos)
    if k == 0:
        return Fraction(1) if alpha >= 0 else Fraction(0)
    total = Fraction(0)
    for r in range(k + 1):
        for S in itertools.combinations(range(k), r):
            t = alpha - sum((pos[i] for i in S), Fraction(0))
            if t > 0:
                total += (-1) ** r * t**k
    prod = Fraction(1)
    for v in pos:
        prod *= v
    vol = total / (math.factorial(k) * prod)
    return min(max(vol, Fraction(0)), Fraction(1))


def slab_fraction(cell, normal, lo, hi, period_shift=None, shifts=(0,)) -> Fraction:
    """Exact fraction of cell (i,j,k) inside {lo <= n.x <= hi + s} union over shifts.

    `normal` is rational; the region is the union over integer multiples s in
    `shifts` of {lo + s <= n.x <= hi + s}; the slabs must not overlap.
    """
    i, j, k = cell
    n = [Fraction(v) for v in normal]
    base = n[0] * i + n[1] * j + n[2] * k
    tot = Fraction(0)
    for s in shifts:
        a = Fraction(lo) + s - base
        b = Fraction(hi) + s - base
        tot += cube_cut_volume(n, b) - cube_cut_volume(n, a)
    return tot
