"""Pins of the oracle's literal near-contact mode (Steps 1-4 of section "The
no-coalescence.h algorithm", the near-contact criterion figure).

Step 1 flags an empty centre cell with two opposite occupied cells in the
5x5(x5) stencil; Step 3 keeps the flag only when the two cells carry
different tags; Step 4 moves a later drop of each flagged pair to a tracer
that no drop in contact with it holds (contact across tracers: within the
stencil's reach of 4 cells along every axis, a reading). The pins: the
figure's two panels, the reach of the criterion along an axis and along a
diagonal (it sees gaps of at most 3 empty cells, and only offsets that an
integer centre halves), and a proper colouring after the pass.
"""
import numpy as np
import pytest

import oracle
from fixtures import near_contact_panels, panel_fields, random_blobs


def _labels(c, ntr):
    ls = [oracle.label(c[t]) for t in range(ntr)]
    return np.stack([l for l, _ in ls]), np.array([k for _, k in ls], dtype=np.int32)


def test_figure_left_flags_exactly_the_drawn_centres():
    """Left panel, embedded in an empty border (the figure is not periodic): the criterion of
    Steps 1 and 3 holds at exactly three centres, x = 10 and y = 4, 5, 6, between tag 1 and
    tag 2 -- e.g. centre (10, 4) with the pairs (8, 3)/(12, 5) and (8, 2)/(12, 6)."""
    p = near_contact_panels()
    c = panel_fields(p["left"], pad=(8, 8), nz=5)
    lab, nd = _labels(c, 2)
    assert list(nd) == [2, 1]
    f = oracle.stencil_flags(lab[0])
    for z in range(c.shape[1]):
        assert sorted(zip(*np.nonzero(f[z] == 2)[::-1])) == [(10, 4), (10, 5), (10, 6)]
        assert sorted(zip(*np.nonzero(f[z] >= 1)[::-1])) == [(10, 4), (10, 5), (10, 6)]
    assert lab[0][0, 3, 8] != lab[0][0, 5, 12] and lab[0][0, 3, 8] > 0 and lab[0][0, 5, 12] > 0
    assert lab[0][0, 4, 10] == 0


def test_figure_left_moves_drop_2_to_a_new_tracer():
    """Step 4 on the left panel: drop 2 (later in the visiting order) conflicts with drop 1,
    and it overlaps tracer j, so neither i nor j will do: a new tracer is created."""
    p = near_contact_panels()
    c2 = panel_fields(p["left"], pad=(8, 8), nz=5)
    maxt = 4
    c = np.zeros((maxt,) + c2.shape[1:])
    c[:2] = c2
    lab, nd = _labels(c, 2)
    c1, ntr, newt, nmoved, rc = oracle.recolor_stencil(c, lab, nd, 2, maxt)
    assert rc == 0
    assert list(newt) == [0, 2, 1] and ntr == 3 and nmoved == 1
    assert np.array_equal(c1[2], np.where(lab[0] == 2, 1.0, 0.0))
    assert np.array_equal(c1[0], np.where(lab[0] == 1, 1.0, 0.0))
    assert np.array_equal(c1[1], c[1])
    # without room for a third tracer: capacity error, nothing returned changed
    _, _, _, _, rc = oracle.recolor_stencil(c[:2], lab, nd, 2, 2)
    assert rc == oracle.E_CAPACITY


def test_figure_right_rejected_by_step_3():
    """Right panel: one region close to itself. Step 1 holds at several centres of its
    concave bay, Step 3 at none (one tag), so nothing moves."""
    p = near_contact_panels()
    c2 = panel_fields(p["right"], pad=(8, 8), nz=5)
    c = np.zeros((3,) + c2.shape[1:])
    c[:2] = c2
    lab, nd = _labels(c, 2)
    assert list(nd) == [1, 0]
    f = oracle.stencil_flags(lab[0])
    assert np.count_nonzero(f == 1) >= 5 * 5 and not np.any(f == 2)
    c1, ntr, newt, nmoved, rc = oracle.recolor_stencil(c, lab, nd, 2, 3)
    assert rc == 0 and nmoved == 0 and ntr == 2 and np.array_equal(c1, c)


@pytest.mark.parametrize("gap", [1, 2, 3, 4, 5])
def test_reach_along_an_axis(gap):
    """Two thick slabs of one tracer `gap` empty cells apart (the other way round the periodic
    box far away): the opposite cells of a 5-cell stencil are at most 4 apart, so the slabs are
    in near contact exactly when gap <= 3, at every gap parity (an odd distance is bridged by a
    pair one cell further in)."""
    nx = 40
    c = np.zeros((2, 4, 4, nx))
    c[0, :, :, 0:10] = 1.0
    c[0, :, :, 10 + gap:20 + gap] = 1.0
    lab, nd = _labels(c, 1)
    assert nd[0] == 2
    flagged = np.any(oracle.stencil_flags(lab[0]) == 2)
    assert flagged == (gap <= 3)
    c1, ntr, newt, nmoved, rc = oracle.recolor_stencil(c, lab, nd, 1, 2)
    assert rc == 0 and nmoved == (1 if gap <= 3 else 0)


def test_reach_along_a_diagonal_and_odd_offsets():
    """Single occupied cells: offset (4, 4, 4) has the empty integer centre (2, 2, 2) -> near
    contact; offset (4, 4, 2) -> near contact; (5, 4, 4) has no integer centre within the
    stencil and (3, 1, 0) none at all (the criterion sees only even offsets): no contact."""
    def pair(off):
        c = np.zeros((1, 16, 16, 16))
        c[0, 4, 4, 4] = 1.0
        c[0, 4 + off[2], 4 + off[1], 4 + off[0]] = 1.0
        lab, nd = _labels(c, 1)
        assert nd[0] == 2
        return bool(np.any(oracle.stencil_flags(lab[0]) == 2))

    assert pair((4, 4, 4)) and pair((4, 4, 2)) and pair((2, 0, 0)) and pair((-4, 2, 0))
    assert not pair((5, 4, 4)) and not pair((3, 1, 0)) and not pair((6, 0, 0)) and not pair((1, 1, 1))


def test_contact_across_tracers_decides_the_new_tracer():
    """Drops 0:1 and 0:2 are in near contact (gap 3 along x); drop 1:1 lies 4 cells from 0:2
    along every axis (within reach) and 2:1 five cells along one axis (out of reach). Drop 0:2
    moves, not to tracer 1 (in contact), but to tracer 2 (free of contact)."""
    c = np.zeros((4, 24, 24, 24))
    c[0, 4:7, 4:7, 2:5] = 1.0      # drop 0:1, x in [2, 5)
    c[0, 4:7, 4:7, 8:11] = 1.0     # drop 0:2, x in [8, 11): gap 3
    c[1, 10, 10, 14] = 1.0         # tracer 1: (14,10,10) - (10,6,6) = (4,4,4): in reach
    c[2, 6, 6, 16] = 1.0           # tracer 2: (16,6,6) - (10,6,6) = (6,0,0): out of reach
    lab, nd = _labels(c, 3)
    assert list(nd) == [2, 1, 1]
    c1, ntr, newt, nmoved, rc = oracle.recolor_stencil(c, lab, nd, 3, 4)
    assert rc == 0 and nmoved == 1 and ntr == 3
    assert list(newt) == [0, 2, 1, 2]
    assert np.array_equal(c1[2], c[2] + np.where(lab[0] == 2, 1.0, 0.0))


@pytest.mark.parametrize("seed", range(4))
def test_pass_leaves_a_proper_colouring(seed):
    """After one pass no tracer holds two drops in near contact: a moved drop avoids the
    tracers of every drop within reach (which includes every drop it could conflict or merge
    with), so the re-labelled fields show no Step-3 flag anywhere. Volume is unchanged, every
    drop's cells sit in its new tracer, and the number of moves is the number of drops whose
    tracer changed."""
    rng = np.random.default_rng(300 + seed)
    shape = (10, 11, 12)
    ntr, maxt = 2, 12
    c = np.zeros((maxt,) + shape)
    c[:ntr] = random_blobs(rng, shape, ntr, 14, 0.8, 1.8)
    lab, nd = _labels(c, ntr)
    c1, ntr1, newt, nmoved, rc = oracle.recolor_stencil(c, lab, nd, ntr, maxt)
    assert rc == 0
    assert c1.sum() == pytest.approx(c.sum(), rel=1e-15)
    assert nmoved == int((newt != np.repeat(np.arange(ntr), nd)).sum())
    # every drop's cells sit, unchanged, in its new tracer
    off = np.concatenate([[0], np.cumsum(nd)])
    for t in range(ntr):
        for l in range(1, nd[t] + 1):
            n = newt[off[t] + l - 1]
            m = lab[t] == l
            assert np.all(c1[n][m] >= c[t][m])
    # no conflict left: the drops of each new tracer, re-labelled, are never in near contact
    lab1, nd1 = _labels(c1, ntr1)
    for t in range(ntr1):
        assert not np.any(oracle.stencil_flags(lab1[t]) == 2), (seed, t)
    # the edge list is symmetric and relates drops of one tracer only through Steps 1-3
    pairs = oracle.neighbour_pairs_stencil(lab, nd)
    s = {(int(a), int(b)) for a, b in pairs}
    assert all((b, a) in s for a, b in s)
