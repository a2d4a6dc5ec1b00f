"""Pins of the oracle's drop labelling, drop moments and tracer recolouring.

Section "The no-coalescence.h algorithm": tag.h labels the regions bounded
by interfaces; drop properties are integrals over the cells of one tag;
Steps 1-4 detect drops of one tracer in near contact and move one of them to
a tracer used by none of the drops it touches, creating a new tracer if
needed. The near-contact figure of that section is the worked example.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from fixtures import near_contact_panels, panel_fields, random_blobs
from paper_2407_07463_amd import synth


# ------------------------------------------------------------------ labelling

def union_find_labels(mask):
    """Independent labeller: union-find over faces with periodic wrap, then
    renumber components by their smallest linear index."""
    nz, ny, nx = mask.shape
    n3 = mask.size
    parent = list(range(n3))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    flat = mask.reshape(-1)
    for p in range(n3):
        if not flat[p]:
            continue
        i, j, k = p % nx, (p // nx) % ny, p // (nx * ny)
        for q in ((i + 1) % nx + nx * (j + ny * k), i + nx * ((j + 1) % ny + ny * k),
                  i + nx * (j + ny * ((k + 1) % nz))):
            if flat[q]:
                ra, rb = find(p), find(q)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    lab = np.zeros(n3, dtype=np.int32)
    names = {}
    for p in range(n3):
        if flat[p]:
            r = find(p)
            if r not in names:
                names[r] = len(names) + 1
            lab[p] = names[r]
    return lab.reshape(mask.shape), len(names)


@pytest.mark.parametrize("seed", range(6))
def test_label_matches_union_find(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(5, 14, 3))
    c = random_blobs(rng, shape, 1, 12)[0]
    c[rng.uniform(size=shape) < 0.02] = 1e-9  # sub-threshold flotsam must not bridge
    lab, k = oracle.label(c, 1e-6)
    ref, kr = union_find_labels(c > 1e-6)
    assert k == kr
    assert np.array_equal(lab, ref)


def test_label_near_contact_figure():
    p = near_contact_panels()
    c = panel_fields(p["left"], pad=(8, 8))
    lab, k = oracle.label(c[0])
    assert k == 2  # tags 1 and 2 of tracer i
    assert (lab == 1).sum() == 47 * 5 and (lab == 2).sum() == 41 * 5
    _, kj = oracle.label(c[1])
    assert kj == 1
    c = panel_fields(p["right"])
    _, k = oracle.label(c[0])
    assert k == 1  # one region, connected through the periodic boundaries


def test_label_canonical_order_and_wrap():
    c = np.zeros((4, 6, 8))
    c[0, 0, 7] = 0.5
    c[0, 0, 0] = 0.5  # joined to the previous one across x
    c[2, 3, 3] = 0.2
    lab, k = oracle.label(c)
    assert k == 2
    assert lab[0, 0, 0] == 1 and lab[0, 0, 7] == 1 and lab[2, 3, 3] == 2


# ------------------------------------------------------------------ moments

def test_moments_sphere_centroid_and_volume():
    n = 32
    # symmetric placements (centre at a cell centre or a cell corner) make the
    # cell-centre-weighted centroid exact; the second sphere straddles the box corner
    for centre, R in (((10.5, 12.5, 15.5), 5.5), ((0.0, 31.0, 16.0), 6.2), ((0.5, 0.0, 31.5), 4.3)):
        c = synth.fill_spheres((n, n, n), 1, [centre], [R], [0])[0]
        lab, k = oracle.label(c)
        assert k == 1
        vol, xyz, rc = oracle.drop_moments(c, lab, k)
        assert rc == 0
        # cells at or below c_eps = 1e-6 are not part of the drop: slivers of ~1e-6 are left out
        assert vol[0] == pytest.approx(c[lab == 1].sum(), rel=1e-13)
        assert vol[0] == pytest.approx(4 / 3 * math.pi * R**3, rel=1e-7)
        d = (xyz[0] - np.array(centre) + n / 2) % n - n / 2
        assert np.abs(d).max() < 1e-10
        # centroid of the labelled cells computed directly with unwrapped coordinates
        zz, yy, xx = np.nonzero(lab == 1)
        w = c[zz, yy, xx]
        for a, (coord, ctr) in enumerate(zip((xx, yy, zz), centre)):
            u = (coord + 0.5 - ctr + n / 2) % n - n / 2 + ctr
            assert ((w * u).sum() / w.sum() - xyz[0][a] + n / 2) % n - n / 2 == pytest.approx(0, abs=1e-11)


def test_moments_extent_error():
    c = np.zeros((4, 4, 16))
    c[1, 1, :9] = 1.0  # spans 9 >= 16/2 cells along x
    lab, k = oracle.label(c)
    _, _, rc = oracle.drop_moments(c, lab, k)
    assert rc == oracle.E_EXTENT


# ------------------------------------------------------------------ recolouring

def _min_image_d2(p, q, shape):
    d2 = 0
    for a, b, n in zip(p, q, shape):
        d = abs(a - b) % n
        d = min(d, n - d)
        d2 += d * d
    return d2


def _brute_neighbours(labels, tau):
    """All pairs of distinct drops with occupied cells closer than (1+tau), by brute force."""
    ntr = labels.shape[0]
    shape = labels.shape[1:]
    cells = []
    offs = [0]
    for t in range(ntr):
        k = labels[t].max()
        offs.append(offs[-1] + k)
    for t in range(ntr):
        for idx in zip(*np.nonzero(labels[t])):
            cells.append((offs[t] + labels[t][idx] - 1, idx))
    lim = (1 + tau) ** 2
    pairs = set()
    for (ga, pa), (gb, pb) in itertools.combinations(cells, 2):
        if ga != gb and _min_image_d2(pa, pb, shape) < lim:
            pairs.add((min(ga, gb), max(ga, gb)))
    return pairs


@pytest.mark.parametrize("seed", range(4))
def test_neighbours_match_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    shape = (7, 9, 11)
    c = random_blobs(rng, shape, 3, 10, 0.8, 1.8)
    labels = np.stack([oracle.label(c[t])[0] for t in range(3)])
    nd = labels.reshape(3, -1).max(1)
    pairs = oracle.neighbour_pairs(labels, nd, 1.5)
    got = {(int(a), int(b)) for a, b in pairs if a < b}
    assert got == _brute_neighbours(labels, 1.5)
    # symmetric
    assert {(int(b), int(a)) for a, b in pairs if a > b} == got


def _check_recolour(c0, labels, nd, ntr, newt, ntr_new, c1, tau):
    D = int(nd.sum())
    offs = np.concatenate([[0], np.cumsum(nd)])
    tracer0 = np.repeat(np.arange(ntr), nd)
    brute = _brute_neighbours(labels, tau)
    # proper colouring: no two neighbouring drops share a tracer
    for a, b in brute:
        assert newt[a] != newt[b]
    # a drop that touches no other drop never moves
    for g in range(D):
        if newt[g] != tracer0[g]:
            assert any(g in pr for pr in brute)
    # cell values move with their drop; the total is conserved cell by cell
    assert np.allclose(c1.sum(0), c0.sum(0), rtol=0, atol=1e-15)
    moved_in = np.zeros(c1.shape, dtype=bool)
    for t in range(ntr):
        for g in range(offs[t], offs[t + 1]):
            cells = labels[t] == g - offs[t] + 1
            assert np.all(c1[newt[g]][cells] >= c0[t][cells])
            if newt[g] != t:
                moved_in[newt[g]][cells] = True
    for t in range(ntr):
        for g in range(offs[t], offs[t + 1]):
            cells = (labels[t] == g - offs[t] + 1) & ~moved_in[t]
            if newt[g] != t:
                assert np.all(c1[t][cells] == 0)
    assert ntr_new >= ntr


@pytest.mark.parametrize("seed", range(5))
def test_recolour_random_tiny_grids(seed):
    rng = np.random.default_rng(200 + seed)
    shape = (8, 9, 10)
    ntr, maxt = 2, 8
    c = np.zeros((maxt,) + shape)
    c[:ntr] = random_blobs(rng, shape, ntr, 12, 0.8, 1.6)
    labels = np.stack([oracle.label(c[t])[0] for t in range(ntr)])
    nd = labels.reshape(ntr, -1).max(1).astype(np.int32)
    c1, ntr_new, newt, nmoved, rc = oracle.recolor(c, labels, nd, ntr, maxt, 1.5)
    assert rc == 0
    assert nmoved == int((newt != np.repeat(np.arange(ntr), nd)).sum())
    _check_recolour(c, labels, nd, ntr, newt, ntr_new, c1, 1.5)


def test_recolour_near_contact_figure_left():
    p = near_contact_panels()
    c2 = panel_fields(p["left"], pad=(8, 8))
    maxt = 4
    c = np.zeros((maxt,) + c2.shape[1:])
    c[:2] = c2
    labels = np.stack([oracle.label(c[t])[0] for t in range(2)])
    nd = np.array([2, 1], dtype=np.int32)
    # the figure's gap between drops 1 and 2 is sqrt(17) cells centre to centre:
    # a threshold tau with (1+tau)^2 > 17 declares them in near contact
    c1, ntr, newt, nmoved, rc = oracle.recolor(c, labels, nd, 2, maxt, 3.2)
    assert rc == 0
    assert list(newt) == [0, 2, 1] and ntr == 3 and nmoved == 1
    assert np.array_equal(c1[2], np.where(labels[0] == 2, 1.0, 0.0))
    # with a smaller threshold the two drops are not in near contact
    c1, ntr, newt, nmoved, rc = oracle.recolor(c, labels, nd, 2, maxt, 3.0)
    assert nmoved == 0 and ntr == 2
    # capacity exceeded: nothing changes, error returned
    c1, ntr, newt, nmoved, rc = oracle.recolor(c[:2], labels, nd, 2, 2, 3.2)
    assert rc == oracle.E_CAPACITY


def test_recolour_near_contact_figure_right():
    p = near_contact_panels()
    c2 = panel_fields(p["right"])
    c = np.zeros((3,) + c2.shape[1:])
    c[:2] = c2
    labels = np.stack([oracle.label(c[t])[0] for t in range(2)])
    nd = labels.reshape(2, -1).max(1).astype(np.int32)
    assert list(nd) == [1, 0]
    c1, ntr, newt, nmoved, rc = oracle.recolor(c, labels, nd, 2, 3, 3.2)
    assert rc == 0 and nmoved == 0 and ntr == 2
    assert np.array_equal(c1, c)


def test_compact_tracers_pins():
    """Tracers 1 and 3 hold no drop, only dust of known size: they are
    retired, 0, 2, 4 move to 0, 1, 2 unchanged, the freed fields are zero,
    and the discarded volume is the dust's (exactly representable sums)."""
    shape = (4, 5, 6)
    c = np.zeros((5,) + shape)
    c[0, 1, 1, 1:4] = [0.5, 1.0, 0.25]
    c[2, 3, 2, 2] = 0.75
    c[4, 0, 4, 5] = 1.0
    c[1, 2, 2, 2] = 2.0 ** -30  # dust below the labelling threshold
    c[3, 0, 0, 0] = 2.0 ** -31
    nd = [oracle.label(c[t])[1] for t in range(5)]
    assert nd == [1, 0, 1, 0, 1]
    out, n, idx, disc = oracle.compact_tracers(c, nd)
    assert n == 3 and list(idx) == [0, -1, 1, -1, 2]
    assert np.array_equal(out[0], c[0]) and np.array_equal(out[1], c[2]) and np.array_equal(out[2], c[4])
    assert not out[3:].any()
    assert disc == 2.0 ** -30 + 2.0 ** -31
    # nothing to retire; everything retired
    out, n, idx, disc = oracle.compact_tracers(c[[0, 2]], [1, 1])
    assert n == 2 and list(idx) == [0, 1] and disc == 0.0 and np.array_equal(out, c[[0, 2]])
    out, n, idx, disc = oracle.compact_tracers(c[[1, 3]], [0, 0])
    assert n == 0 and list(idx) == [-1, -1] and not out.any() and disc == 2.0 ** -30 + 2.0 ** -31
