"""Pins of the oracle's nearest-particle statistics.

Section "Nearest particle statistics": eq. (4) defines P_nst with the tie
weight h_ij = 1/N_i, the unnumbered normalisation says P_nst integrates to
one, eqs. (8) and (10) are the histogram estimators, and eqs. (11) and (14)
define the first and second moments M and R (A = R - tr(R)/3 delta). The
pins: the definition by brute force, a cubic lattice (exact ties, M = 0,
R = a^2/3 delta), the normalisation sum_k E_k = E, uniform random points
(E[r^2] of the Poisson nearest-neighbour law) and the dilute-limit mean
square distance r_m of eq. (15).
"""
import math

import numpy as np
import pytest
from scipy.special import gamma, gammaincc

import oracle
from paper_2407_07463_amd import synth

FIX = oracle.FIXED_ONE


def edges(nr, rmax, nth):
    r = np.linspace(0.0, rmax, nr + 1)
    th = np.linspace(0.0, math.pi, nth + 1)
    return r * r, np.cos(th)


def brute(xyz, L):
    n = len(xyz)
    out = []
    for i in range(n):
        r = xyz - xyz[i]
        r = np.where(r > L / 2, r - L, np.where(r <= -L / 2, r + L, r))
        d2 = (r[:, 0] ** 2 + r[:, 1] ** 2) + r[:, 2] ** 2
        d2[i] = np.inf
        m = d2.min()
        js = np.nonzero(d2 == m)[0]
        out.append((js, r[js], m))
    return out


def test_brute_force_definition():
    rng = synth.Splitmix64(17)
    n = 300
    L = np.array([40.0, 50.0, 60.0])
    xyz = rng.uniform(3 * n).reshape(n, 3) * L
    r2e, ce = edges(16, 20.0, 8)
    st = oracle.nearest_pair_stats(xyz, L, 2, r2e, ce)
    ref = brute(xyz, L)
    M = np.zeros(3)
    R = np.zeros((3, 3))
    for i, (js, rs, m) in enumerate(ref):
        assert st["nn_index"][i] == js[0] and st["nn_ties"][i] == len(js)
        for r in rs:
            M += r / len(js)
            R += np.outer(r, r) / len(js)
    assert np.allclose(st["M"], M / n, rtol=0, atol=1e-12)
    assert np.allclose(st["R"], R / n, rtol=1e-13, atol=0)
    # bins by explicit angle and radius (no ties on bin edges for random input)
    hist = np.zeros((16, 8), dtype=np.int64)
    over = 0
    for i, (js, rs, m) in enumerate(ref):
        for r in rs:
            d = math.sqrt(m)
            k = int(d / (20.0 / 16))
            th = math.acos(max(-1.0, min(1.0, r[2] / d)))
            mm = min(int(th / (math.pi / 8)), 7)
            if k >= 16:
                over += FIX // len(js)
            else:
                hist[k, mm] += FIX // len(js)
    assert np.array_equal(st["hist"].astype(np.int64), hist) and st["overflow"] == over
    assert int(st["hist"].sum()) + st["overflow"] == FIX * n  # P_nst integrates to one


def test_cubic_lattice_ties_and_moments():
    a = 8.0
    g = np.arange(5) * a
    xyz = np.array([(x, y, z) for z in g for y in g for x in g])
    L = np.array([40.0, 40.0, 40.0])
    r2e, ce = edges(4, 16.0, 6)
    st = oracle.nearest_pair_stats(xyz, L, 2, r2e, ce)
    assert np.all(st["nn_ties"] == 6)
    assert np.all(st["M"] == 0.0)
    assert np.allclose(st["R"], np.eye(3) * a * a / 3, rtol=1e-13, atol=0)
    A = st["R"] - np.trace(st["R"]) / 3 * np.eye(3)
    assert np.abs(A).max() < 1e-13
    # six neighbours at r = a: polar bins 0 (up), 5 (down) get 1/6 each, the equator 4/6
    k = int(np.searchsorted(r2e, a * a, side="right")) - 1
    row = st["hist"][k]
    assert row[0] == FIX // 6 * len(xyz) and row[5] == FIX // 6 * len(xyz)
    assert row[2] + row[3] == 4 * (FIX // 6) * len(xyz)


def test_uniform_points_mean_square_distance():
    """Poisson points: V = (4/3) pi n r^3 is Exp(1), so E[r^2] = Gamma(5/3) (4 pi n/3)^(-2/3)."""
    rng = synth.Splitmix64(23)
    n = 20000
    L = np.array([100.0, 100.0, 100.0])
    xyz = rng.uniform(3 * n).reshape(n, 3) * L
    r2e, ce = edges(8, 10.0, 8)
    st = oracle.nearest_pair_stats(xyz, L, 2, r2e, ce)
    dens = n / L.prod()
    lam = 4 * math.pi * dens / 3
    e_r2 = gamma(5 / 3) * lam ** (-2 / 3)
    sd = math.sqrt(gamma(7 / 3) * lam ** (-4 / 3) - e_r2**2) / math.sqrt(n)
    tr = np.trace(st["R"])
    assert abs(tr - e_r2) < 3 * sd
    A = st["R"] - tr / 3 * np.eye(3)
    assert np.abs(A).max() < 3 * 2 * sd


def test_dilute_random_spheres_r_m():
    """Eq. (15): r_m^2/d^2 = Gamma(5/3, 8 phi) e^{8 phi} / (8^{2/3} phi^{2/3}) for dilute hard
    spheres (eq. 12, accurate to O(phi)). Random sequential addition at phi = 0.01."""
    rng = synth.Splitmix64(31)
    phi, d, L = 0.01, 1.0, 40.0
    n = int(phi * L**3 / (math.pi / 6 * d**3))
    xyz = synth.rsa(rng, np.full(n, d / 2), (L, L, L), gap=0.0)
    r2e, ce = edges(8, 10.0, 8)
    st = oracle.nearest_pair_stats(xyz, np.array([L, L, L]), 2, r2e, ce)
    rm2 = gamma(5 / 3) * gammaincc(5 / 3, 8 * phi) * math.exp(8 * phi) / (8 ** (2 / 3) * phi ** (2 / 3)) * d * d
    assert np.trace(st["R"]) / rm2 == pytest.approx(1.0, abs=0.05)


def test_r_m_closed_form_values():
    """Cross-check eq. (15) against direct integration of eq. (12) (with n_p
    normalising P_nst over r > d) and the cubic-lattice spacing quoted at phi = 0.01."""
    from scipy.integrate import quad

    for phi in (0.01, 0.05, 0.1, 0.2):
        closed = gamma(5 / 3) * gammaincc(5 / 3, 8 * phi) * math.exp(8 * phi) / (8 ** (2 / 3) * phi ** (2 / 3))
        f = lambda r: math.exp(-8 * phi * (r**3 - 1))  # noqa: E731
        norm = quad(lambda r: 4 * math.pi * r * r * f(r), 1, np.inf)[0]
        mom = quad(lambda r: 4 * math.pi * r**4 * f(r), 1, np.inf)[0]
        assert mom / norm == pytest.approx(closed, rel=1e-9)
    assert 0.5 * (4 * math.pi / (3 * 0.01)) ** (1 / 3) == pytest.approx(3.7411, abs=1e-4)


def test_deviator_on_lattices():
    """A = R - tr(R)/3 delta (second-moment section). Cubic lattice: A = 0. A lattice with
    spacings (a, a, b), b > a: the four in-plane neighbours tie (h = 1/4), R = diag(a^2/2,
    a^2/2, 0), tr R = a^2 and A = diag(a^2/6, a^2/6, -a^2/3)."""
    a, b = 6.0, 9.0
    g = np.arange(4)
    xyz = np.array([(x * a, y * a, z * b) for z in g for y in g for x in g])
    L = np.array([4 * a, 4 * a, 4 * b])
    r2e, ce = edges(4, 12.0, 4)
    st = oracle.nearest_pair_stats(xyz, L, 2, r2e, ce)
    assert np.all(st["nn_ties"] == 4)
    assert np.allclose(st["R"], np.diag([a * a / 2, a * a / 2, 0.0]), rtol=0, atol=1e-12)
    assert np.allclose(st["A"], np.diag([a * a / 6, a * a / 6, -a * a / 3]), rtol=0, atol=1e-12)
    cube = np.array([(x * a, y * a, z * a) for z in g for y in g for x in g])
    st = oracle.nearest_pair_stats(cube, np.array([4 * a] * 3), 2, r2e, ce)
    assert np.abs(st["A"]).max() < 1e-12


def _poisson_points(seed, n, L):
    rng = synth.Splitmix64(seed)
    return rng.uniform(3 * n).reshape(n, 3) * L


def test_pdfs_of_uniform_points():
    """Uniform (Poisson) points: the nearest neighbour lies at r with density
    f(r) = n_p exp(-(4 pi / 3) n_p r^3) per unit volume, the same in every direction (the
    point-particle limit of eq. 12, 8 phi (r/d)^3 = (4 pi/3) n_p r^3). A radial bin therefore
    holds the fraction p_k = exp(-c r_k^3) - exp(-c r_k+1^3), c = (4 pi/3) n_p, of the events,
    and a polar bin of it the share (cos theta_m - cos theta_m+1)/2. The estimators of eqs. (8)
    and (10) at the bin centres must equal those fractions divided by 4 pi r_c^2 dr (and by
    2 pi r_c^2 sin(theta_c) dr dtheta) within counting noise; away from r = 0 they also follow
    f(r_c) up to the midpoint error."""
    n, L = 20000, 100.0
    xyz = _poisson_points(41, n, L)
    npd = n / L**3
    cc = 4 * math.pi / 3 * npd
    rmean = gamma(4 / 3) * cc ** (-1 / 3)
    nr, nth = 16, 6
    r_edges = np.linspace(0.0, 2.5 * rmean, nr + 1)
    th_edges = np.linspace(0.0, math.pi, nth + 1)
    st = oracle.nearest_pair_stats(xyz, np.array([L] * 3), 2, r_edges**2, np.cos(th_edges))
    P, Pr = oracle.pair_pdfs(r_edges, th_edges, st["hist"], n)
    rc = 0.5 * (r_edges[1:] + r_edges[:-1])
    dr = np.diff(r_edges)
    pk = np.exp(-cc * r_edges[:-1] ** 3) - np.exp(-cc * r_edges[1:] ** 3)
    expect = pk / (4 * math.pi * rc**2 * dr)
    ok = pk * n > 20
    assert ok.sum() >= 12
    sig = expect[ok] / np.sqrt(pk[ok] * n)
    assert np.all(np.abs(Pr[ok] - expect[ok]) <= 4 * sig), Pr[ok] / expect[ok]
    # the radial estimator approximates the density itself once r_c >> dr
    f = npd * np.exp(-cc * rc**3)
    far = ok & (np.arange(nr) >= 3)
    assert np.all(np.abs(Pr[far] - f[far]) <= 4 * f[far] / np.sqrt(pk[far] * n) + 0.01 * f[far])
    # the (r, theta) estimator: isotropic shares of each radial bin
    share = 0.5 * (np.cos(th_edges[:-1]) - np.cos(th_edges[1:]))
    tc = 0.5 * (th_edges[1:] + th_edges[:-1])
    for k in np.nonzero(pk * n > 1500)[0]:
        e2 = pk[k] * share / (2 * math.pi * rc[k] ** 2 * np.sin(tc) * dr[k] * np.diff(th_edges))
        assert np.all(np.abs(P[k] - e2) <= 4 * e2 / np.sqrt(pk[k] * share * n)), (k, P[k] / e2)


def test_radial_pdf_is_the_sphere_average():
    """Eq. (9): P_r-nst is the average of P_nst(r, theta, beta) over the sphere of radius r,
    (1/4 pi) int int P sin(theta) dtheta dbeta; with the azimuth integrated out it is
    (1/2) sum_m P(r, theta_m) sin(theta_m) dtheta at the same bin centres."""
    n, L = 3000, 60.0
    xyz = _poisson_points(43, n, L)
    r_edges = np.linspace(0.0, 8.0, 9)
    th_edges = np.linspace(0.0, math.pi, 9)
    st = oracle.nearest_pair_stats(xyz, np.array([L] * 3), 1, r_edges**2, np.cos(th_edges))
    P, Pr = oracle.pair_pdfs(r_edges, th_edges, st["hist"], n)
    tc = 0.5 * (th_edges[1:] + th_edges[:-1])
    avg = 0.5 * (P * np.sin(tc) * np.diff(th_edges)).sum(axis=1)
    assert np.allclose(avg, Pr, rtol=1e-13, atol=0)
    # and the binned density integrates to the fraction of events inside the radial range
    rc = 0.5 * (r_edges[1:] + r_edges[:-1])
    tot = (Pr * 4 * math.pi * rc**2 * np.diff(r_edges)).sum()
    assert tot == pytest.approx(1.0 - st["overflow"] / (FIX * n), abs=1e-13)
