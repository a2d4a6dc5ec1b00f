"""Seeded synthetic workloads: drop fields and prescribed velocity fields.

Both the HIP path and the CPU oracle consume exactly the arrays built here;
this module contains none of the Volume-of-Fluid method's own arithmetic
(no reconstruction, no plane/cube volume, no flux, no labelling).

Inputs follow the paper's setting (Numerical method section): monodisperse
spherical drops in a tri-periodic cubic box, all units in cells. The drops
are placed by random sequential addition with a minimum surface gap, and
their volume fractions are integrated accurately (error well below 1e-9 per
cell at the default quadrature order), which the curvature tests require.

Velocities are face Courant numbers s_d (cells per step) stored at the lower
d-face of each cell, s_d[z][y][x], discretely divergence-free:
  - `abc_velocity`: an Arnold-Beltrami-Childress flow plus a uniform rise,
    whose staggered samples have exactly zero discrete divergence;
  - `fourier_velocity`: a random solenoidal field with E(k) ~ k^(-5/3) on
    integer modes 1 <= |k| <= kmax, projected perpendicular to the modified
    wavenumber 2 sin(pi k_d / n_d) so the staggered divergence vanishes to
    round-off, plus a uniform rise.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def lib():
    """Load the in-tree generator library (built by the package build step)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(_LIB_PATH)
        L.synth_uniform.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64, ctypes.c_void_p]
        L.synth_uniform.restype = None
        L.synth_rsa.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int64, ctypes.c_void_p]
        L.synth_rsa.restype = ctypes.c_int
        L.synth_fill_ellipsoids.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int]
        L.synth_fill_ellipsoids.restype = ctypes.c_int
        L.synth_cell_fraction.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int]
        L.synth_cell_fraction.restype = ctypes.c_double
        L.synth_fill_cylinders_z.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.synth_fill_cylinders_z.restype = ctypes.c_int
        _lib = L
    return _lib


class Splitmix64:
    """splitmix64 stream (Steele, Lea & Flood 2014); doubles from the top 53 bits."""

    def __init__(self, seed: int):
        self.state = ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)

    def uniform(self, n: int) -> np.ndarray:
        out = np.empty(int(n), dtype=np.float64)
        if n > 0:
            lib().synth_uniform(ctypes.byref(self.state), int(n), out.ctypes.data)
        return out

    def normal(self, n: int) -> np.ndarray:
        """Standard normals by the Box-Muller transform, two uniforms each."""
        u = self.uniform(2 * int(n)).reshape(-1, 2)
        u1 = 1.0 - u[:, 0]  # in (0, 1]
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u[:, 1])


def workload_seed(workload: int, run: int = 0) -> int:
    return 20240710 + 1000 * workload + run


# --------------------------------------------------------------------------
# drops
# --------------------------------------------------------------------------

def rsa(rng: Splitmix64, radii, box, gap: float, max_attempts: int = 1_000_000) -> np.ndarray:
    """Random sequential addition of spheres with surface gap >= `gap` (periodic)."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    out = np.zeros((len(radii), 3), dtype=np.float64)
    lx, ly, lz = (float(b) for b in box)
    placed = lib().synth_rsa(ctypes.byref(rng.state), len(radii), radii.ctypes.data, lx, ly, lz,
                             float(gap), int(max_attempts), out.ctypes.data)
    if placed != len(radii):
        raise RuntimeError(f"random sequential addition placed only {placed} of {len(radii)} drops")
    return out


def fill_ellipsoids(shape, ntracers: int, centres, Qs, tracer_of, order: int = 16,
                    out: np.ndarray | None = None) -> np.ndarray:
    """Volume fractions of ellipsoids {(p-c)^T Q (p-c) <= 1} on a periodic grid.

    shape = (nz, ny, nx); returns (or accumulates into) float64 [ntracers, nz, ny, nx].
    """
    nz, ny, nx = (int(s) for s in shape)
    if out is None:
        out = np.zeros((ntracers, nz, ny, nx), dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == (ntracers, nz, ny, nx)
    centres = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
    Qs = np.ascontiguousarray(Qs, dtype=np.float64).reshape(-1, 3, 3)
    tracer_of = np.ascontiguousarray(tracer_of, dtype=np.int32).reshape(-1)
    assert len(centres) == len(Qs) == len(tracer_of)
    assert tracer_of.size == 0 or (tracer_of.min() >= 0 and tracer_of.max() < ntracers)
    rc = lib().synth_fill_ellipsoids(nx, ny, nz, out.ctypes.data, len(centres), centres.ctypes.data,
                                     Qs.ctypes.data, tracer_of.ctypes.data, int(order))
    if rc == -2:
        raise ValueError("a body is wider than the periodic box")
    if rc != 0:
        raise ValueError("bad quadrature order")
    return out


def fill_cylinders_z(shape, ntracers: int, centres_xy, radii, tracer_of, out: np.ndarray | None = None):
    """Exact volume fractions of infinite cylinders parallel to z."""
    nz, ny, nx = (int(s) for s in shape)
    if out is None:
        out = np.zeros((ntracers, nz, ny, nx), dtype=np.float64)
    cxy = np.ascontiguousarray(centres_xy, dtype=np.float64).reshape(-1, 2)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    t = np.ascontiguousarray(tracer_of, dtype=np.int32).reshape(-1)
    rc = lib().synth_fill_cylinders_z(nx, ny, nz, out.ctypes.data, len(r), cxy.ctypes.data, r.ctypes.data,
                                      t.ctypes.data)
    if rc != 0:
        raise ValueError("a cylinder is wider than the periodic box")
    return out


def fill_spheres(shape, ntracers: int, centres, radii, tracer_of, order: int = 16,
                 out: np.ndarray | None = None) -> np.ndarray:
    radii = np.asarray(radii, dtype=np.float64).reshape(-1)
    Qs = np.einsum("i,jk->ijk", 1.0 / radii**2, np.eye(3))
    return fill_ellipsoids(shape, ntracers, centres, Qs, tracer_of, order, out)


def cell_fraction(centre, Q, corner, order: int = 16) -> float:
    """Volume of one ellipsoid inside the unit cell whose lower corner is `corner`."""
    c = np.ascontiguousarray(centre, dtype=np.float64)
    q = np.ascontiguousarray(Q, dtype=np.float64)
    return lib().synth_cell_fraction(c.ctypes.data, q.ctypes.data, float(corner[0]), float(corner[1]),
                                     float(corner[2]), int(order))


def ellipsoid_matrix(axes, rotation) -> np.ndarray:
    """Q = R diag(1/a^2) R^T for semi-axes `axes` along the columns of `rotation`."""
    Rm = np.asarray(rotation, dtype=np.float64)
    a = np.asarray(axes, dtype=np.float64)
    return Rm @ np.diag(1.0 / a**2) @ Rm.T


def random_rotation(rng: Splitmix64) -> np.ndarray:
    """Uniform random rotation from a uniform unit quaternion (Shoemake 1992)."""
    u1, u2, u3 = rng.uniform(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    q = (a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2),
         b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3))
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# --------------------------------------------------------------------------
# velocities
# --------------------------------------------------------------------------

def abc_velocity(n: int, courant: float = 0.25, rise: float = 0.3):
    """ABC flow u = 0.5(sin2pi z + cos2pi y, sin2pi x + cos2pi z, sin2pi y + cos2pi x) + (0,0,rise)
    on the unit box, sampled at face centres and scaled so max |s| = courant.

    s_x depends on (y,z) only, s_y on (x,z), s_z on (x,y): each staggered
    difference s_d[p+e_d] - s_d[p] is exactly zero.
    """
    i = np.arange(n, dtype=np.float64)
    lo = i / n           # face coordinate
    mid = (i + 0.5) / n  # cell-centre coordinate
    two_pi = 2.0 * math.pi
    # s_x at (x=i, y=j+1/2, z=k+1/2): [z][y][x]
    ux = 0.5 * (np.sin(two_pi * mid)[:, None, None] + np.cos(two_pi * mid)[None, :, None]) + 0.0 * lo[None, None, :]
    # s_y at (x=i+1/2, y=j, z=k+1/2)
    uy = 0.5 * (np.sin(two_pi * mid)[None, None, :] + np.cos(two_pi * mid)[:, None, None]) + 0.0 * lo[None, :, None]
    # s_z at (x=i+1/2, y=j+1/2, z=k)
    uz = 0.5 * (np.sin(two_pi * mid)[None, :, None] + np.cos(two_pi * mid)[None, None, :]) + rise + 0.0 * lo[:, None, None]
    umax = max(np.abs(ux).max(), np.abs(uy).max(), np.abs(uz).max())
    scale = courant / umax
    return tuple(np.ascontiguousarray(u * scale) for u in (ux, uy, uz))


def fourier_velocity(shape, seed: int, kmax: int = 8, rms: float = 0.2, rise: float = 0.1,
                     smax: float = 0.45, workers: int | None = None):
    """Random discretely solenoidal face-Courant field plus a uniform rise along z.

    Modes: integer k with 1 <= |k| <= kmax (and |k_d| < n_d/2) in the half
    space {kx>0} U {kx=0,ky>0} U {kx=ky=0,kz>0}; for each mode and component a
    complex Gaussian amplitude of variance |k|^(-11/3) (E(k) ~ k^(-5/3)),
    projected perpendicular to kt_d = 2 sin(pi k_d/n_d). The field is
    s_d(p) = sum_k 2 Re(A_d(k) exp(2 pi i k.x_d(p)/n)) at the face centres x_d.
    The fluctuation is scaled to a per-component rms of `rms`, then reduced if
    needed so that max |s| <= smax once the rise is added. Returns (sx, sy, sz,
    realised_rms).
    """
    import scipy.fft

    nz, ny, nx = (int(s) for s in shape)
    rng = Splitmix64(seed)
    modes = []
    for kz in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kx in range(0, kmax + 1):
                k2 = kx * kx + ky * ky + kz * kz
                if k2 < 1 or k2 > kmax * kmax:
                    continue
                if not (kx > 0 or (kx == 0 and ky > 0) or (kx == 0 and ky == 0 and kz > 0)):
                    continue
                if 2 * abs(kx) >= nx or 2 * abs(ky) >= ny or 2 * abs(kz) >= nz:
                    continue
                modes.append((kx, ky, kz))
    modes = np.array(modes, dtype=np.int64).reshape(-1, 3)
    nm = len(modes)
    kk = np.sqrt((modes.astype(np.float64) ** 2).sum(1))
    sigma = kk ** (-11.0 / 6.0)  # std, variance |k|^(-11/3)
    g = rng.normal(6 * nm).reshape(nm, 3, 2)
    A = (g[..., 0] + 1j * g[..., 1]) * (sigma[:, None] / math.sqrt(2.0))
    nvec = np.array([nx, ny, nz], dtype=np.float64)
    kt = 2.0 * np.sin(math.pi * modes / nvec[None, :])
    proj = (A * kt).sum(1) / (kt * kt).sum(1)
    A = A - proj[:, None] * kt
    N = nx * ny * nz
    half = modes[:, 0] / nx + modes[:, 1] / ny + modes[:, 2] / nz
    fields = []
    for d in range(3):
        phase = np.exp(1j * math.pi * (half - modes[:, d] / nvec[d]))
        F = np.zeros((nz, ny, nx // 2 + 1), dtype=np.complex128)
        amp = A[:, d] * phase * N * np.where(modes[:, 0] == 0, 2.0, 1.0)
        np.add.at(F, (modes[:, 2] % nz, modes[:, 1] % ny, modes[:, 0]), amp)
        f = scipy.fft.irfftn(F, s=(nz, ny, nx), axes=(0, 1, 2), workers=workers)
        fields.append(np.ascontiguousarray(f))
        del F
    ms = sum(float(np.mean(f * f)) for f in fields) / 3.0
    scale = rms / math.sqrt(ms) if ms > 0 else 0.0
    # largest scale keeping max |scale*f + rise_d| <= smax on every component
    lim = scale
    for d, f in enumerate(fields):
        r = rise if d == 2 else 0.0
        fmax, fmin = float(f.max()), float(f.min())
        if fmax > 0:
            lim = min(lim, (smax - r) / fmax)
        if fmin < 0:
            lim = min(lim, (smax + r) / (-fmin))
    scale = min(scale, lim)
    out = []
    for d, f in enumerate(fields):
        f *= scale
        if d == 2:
            f += rise
        out.append(f)
    return out[0], out[1], out[2], scale * math.sqrt(ms)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def spheres64(seed: int | None = None, order: int = 16):
    """64^3 box, 2 tracers, 8 spheres of radius 6 at uniform random centres with
    surface gap >= 2, sphere k in tracer k mod 2; ABC velocity with rise 0.3 at
    Courant 0.25; 20 steps."""
    seed = workload_seed(0) if seed is None else seed
    rng = Splitmix64(seed)
    n, nd, R = 64, 8, 6.0
    radii = np.full(nd, R)
    centres = rsa(rng, radii, (n, n, n), gap=2.0)
    tr = np.arange(nd) % 2
    c = fill_spheres((n, n, n), 2, centres, radii, tr, order)
    sx, sy, sz = abc_velocity(n, 0.25, 0.3)
    return dict(name="spheres64", shape=(n, n, n), ntracers=2, c=c, sx=sx, sy=sy, sz=sz,
                centres=centres, radii=radii, tracer_of=tr, nsteps=20, seed=seed)


def random_drops(n: int, ntracers: int, phi: float, diameter: float, spread: float, gap: float,
                 seed: int, order: int = 16, kmax: int = 8, rms: float = 0.2, rise: float = 0.1,
                 workers: int | None = None, velocity: bool = True):
    """Periodic n^3 box with drops of mean diameter `diameter` (uniform relative
    spread +-`spread`) at volume fraction `phi`, placed by random sequential
    addition with surface gap `gap`; drop k in tracer k mod ntracers; random
    Fourier velocity."""
    rng = Splitmix64(seed)
    ed3 = diameter**3 * (1.0 + spread * spread) if spread > 0 else diameter**3
    nd = int(phi * n**3 / (math.pi / 6.0 * ed3) + 0.5)
    u = rng.uniform(nd) if spread > 0 else np.zeros(nd)
    radii = 0.5 * diameter * (1.0 + spread * (2.0 * u - 1.0))
    centres = rsa(rng, radii, (n, n, n), gap=gap)
    tr = np.arange(nd) % ntracers
    c = fill_spheres((n, n, n), ntracers, centres, radii, tr, order)
    out = dict(shape=(n, n, n), ntracers=ntracers, c=c, centres=centres, radii=radii, tracer_of=tr, seed=seed)
    if velocity:
        sx, sy, sz, rr = fourier_velocity((n, n, n), seed + 1, kmax=kmax, rms=rms, rise=rise, workers=workers)
        out.update(sx=sx, sy=sy, sz=sz, rms=rr)
    return out


def drops256(seed: int | None = None, **kw):
    """256^3, 8 tracers, ~400 drops of diameter 20 at phi = 0.1, gap 2; 200 steps."""
    seed = workload_seed(1) if seed is None else seed
    d = random_drops(256, 8, 0.1, 20.0, 0.0, 2.0, seed, **kw)
    d.update(name="drops256", nsteps=200)
    return d


def drops512(seed: int | None = None, **kw):
    """512^3, 8 tracers, ~5508 drops of diameter 24 +-10% at phi = 0.3, gap 1; 100 steps."""
    seed = workload_seed(2) if seed is None else seed
    d = random_drops(512, 8, 0.3, 24.0, 0.1, 1.0, seed, **kw)
    d.update(name="drops512", nsteps=100)
    return d


def batch_boxes(nboxes: int = 32, sizes=(64, 96, 128, 160, 192), seed: int | None = None,
                diameter: float = 20.0, phi_range=(0.05, 0.3), tracer_range=(2, 8), gap: float = 1.0,
                workers: int | None = None):
    """Uneven boxes for batched advection: each box is cubic with its edge drawn
    from `sizes`, 2-8 tracers and a drop volume fraction in [0.05, 0.3] (all
    drawn from one seeded stream), filled like `random_drops` (surface gap of
    1 cell, as for the 512^3 field: 2 cells jam random sequential addition
    near phi = 0.3) with its own random Fourier velocity."""
    seed = workload_seed(4) if seed is None else seed
    rng = Splitmix64(seed)
    out = []
    for b in range(nboxes):
        n = int(sizes[min(int(rng.uniform(1)[0] * len(sizes)), len(sizes) - 1)])
        lo, hi = tracer_range
        ntr = lo + min(int(rng.uniform(1)[0] * (hi - lo + 1)), hi - lo)
        phi = phi_range[0] + (phi_range[1] - phi_range[0]) * rng.uniform(1)[0]
        d = min(diameter, 0.3 * n)
        out.append(random_drops(n, ntr, phi, d, 0.0, gap, seed + 7919 * (b + 1), workers=workers))
    return out
