"""CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around `vof_oracle.c` (plain C, built with
-O2 -ffp-contract=off -fno-fast-math). Only the tests, the package smoke
check and the benchmark's CPU-baseline leg may import this module; the
product path never does, and nothing here imports the product package.

Each function cites the passage of Fintzi, Pierson & Popinet (arXiv
2407.07463) it follows; where the paper is silent the reading is stated in
the C source next to the code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = [os.path.join(_HERE, "vof_oracle.c"), os.path.join(_HERE, "mlp_oracle.c")]
_lib = None

E_ARG, E_CAPACITY, E_EXTENT = -1, -3, -4


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    srcs = [s for s in SRC if os.path.exists(s)]
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB_PATH + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.orc_plane_volume.argtypes = [d, d, d, d]
        L.orc_plane_volume.restype = d
        L.orc_plane_alpha.argtypes = [d, d, d, d]
        L.orc_plane_alpha.restype = d
        L.orc_myc_normal.argtypes = [vp, vp]
        L.orc_myc_normal.restype = ctypes.c_int
        L.orc_face_flux.argtypes = [vp, i64, i64, i64, ctypes.c_int, i64, i64, i64, d]
        L.orc_face_flux.restype = d
        L.orc_sweep.argtypes = [i64, i64, i64, ctypes.c_int, vp, vp, vp, vp]
        L.orc_sweep.restype = None
        L.orc_advect.argtypes = [i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, i64, ctypes.c_int]
        L.orc_advect.restype = ctypes.c_int
        L.orc_drop_shapes.argtypes = [i64, i64, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        L.orc_drop_shapes.restype = ctypes.c_int
        L.orc_csf_force.argtypes = [i64, i64, i64, i32, vp, vp, d, vp, vp, vp]
        L.orc_csf_force.restype = None
        L.orc_compact_tracers.argtypes = [i64, i32, vp, vp, vp, vp]
        L.orc_compact_tracers.restype = ctypes.c_int
        L.orc_label.argtypes = [i64, i64, i64, vp, d, vp]
        L.orc_label.restype = ctypes.c_int
        L.orc_drop_moments.argtypes = [i64, i64, i64, vp, vp, i32, vp, vp]
        L.orc_drop_moments.restype = ctypes.c_int
        L.orc_neighbour_pairs.argtypes = [i64, i64, i64, ctypes.c_int, vp, vp, d, vp, i64]
        L.orc_neighbour_pairs.restype = i64
        L.orc_recolor.argtypes = [i64, i64, i64, vp, i32, vp, vp, vp, d, vp, vp]
        L.orc_recolor.restype = ctypes.c_int
        L.orc_recolor_stencil.argtypes = [i64, i64, i64, vp, i32, vp, vp, vp, vp, vp]
        L.orc_recolor_stencil.restype = ctypes.c_int
        L.orc_stencil_flags.argtypes = [i64, i64, i64, vp, vp]
        L.orc_stencil_flags.restype = None
        L.orc_neighbour_pairs_stencil.argtypes = [i64, i64, i64, ctypes.c_int, vp, vp, vp, i64]
        L.orc_neighbour_pairs_stencil.restype = i64
        L.orc_nearest_pair_stats.argtypes = [i32, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_nearest_pair_stats.restype = ctypes.c_int
        L.orc_pair_pdfs.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp]
        L.orc_pair_pdfs.restype = ctypes.c_int
        L.orc_curvature_hf.argtypes = [i64, i64, i64, vp, vp, vp]
        L.orc_curvature_hf.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        if hasattr(L, "orc_mlp_forward"):
            _setup_mlp(L)
        _lib = L
    return _lib


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops from now on."""
    lib().orc_set_num_threads(int(n))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _shape3(c, ndim: int = 0):
    """(nx, ny, nz) of a [nz][ny][nx] field or a [N][nz][ny][nx] stack; with ndim
    given, other shapes raise ValueError (the C functions would read past them)."""
    if ndim and c.ndim != ndim:
        raise ValueError(f"expected a {ndim}-D array, got shape {c.shape}")
    nz, ny, nx = c.shape[-3:]
    return int(nx), int(ny), int(nz)


# ---------------------------------------------------------------- geometry

def plane_volume(m, alpha: float) -> float:
    """V(m, alpha): volume of {x in [0,1]^3 : m.x <= alpha}."""
    return lib().orc_plane_volume(float(m[0]), float(m[1]), float(m[2]), float(alpha))


def plane_alpha(m, c: float) -> float:
    """alpha with V(m, alpha) = c, by bisection."""
    return lib().orc_plane_alpha(float(m[0]), float(m[1]), float(m[2]), float(c))


def myc_normal(block) -> tuple[np.ndarray, bool]:
    """Mixed-Youngs-Centred normal of a 3x3x3 block given as b[az][ay][ax]."""
    b = _f64(block).reshape(27)
    m = np.zeros(3)
    used_cs = lib().orc_myc_normal(b.ctypes.data, m.ctypes.data)
    return m, bool(used_cs)


# ---------------------------------------------------------------- advection

def sweep(c, s, d: int, cc=None):
    """One Jacobi sweep along axis d of one field c[nz][ny][nx]; returns the new field."""
    c = _f64(c)
    s = _f64(s)
    nx, ny, nz = _shape3(c, 3)
    if cc is None:
        cc = (c > 0.5)
    cc = np.ascontiguousarray(cc, dtype=np.uint8)
    out = np.empty_like(c)
    lib().orc_sweep(nx, ny, nz, int(d), c.ctypes.data, out.ctypes.data, s.ctypes.data, cc.ctypes.data)
    return out


def advect(c, sx, sy, sz, step0: int = 0, nsteps: int = 1):
    """nsteps direction-split steps of every tracer of c[N][nz][ny][nx]; returns a new array.

    Follows eq. (3) for each tracer C_i (section "The no-coalescence.h
    algorithm": one transport equation per tracer)."""
    c = np.array(c, dtype=np.float64, copy=True, order="C")
    if c.ndim == 3:
        c = c[None]
    nx, ny, nz = _shape3(c)
    sx, sy, sz = _f64(sx), _f64(sy), _f64(sz)
    for s in (sx, sy, sz):
        assert s.shape == (nz, ny, nx)
    rc = lib().orc_advect(nx, ny, nz, c.shape[0], c.ctypes.data, sx.ctypes.data, sy.ctypes.data, sz.ctypes.data,
                          int(step0), int(nsteps))
    if rc != 0:
        raise ValueError(f"orc_advect failed: {rc}")
    return c


# ---------------------------------------------------------------- drops

def label(c, c_eps: float = 1e-6):
    """Canonical 6-connected periodic components of {c > c_eps} (tag.h step)."""
    c = _f64(c)
    nx, ny, nz = _shape3(c, 3)
    lab = np.zeros(c.shape, dtype=np.int32)
    k = lib().orc_label(nx, ny, nz, c.ctypes.data, float(c_eps), lab.ctypes.data)
    return lab, int(k)


def drop_moments(c, labels, k: int):
    c = _f64(c)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _shape3(c, 3)
    vol = np.zeros(max(k, 0))
    xyz = np.zeros((max(k, 0), 3))
    rc = lib().orc_drop_moments(nx, ny, nz, c.ctypes.data, labels.ctypes.data, int(k), vol.ctypes.data,
                                xyz.ctypes.data)
    return vol, xyz, rc


def drop_shapes(c, labels, k: int, xyz, s=None):
    """Inertia tensor of every drop about its centroid xyz, [k][6] =
    (Ixx, Iyy, Izz, Ixy, Ixz, Iyz), and with s = (sx, sy, sz) the drop's mean
    velocity [k][3] (else None). Appendix "Deformation of the drops"."""
    c = _f64(c)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _shape3(c, 3)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    assert len(xyz) >= k
    inertia = np.zeros((max(k, 0), 6))
    vel = np.zeros((max(k, 0), 3)) if s is not None else None
    sp = [_f64(a) for a in s] if s is not None else [None, None, None]
    if s is not None:
        assert all(a.shape == c.shape for a in sp)
    rc = lib().orc_drop_shapes(nx, ny, nz, c.ctypes.data, labels.ctypes.data, int(k), xyz.ctypes.data,
                               *[a.ctypes.data if a is not None else None for a in sp], inertia.ctypes.data,
                               vel.ctypes.data if vel is not None else None)
    return inertia, vel, rc


def aspect_ratio(inertia):
    """chi = sqrt(I1 / I2) with I1, I2 the largest and smallest eigenvalues of
    each inertia tensor (appendix "Deformation of the drops"); eigenvalues by
    LAPACK's symmetric solver. Returns (eigenvalues ascending [k][3], chi [k])."""
    inertia = np.asarray(inertia, dtype=np.float64).reshape(-1, 6)
    T = np.empty((len(inertia), 3, 3))
    T[:, 0, 0], T[:, 1, 1], T[:, 2, 2] = inertia[:, 0], inertia[:, 1], inertia[:, 2]
    T[:, 0, 1] = T[:, 1, 0] = inertia[:, 3]
    T[:, 0, 2] = T[:, 2, 0] = inertia[:, 4]
    T[:, 1, 2] = T[:, 2, 1] = inertia[:, 5]
    ev = np.linalg.eigvalsh(T) if len(T) else np.zeros((0, 3))
    return ev, np.sqrt(ev[:, 2] / ev[:, 0]) if len(T) else np.zeros(0)


def csf_force(c, kappa, gamma: float):
    """Face-centred surface-tension force gamma * sum_i kappa_i grad C_i on the
    lower faces, (fx, fy, fz) each [nz][ny][nx] (section "The no-coalescence.h
    algorithm", balanced-force form). c, kappa: [ntr][nz][ny][nx], NaN where
    a curvature is undefined."""
    c = _f64(c)
    kappa = _f64(kappa)
    if c.ndim == 3:
        c, kappa = c[None], kappa[None]
    assert c.shape == kappa.shape
    ntr = c.shape[0]
    nx, ny, nz = _shape3(c, 4)
    out = [np.zeros(c.shape[1:]) for _ in range(3)]
    lib().orc_csf_force(nx, ny, nz, ntr, c.ctypes.data, kappa.ctypes.data, float(gamma),
                        *[o.ctypes.data for o in out])
    return tuple(out)


def compact_tracers(c, ndrops):
    """Retire the tracers without drops (reading of the tracer count N(t),
    section "The no-coalescence.h algorithm"). c: [ntr][nz][ny][nx] (copied).
    Returns (c_new, n_new, new_index[ntr], discarded volume)."""
    c = np.array(c, dtype=np.float64, order="C", copy=True)
    ntr = c.shape[0]
    n3 = int(np.prod(c.shape[1:]))
    nd = np.ascontiguousarray(ndrops, dtype=np.int32)
    assert len(nd) == ntr
    idx = np.zeros(ntr, dtype=np.int32)
    disc = ctypes.c_double(0.0)
    k = lib().orc_compact_tracers(n3, ntr, c.ctypes.data, nd.ctypes.data, idx.ctypes.data, ctypes.byref(disc))
    return c, int(k), idx, disc.value


def neighbour_pairs(labels, ndrops, tau: float):
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    ntr = labels.shape[0]
    nx, ny, nz = _shape3(labels, 4)
    nd = np.ascontiguousarray(ndrops, dtype=np.int32)
    cap = 1 << 16
    while True:
        pairs = np.zeros((cap, 2), dtype=np.int32)
        m = lib().orc_neighbour_pairs(nx, ny, nz, ntr, labels.ctypes.data, nd.ctypes.data, float(tau),
                                      pairs.ctypes.data, cap)
        if m <= cap:
            return pairs[:m]
        cap = int(m)


def recolor(c, labels, ndrops, ntracers: int, max_tracers: int, tau: float):
    """Steps 1-4 of the no-coalescence algorithm (greedy reading).

    c: [max_tracers][nz][ny][nx] (copied); labels: [ntracers][nz][ny][nx].
    Returns (c_new, ntracers_new, new_tracer[D], nmoved, rc)."""
    c = np.array(c, dtype=np.float64, copy=True, order="C")
    assert c.shape[0] == max_tracers
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _shape3(c, 4)
    nd = np.ascontiguousarray(ndrops, dtype=np.int32)
    D = int(nd.sum())
    newt = np.zeros(max(D, 1), dtype=np.int32)
    ntr = ctypes.c_int32(int(ntracers))
    nmoved = ctypes.c_int32(0)
    rc = lib().orc_recolor(nx, ny, nz, ctypes.byref(ntr), int(max_tracers), c.ctypes.data, labels.ctypes.data,
                           nd.ctypes.data, float(tau), newt.ctypes.data, ctypes.byref(nmoved))
    return c, ntr.value, newt[:D], nmoved.value, rc


def stencil_flags(labels):
    """Literal near-contact criterion per cell of one tracer's labels [nz][ny][nx]: 0 no,
    1 Step 1 (empty centre, two opposite occupied cells in the 5^3 stencil), 2 Steps 1 and 3
    (their labels differ)."""
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _shape3(labels, 3)
    out = np.zeros(labels.shape, dtype=np.uint8)
    lib().orc_stencil_flags(nx, ny, nz, labels.ctypes.data, out.ctypes.data)
    return out


def neighbour_pairs_stencil(labels, ndrops):
    """Directed neighbour pairs of the literal mode (conflicts within a tracer, contacts across)."""
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    ntr = labels.shape[0]
    nx, ny, nz = _shape3(labels, 4)
    nd = np.ascontiguousarray(ndrops, dtype=np.int32)
    cap = 1 << 16
    while True:
        pairs = np.zeros((cap, 2), dtype=np.int32)
        m = lib().orc_neighbour_pairs_stencil(nx, ny, nz, ntr, labels.ctypes.data, nd.ctypes.data,
                                              pairs.ctypes.data, cap)
        if m <= cap:
            return pairs[:m]
        cap = int(m)


def recolor_stencil(c, labels, ndrops, ntracers: int, max_tracers: int):
    """Steps 1-4 with the literal 5^3 stencil criterion. Returns (c_new, ntracers_new,
    new_tracer[D], nmoved, rc) like recolor()."""
    c = np.array(c, dtype=np.float64, copy=True, order="C")
    assert c.shape[0] == max_tracers
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _shape3(c, 4)
    nd = np.ascontiguousarray(ndrops, dtype=np.int32)
    D = int(nd.sum())
    newt = np.zeros(max(D, 1), dtype=np.int32)
    ntr = ctypes.c_int32(int(ntracers))
    nmoved = ctypes.c_int32(0)
    rc = lib().orc_recolor_stencil(nx, ny, nz, ctypes.byref(ntr), int(max_tracers), c.ctypes.data,
                                   labels.ctypes.data, nd.ctypes.data, newt.ctypes.data, ctypes.byref(nmoved))
    return c, ntr.value, newt[:D], nmoved.value, rc


# ---------------------------------------------------------------- statistics

FIXED_ONE = 720720  # lcm(1..16): tie weights 1/N_i are exact integers in these units


def nearest_pair_stats(xyz, box, vaxis: int, r2_edges, cos_edges):
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    box = _f64(box)
    r2e = _f64(r2_edges)
    ce = _f64(cos_edges)
    nr, nth = len(r2e) - 1, len(ce) - 1
    idx = np.zeros(n, dtype=np.int32)
    ties = np.zeros(n, dtype=np.int32)
    hist = np.zeros(nr * nth + 1, dtype=np.uint64)
    M = np.zeros(3)
    R = np.zeros(9)
    A = np.zeros(9)
    rc = lib().orc_nearest_pair_stats(n, xyz.ctypes.data, box.ctypes.data, int(vaxis), nr, nth, r2e.ctypes.data,
                                      ce.ctypes.data, idx.ctypes.data, ties.ctypes.data, hist.ctypes.data,
                                      M.ctypes.data, R.ctypes.data, A.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_nearest_pair_stats failed: {rc}")
    return dict(nn_index=idx, nn_ties=ties, hist=hist[:-1].reshape(nr, nth), overflow=int(hist[-1]),
                M=M, R=R.reshape(3, 3), A=A.reshape(3, 3), raw_hist=hist)


def pair_pdfs(r_edges, th_edges, hist, events: int):
    """P_nst(r, theta) [nr][nth] and P_r-nst(r) [nr] of an accumulated histogram (eqs. 8, 10 at
    bin centres). hist: [nr*nth] or [nr][nth] uint64 in units of 1/720720 (overflow excluded)."""
    re = _f64(r_edges)
    te = _f64(th_edges)
    nr, nth = len(re) - 1, len(te) - 1
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint64).reshape(-1)[: nr * nth])
    P = np.zeros(nr * nth)
    Pr = np.zeros(nr)
    rc = lib().orc_pair_pdfs(nr, nth, re.ctypes.data, te.ctypes.data, h.ctypes.data, int(events), P.ctypes.data,
                             Pr.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_pair_pdfs failed: {rc}")
    return P.reshape(nr, nth), Pr


# ---------------------------------------------------------------- curvature

def curvature_hf(c):
    c = _f64(c)
    nx, ny, nz = _shape3(c, 3)
    kappa = np.zeros(c.shape)
    status = np.zeros(c.shape, dtype=np.uint8)
    lib().orc_curvature_hf(nx, ny, nz, c.ctypes.data, kappa.ctypes.data, status.ctypes.data)
    return kappa, status


# ---------------------------------------------------------------- learned curvature
# Not in the paper (it uses height functions); the reference arithmetic of the
# network is in mlp_oracle.c.

MLP_NPARAMS = 20868
MLP_OFF = dict(W1=0, b1=4096, W2=4224, b2=20608, W3=20736, b3=20864)


def _setup_mlp(L):
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    L.orc_mlp_nparams.argtypes = []
    L.orc_mlp_nparams.restype = i32
    L.orc_bf16.argtypes = [ctypes.c_float]
    L.orc_bf16.restype = ctypes.c_float
    L.orc_canonical_stencil.argtypes = [vp, vp]
    L.orc_canonical_stencil.restype = i32
    L.orc_two_interfaces.argtypes = [vp]
    L.orc_two_interfaces.restype = i32
    L.orc_mlp_forward.argtypes = [vp, i32, vp, i32, vp, vp]
    L.orc_mlp_forward.restype = None
    L.orc_mlp_grad.argtypes = [vp, i32, vp, vp, i32, vp]
    L.orc_mlp_grad.restype = ctypes.c_double
    L.orc_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double]
    L.orc_adam.restype = None
    L.orc_mlp_layer.argtypes = [vp, i32, i32, vp, i32, vp, vp, vp]
    L.orc_mlp_layer.restype = None
    L.orc_mlp_backward_given.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    L.orc_mlp_backward_given.restype = None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return None if a is None else a.ctypes.data


def bf16(v) -> np.ndarray:
    """FP32 -> BF16 -> FP32 with round to nearest even, elementwise."""
    v = _f32(v)
    f = lib().orc_bf16
    return np.array([f(float(t)) for t in v.ravel()], dtype=np.float32).reshape(v.shape)


def canonical_stencil(block) -> tuple[np.ndarray, int]:
    """Canonical form of a 3x3x3 block b[az][ay][ax] -> (27 FP32, sign)."""
    b = _f64(block).reshape(27)
    out = np.zeros(27, dtype=np.float32)
    s = lib().orc_canonical_stencil(b.ctypes.data, out.ctypes.data)
    return out, int(s)


def two_interfaces(block) -> bool:
    """Whether a 3x3x3 block b[az][ay][ax] holds two interfaces: MYC's
    centred-columns orientation along the first height-function axis disagrees
    with the height functions' orientation there (the second fallback trigger)."""
    b = _f64(block).reshape(27)
    return bool(lib().orc_two_interfaces(b.ctypes.data))


def mlp_forward(params, x, exact: bool = False):
    """Network output (FP64) and activations [n][512] = h1, h2, z1, z2."""
    P, x = _f32(params), _f32(x).reshape(-1, 27)
    n = x.shape[0]
    y = np.zeros(n)
    acts = np.zeros((n, 512))
    lib().orc_mlp_forward(P.ctypes.data, n, x.ctypes.data, int(exact), y.ctypes.data, acts.ctypes.data)
    return y, acts


def mlp_grad(params, x, t, exact: bool = False):
    """Batch loss and its gradient (FP64) with respect to every parameter."""
    P, x, t = _f32(params), _f32(x).reshape(-1, 27), _f32(t)
    g = np.zeros(MLP_NPARAMS)
    loss = lib().orc_mlp_grad(P.ctypes.data, x.shape[0], x.ctypes.data, t.ctypes.data, int(exact), g.ctypes.data)
    return loss, g


def adam(params, m, v, grad, step: int, lr: float):
    """One Adam step in FP64 on FP32 copies; returns (params, m, v)."""
    P, M, V = _f32(params).copy(), _f32(m).copy(), _f32(v).copy()
    g = _f64(grad)
    lib().orc_adam(P.ctypes.data, M.ctypes.data, V.ctypes.data, g.ctypes.data, int(step), float(lr))
    return P, M, V


def mlp_layer(params, layer: int, inp, exact: bool = False):
    """One layer on supplied inputs -> (pre, act, absacc)."""
    P = _f32(params)
    nin = 27 if layer == 1 else 128
    inp = _f64(inp).reshape(-1, nin)
    n = inp.shape[0]
    nout = 1 if layer == 3 else 128
    pre, act, aab = np.zeros((n, nout)), np.zeros((n, nout)), np.zeros((n, nout))
    lib().orc_mlp_layer(P.ctypes.data, int(layer), n, inp.ctypes.data, int(exact), pre.ctypes.data,
                        act.ctypes.data, aab.ctypes.data)
    if layer == 3:
        return pre[:, 0], act[:, 0], aab[:, 0]
    return pre, act, aab


def mlp_backward_given(params, x, g, h1, h2, dz2, dz1, exact: bool = False):
    """Backward pass on supplied intermediates -> dict(dz2, dz1, dz1_abs, grad, grad_abs)."""
    P, x = _f32(params), _f32(x).reshape(-1, 27)
    n = x.shape[0]
    g, h1, h2, dz2, dz1 = (_f64(a) for a in (g, h1, h2, dz2, dz1))
    out = dict(dz2=np.zeros((n, 128)), dz1=np.zeros((n, 128)), dz1_abs=np.zeros((n, 128)),
               grad=np.zeros(MLP_NPARAMS), grad_abs=np.zeros(MLP_NPARAMS))
    lib().orc_mlp_backward_given(P.ctypes.data, n, x.ctypes.data, g.ctypes.data, h1.ctypes.data, h2.ctypes.data,
                                 dz2.ctypes.data, dz1.ctypes.data, int(exact), out["dz2"].ctypes.data,
                                 out["dz1"].ctypes.data, out["dz1_abs"].ctypes.data, out["grad"].ctypes.data,
                                 out["grad_abs"].ctypes.data)
    return out
