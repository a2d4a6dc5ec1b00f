"""Python binding of libvofmt (argument marshalling only).

Every function takes torch tensors that already live on the GPU, passes
their device pointers and the current HIP stream to the C ABI declared in
include/vofmt.h, and raises on a non-zero return code. No computation of the
method happens here: all of it runs in the HIP kernels of libvofmt.so. The
library must be built (see `paper_2407_07463_amd._build`); importing this
module on a machine without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvofmt.so")

OK, E_ARG, E_CFL, E_CAPACITY, E_EXTENT, E_NONFINITE, E_HIP, E_NOMEM = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {E_ARG: "E_ARG", E_CFL: "E_CFL", E_CAPACITY: "E_CAPACITY", E_EXTENT: "E_EXTENT",
          E_NONFINITE: "E_NONFINITE", E_HIP: "E_HIP", E_NOMEM: "E_NOMEM"}

class Box(ctypes.Structure):
    """vofmt_box: one box of a batched advection (device pointers inside)."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ntracers", ctypes.c_int32), ("c", ctypes.c_void_p), ("sx", ctypes.c_void_p),
                ("sy", ctypes.c_void_p), ("sz", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """vofmt_tuning: tile parameters of the batched advection."""
    _fields_ = [("chunk", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32)]


# Every symbol include/vofmt.h declares, with (restype, argtypes).
_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_P_i32 = ctypes.POINTER(ctypes.c_int32)
_SIGNATURES = {
    "vofmt_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "vofmt_destroy": (None, [_vp]),
    "vofmt_last_error": (ctypes.c_char_p, [_vp]),
    "vofmt_version": (ctypes.c_char_p, []),
    "vofmt_advect": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _i64, _i32, _vp]),
    "vofmt_check_courant": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "vofmt_label_drops": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _d, _vp, _vp, _vp]),
    "vofmt_drop_moments": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vofmt_compact_tracers": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vofmt_csf_force": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _d, _vp, _vp, _vp, _vp]),
    "vofmt_drop_shapes": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _vp]),
    "vofmt_drop_moments_shapes": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                 _vp, _vp, _vp, _vp, _vp]),
    "vofmt_recolor_tracers": (ctypes.c_int, [_vp, _i32, _i32, _i32, _P_i32, _i32, _vp, _vp, _vp, _d, _vp, _P_i32,
                                             _vp]),
    "vofmt_recolor_tracers_stencil": (ctypes.c_int, [_vp, _i32, _i32, _i32, _P_i32, _i32, _vp, _vp, _vp, _vp,
                                                     _P_i32, _vp]),
    "vofmt_nearest_pair_stats": (ctypes.c_int, [_vp, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                                _vp, _vp, _vp, _vp]),
    "vofmt_nearest_pair_stats_noalloc": (ctypes.c_int, [_vp, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp,
                                                        _vp, _vp, _vp, _vp, _vp]),
    "vofmt_pair_pdfs": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "vofmt_curvature_hf": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "vofmt_mlp_forward": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "vofmt_mlp_train_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, ctypes.c_float, _i32, _vp, _vp, _vp, _vp,
                                            ctypes.POINTER(ctypes.c_float), _vp]),
    "vofmt_mlp_stencils": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _P_i32, _vp]),
    "vofmt_curvature_mlp": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _d, _vp, _vp, _P_i32, _vp]),
    "vofmt_profile_start": (ctypes.c_int, [_vp]),
    "vofmt_profile_stop": (ctypes.c_int, [_vp, _i32, ctypes.c_char_p, _P_i32, ctypes.POINTER(_d), _P_i32]),
    "vofmt_advect_batched": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(Box), _i64, _i32, ctypes.POINTER(Tuning),
                                            _vp]),
    "vofmt_autotune_batched": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(Box), _i32, ctypes.POINTER(Tuning),
                                              ctypes.POINTER(ctypes.c_float), _vp]),
}

MLP_NPARAMS = 20868

_lib = None


class VofmtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libvofmt.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run paper_2407_07463_amd._build.build_all() "
                               "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def exported_symbols(path: str = LIB_PATH):
    L = ctypes.CDLL(path)
    return {n for n in _SIGNATURES if hasattr(L, n)}


def _stream(stream=None):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dims(c):
    nz, ny, nx = (int(v) for v in c.shape[-3:])
    return nx, ny, nz


class Context:
    """A libvofmt context: scratch memory for one stream on one device."""

    def __init__(self, device: int = 0):
        L = load()
        h = ctypes.c_void_p()
        rc = L.vofmt_create(ctypes.byref(h), int(device))
        if rc != 0:
            raise VofmtError(rc, f"vofmt_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            load().vofmt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise VofmtError(rc, load().vofmt_last_error(self.h).decode())
        return rc

    # ------------------------------------------------------------ advection
    def advect(self, c, sx, sy, sz, step0: int = 0, nsteps: int = 1, stream=None):
        """In-place advection of c[N][nz][ny][nx] (float64, contiguous, on the GPU)."""
        _require(c, sx, sy, sz)
        nx, ny, nz = _dims(c)
        ntr = int(c.shape[0]) if c.dim() == 4 else 1
        for s in (sx, sy, sz):
            assert tuple(s.shape) == (nz, ny, nx)
        return self._check(load().vofmt_advect(self.h, nx, ny, nz, ntr, _ptr(c), _ptr(sx), _ptr(sy), _ptr(sz),
                                               int(step0), int(nsteps), _stream(stream)))

    def check_courant(self, sx, sy, sz, stream=None) -> float:
        _require(sx, sy, sz)
        nx, ny, nz = _dims(sx)
        out = ctypes.c_double(0.0)
        self._check(load().vofmt_check_courant(self.h, nx, ny, nz, _ptr(sx), _ptr(sy), _ptr(sz), ctypes.byref(out),
                                               _stream(stream)))
        return out.value

    def _boxes(self, boxes):
        """[(c, sx, sy, sz), ...] -> ctypes array of vofmt_box."""
        arr = (Box * len(boxes))()
        for i, (c, sx, sy, sz) in enumerate(boxes):
            _require(c, sx, sy, sz)
            nx, ny, nz = _dims(c)
            for t in (sx, sy, sz):
                assert tuple(t.shape) == (nz, ny, nx)
            ntr = int(c.shape[0]) if c.dim() == 4 else 1
            arr[i] = Box(nx, ny, nz, ntr, c.data_ptr(), sx.data_ptr(), sy.data_ptr(), sz.data_ptr())
        return arr

    def advect_batched(self, boxes, step0: int = 0, nsteps: int = 1, tuning=None, stream=None):
        """Advect every (c, sx, sy, sz) of `boxes` in place with one graph launch."""
        arr = self._boxes(boxes)
        tp = None if tuning is None else ctypes.byref(Tuning(int(tuning[0]), int(tuning[1])))
        return self._check(load().vofmt_advect_batched(self.h, len(boxes), arr, int(step0), int(nsteps), tp,
                                                       _stream(stream)))

    def autotune_batched(self, boxes, nsteps: int = 1, stream=None):
        """Fastest (chunk, workgroups_per_cu) for these boxes, and its time in ms."""
        arr = self._boxes(boxes)
        best = Tuning(0, 0)
        ms = ctypes.c_float(0.0)
        self._check(load().vofmt_autotune_batched(self.h, len(boxes), arr, int(nsteps), ctypes.byref(best),
                                                  ctypes.byref(ms), _stream(stream)))
        return (best.chunk, best.workgroups_per_cu), ms.value

    # ------------------------------------------------------------ instrumentation
    def profile_start(self):
        return self._check(load().vofmt_profile_start(self.h))

    def profile_stop(self, max_kinds: int = 64):
        """{kernel kind: (launches, total_ms)} of the launches since profile_start."""
        names = ctypes.create_string_buffer(48 * max_kinds)
        launches = (ctypes.c_int32 * max_kinds)()
        total = (ctypes.c_double * max_kinds)()
        nk = ctypes.c_int32(0)
        self._check(load().vofmt_profile_stop(self.h, max_kinds, names, launches, total, ctypes.byref(nk)))
        out = {}
        for k in range(min(nk.value, max_kinds)):
            name = names.raw[48 * k:48 * (k + 1)].split(b"\0", 1)[0].decode()
            out[name] = (int(launches[k]), float(total[k]))
        return out

    # ------------------------------------------------------------ drops
    def label_drops(self, c, labels, c_eps: float = 1e-6, stream=None):
        """Labels into `labels` (int32, same shape as c); returns the per-tracer drop counts."""
        _require(c, labels)
        nx, ny, nz = _dims(c)
        ntr = int(c.shape[0]) if c.dim() == 4 else 1
        nd = np.zeros(max(ntr, 1), dtype=np.int32)
        self._check(load().vofmt_label_drops(self.h, nx, ny, nz, ntr, _ptr(c), float(c_eps), _ptr(labels),
                                             nd.ctypes.data, _stream(stream)))
        return nd[:ntr]

    def drop_moments(self, c, labels, ndrops, vol, xyz, stream=None):
        _require(c, labels, vol, xyz)
        nx, ny, nz = _dims(c)
        ntr = int(c.shape[0]) if c.dim() == 4 else 1
        nd = np.ascontiguousarray(ndrops, dtype=np.int32)
        return self._check(load().vofmt_drop_moments(self.h, nx, ny, nz, ntr, _ptr(c), _ptr(labels),
                                                     nd.ctypes.data, _ptr(vol), _ptr(xyz), _stream(stream)))

    def drop_shapes(self, c, labels, ndrops, inertia, chi, s=None, vel=None, stream=None):
        """Inertia tensors [D][6], aspect ratios [D] and, with s = (sx, sy, sz)
        and vel [D][3], mean velocities."""
        _require(c, labels, inertia, chi)
        if (s is None) != (vel is None):
            raise ValueError("drop_shapes: give s and vel together")
        sp = [None, None, None]
        if s is not None:
            _require(*s, vel)
            sp = [_ptr(a) for a in s]
        nx, ny, nz = _dims(c)
        ntr = int(c.shape[0]) if c.dim() == 4 else 1
        nd = np.ascontiguousarray(ndrops, dtype=np.int32)
        return self._check(load().vofmt_drop_shapes(self.h, nx, ny, nz, ntr, _ptr(c), _ptr(labels), nd.ctypes.data,
                                                    *sp, _ptr(inertia), _ptr(chi),
                                                    _ptr(vel) if vel is not None else None, _stream(stream)))

    def drop_moments_shapes(self, c, labels, ndrops, vol, xyz, inertia, chi, s=None, vel=None, stream=None):
        """Volumes [D], centroids [D][3], inertia tensors [D][6], aspect ratios [D] and, with
        s = (sx, sy, sz) and vel [D][3], mean velocities, in one pass over the drops."""
        _require(c, labels, vol, xyz, inertia, chi)
        if (s is None) != (vel is None):
            raise ValueError("drop_moments_shapes: give s and vel together")
        sp = [None, None, None]
        if s is not None:
            _require(*s, vel)
            sp = [_ptr(a) for a in s]
        nx, ny, nz = _dims(c)
        ntr = int(c.shape[0]) if c.dim() == 4 else 1
        nd = np.ascontiguousarray(ndrops, dtype=np.int32)
        return self._check(load().vofmt_drop_moments_shapes(
            self.h, nx, ny, nz, ntr, _ptr(c), _ptr(labels), nd.ctypes.data, *sp, _ptr(vol), _ptr(xyz), _ptr(inertia),
            _ptr(chi), _ptr(vel) if vel is not None else None, _stream(stream)))

    def csf_force(self, c, kappa, gamma: float, fx, fy, fz, stream=None):
        """Surface-tension force on the lower faces; c, kappa: [N][nz][ny][nx]
        (or one field [nz][ny][nx]); fx, fy, fz: [nz][ny][nx]."""
        _require(c, kappa, fx, fy, fz)
        if tuple(c.shape) != tuple(kappa.shape):
            raise ValueError("csf_force: c and kappa differ in shape")
        nx, ny, nz = _dims(c)
        ntr = int(c.shape[0]) if c.dim() == 4 else 1
        return self._check(load().vofmt_csf_force(self.h, nx, ny, nz, ntr, _ptr(c), _ptr(kappa), float(gamma),
                                                  _ptr(fx), _ptr(fy), _ptr(fz), _stream(stream)))

    def recolor_tracers(self, c, ntracers: int, labels, ndrops, gap_cells: float, new_tracer, stream=None):
        """c: [max_tracers][nz][ny][nx]; returns (ntracers_after, nmoved)."""
        _require(c, labels, new_tracer)
        nx, ny, nz = _dims(c)
        maxt = int(c.shape[0])
        nd = np.ascontiguousarray(ndrops, dtype=np.int32)
        ntr = ctypes.c_int32(int(ntracers))
        nmoved = ctypes.c_int32(0)
        self._check(load().vofmt_recolor_tracers(self.h, nx, ny, nz, ctypes.byref(ntr), maxt, _ptr(c),
                                                 _ptr(labels), nd.ctypes.data, float(gap_cells),
                                                 _ptr(new_tracer), ctypes.byref(nmoved), _stream(stream)))
        return ntr.value, nmoved.value

    def recolor_tracers_stencil(self, c, ntracers: int, labels, ndrops, new_tracer, stream=None):
        """Literal 5x5x5 near-contact criterion; c: [max_tracers][nz][ny][nx]; returns (ntracers_after,
        nmoved)."""
        _require(c, labels, new_tracer)
        nx, ny, nz = _dims(c)
        maxt = int(c.shape[0])
        nd = np.ascontiguousarray(ndrops, dtype=np.int32)
        ntr = ctypes.c_int32(int(ntracers))
        nmoved = ctypes.c_int32(0)
        self._check(load().vofmt_recolor_tracers_stencil(self.h, nx, ny, nz, ctypes.byref(ntr), maxt, _ptr(c),
                                                         _ptr(labels), nd.ctypes.data, _ptr(new_tracer),
                                                         ctypes.byref(nmoved), _stream(stream)))
        return ntr.value, nmoved.value

    def compact_tracers(self, c, ntracers: int, ndrops, stream=None):
        """Retire the tracers without drops among the first `ntracers` fields of
        c [max_tracers][nz][ny][nx]; returns (tracers kept, new index per
        tracer, discarded volume)."""
        _require(c)
        nx, ny, nz = _dims(c)
        if not 0 <= ntracers <= int(c.shape[0]):
            raise ValueError("compact_tracers: ntracers outside the field array")
        nd = np.ascontiguousarray(ndrops, dtype=np.int32)
        if len(nd) != ntracers:
            raise ValueError("compact_tracers: one drop count per tracer")
        n = ctypes.c_int32(int(ntracers))
        idx = np.zeros(max(ntracers, 1), dtype=np.int32)
        disc = ctypes.c_double(0.0)
        self._check(load().vofmt_compact_tracers(self.h, nx, ny, nz, ctypes.byref(n), _ptr(c), nd.ctypes.data,
                                                 idx.ctypes.data, ctypes.byref(disc), _stream(stream)))
        return n.value, idx[:ntracers], disc.value

    # ------------------------------------------------------------ statistics
    def nearest_pair_stats(self, xyz, box, vertical_axis: int, r2_edges, cos_edges, nn_index, nn_ties, hist, M, R,
                           A=None, stream=None):
        _require(xyz, nn_index, nn_ties, hist, M, R, *([A] if A is not None else []))
        n = int(xyz.shape[0])
        b = np.ascontiguousarray(box, dtype=np.float64)
        r2 = np.ascontiguousarray(r2_edges, dtype=np.float64)
        ce = np.ascontiguousarray(cos_edges, dtype=np.float64)
        return self._check(load().vofmt_nearest_pair_stats(
            self.h, n, _ptr(xyz), b.ctypes.data, int(vertical_axis), len(r2) - 1, len(ce) - 1, r2.ctypes.data,
            ce.ctypes.data, _ptr(nn_index), _ptr(nn_ties), _ptr(hist), _ptr(M), _ptr(R), _ptr(A), _stream(stream)))

    def nearest_pair_stats_noalloc(self, xyz, box, vertical_axis: int, r2_edges, cos_edges, nn_index, nn_ties, hist,
                                   M, R, A=None, stream=None):
        """As nearest_pair_stats, in the library's fixed scratch (no allocation, no synchronisation;
        n <= 8192, nr + ntheta + 2 <= 384)."""
        _require(xyz, nn_index, nn_ties, hist, M, R, *([A] if A is not None else []))
        n = int(xyz.shape[0])
        b = np.ascontiguousarray(box, dtype=np.float64)
        r2 = np.ascontiguousarray(r2_edges, dtype=np.float64)
        ce = np.ascontiguousarray(cos_edges, dtype=np.float64)
        return self._check(load().vofmt_nearest_pair_stats_noalloc(
            self.h, n, _ptr(xyz), b.ctypes.data, int(vertical_axis), len(r2) - 1, len(ce) - 1, r2.ctypes.data,
            ce.ctypes.data, _ptr(nn_index), _ptr(nn_ties), _ptr(hist), _ptr(M), _ptr(R), _ptr(A), _stream(stream)))

    def pair_pdfs(self, r_edges, theta_edges, hist, events: int, P, Pr, stream=None):
        """P_nst(r, theta) into P[nr][ntheta] and P_r-nst(r) into Pr[nr] (float64) from a uint64
        histogram (the first nr*ntheta entries of hist are read)."""
        _require(hist, P, Pr)
        re = np.ascontiguousarray(r_edges, dtype=np.float64)
        te = np.ascontiguousarray(theta_edges, dtype=np.float64)
        nr, nth = len(re) - 1, len(te) - 1
        if hist.numel() < nr * nth or P.numel() != nr * nth or Pr.numel() != nr:
            raise ValueError("pair_pdfs: histogram or outputs do not match the edges")
        return self._check(load().vofmt_pair_pdfs(self.h, nr, nth, re.ctypes.data, te.ctypes.data, _ptr(hist),
                                                  int(events), _ptr(P), _ptr(Pr), _stream(stream)))


    # ------------------------------------------------------------ curvature
    def curvature_hf(self, c, kappa, status, stream=None):
        """Height-function curvature of one field c[nz][ny][nx] into kappa (float64) and status (uint8)."""
        _require(c, kappa, status)
        nx, ny, nz = _dims(c)
        return self._check(load().vofmt_curvature_hf(self.h, nx, ny, nz, _ptr(c), _ptr(kappa), _ptr(status),
                                                     _stream(stream)))

    # ------------------------------------------------------------ learned curvature
    def mlp_forward(self, params, x, y, acts=None, stream=None):
        """Network outputs y[m] (float32) of stencils x[m][27]; acts: optional uint16/int16 [m][256]."""
        _require(params, x, y, *([acts] if acts is not None else []))
        m = int(x.shape[0])
        return self._check(load().vofmt_mlp_forward(self.h, _ptr(params), m, _ptr(x), _ptr(y), _ptr(acts),
                                                    _stream(stream)))

    def mlp_train_step(self, params, adam_m, adam_v, step: int, lr: float, x, y_target, grads=None, trace=None,
                       stream=None) -> float:
        """One forward + backward + Adam step in place; returns the batch loss before the update."""
        _require(params, adam_m, adam_v, x, y_target, *[t for t in (grads, trace) if t is not None])
        m = int(x.shape[0])
        loss = ctypes.c_float(0.0)
        self._check(load().vofmt_mlp_train_step(self.h, _ptr(params), _ptr(adam_m), _ptr(adam_v), int(step),
                                                float(lr), m, _ptr(x), _ptr(y_target), _ptr(grads), _ptr(trace),
                                                ctypes.byref(loss), _stream(stream)))
        return loss.value

    def mlp_stencils(self, c, xs, cell, sign, stream=None) -> int:
        """Canonical stencils of the mixed cells of c[nz][ny][nx]; returns their number."""
        _require(c, xs, cell, sign)
        nx, ny, nz = _dims(c)
        cnt = ctypes.c_int32(0)
        self._check(load().vofmt_mlp_stencils(self.h, nx, ny, nz, _ptr(c), int(xs.shape[0]), _ptr(xs), _ptr(cell),
                                              _ptr(sign), ctypes.byref(cnt), _stream(stream)))
        return cnt.value

    def curvature_mlp(self, c, params, kappa_lo: float, kappa, status, stream=None) -> int:
        """Network curvature with height-function fallback; returns the number of mixed cells."""
        _require(c, params, kappa, status)
        nx, ny, nz = _dims(c)
        cnt = ctypes.c_int32(0)
        self._check(load().vofmt_curvature_mlp(self.h, nx, ny, nz, _ptr(c), _ptr(params), float(kappa_lo),
                                               _ptr(kappa), _ptr(status), ctypes.byref(cnt), _stream(stream)))
        return cnt.value


def _require(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("vofmt: tensors must be on the GPU")
        if not t.is_contiguous():
            raise ValueError("vofmt: tensors must be contiguous")
