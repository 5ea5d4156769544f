"""FP64 CPU oracle for space-time kernel density estimation (arXiv 1705.09366).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never calls it.

Contents
--------
* :func:`pbsym`   -- Alg. PB-SYM (Sec. 3.2) in FP64, plain C with OpenMP slabs.
* :func:`vb_voxels` -- Alg. VB (Sec. 2.2) in FP64 at chosen voxels, plain C.
* :func:`vb_grid_numpy` -- Alg. VB over a whole (tiny) grid, written a second
  time in numpy so that the brute-force check does not share code with the C
  loops.
* :func:`point_sums` -- per-point in-grid kernel sums and support counts.
* :func:`pbsym_adaptive`, :func:`vb_voxels_adaptive`, :func:`point_sums_adaptive`,
  :func:`vb_grid_numpy_adaptive` -- the same with a bandwidth pair per event
  (the sample-point reading of the adaptive bandwidth of Sec. 8).

Kernels follow the Epanechnikov reading of the garbled kernel formulas of
Sec. 2.1: ks(u,v) = (2/pi)(1-u^2-v^2) on the open unit disc,
kt(w) = (3/4)(1-w^2) on |w| <= 1.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None


class _Grid(ctypes.Structure):
    _fields_ = [("gx", ctypes.c_int64), ("gy", ctypes.c_int64), ("gt", ctypes.c_int64),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("t0", ctypes.c_double),
                ("sres", ctypes.c_double), ("tres", ctypes.c_double),
                ("hs", ctypes.c_double), ("ht", ctypes.c_double),
                ("kernel", ctypes.c_int32), ("corner", ctypes.c_int32)]


KERNEL_EPANECHNIKOV, KERNEL_QUARTIC, KERNEL_GAUSSIAN, KERNEL_PRINTED = 0, 1, 2, 3


@dataclass(frozen=True)
class Grid:
    """Discretised domain (Sec. 2.1): gx x gy x gt voxels of sres x sres x tres
    with voxel (0,0,0) cornered at (x0, y0, t0), bandwidths hs, ht, the kernel
    pair (KERNEL_*, see stkde_oracle.h) and where voxels are sampled (centre,
    or lower corner with ``corner``)."""
    gx: int
    gy: int
    gt: int
    hs: float
    ht: float
    sres: float = 1.0
    tres: float = 1.0
    x0: float = 0.0
    y0: float = 0.0
    t0: float = 0.0
    kernel: int = KERNEL_EPANECHNIKOV
    corner: bool = False

    def _c(self):
        return _Grid(self.gx, self.gy, self.gt, self.x0, self.y0, self.t0,
                     self.sres, self.tres, self.hs, self.ht, int(self.kernel), int(bool(self.corner)))


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        lib.oracle_pbsym.argtypes = [P(_Grid), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     P(ctypes.c_int64), ctypes.c_int]
        lib.oracle_vb_voxels.argtypes = [P(_Grid), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_point_sums.argtypes = [P(_Grid), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int]
        lib.oracle_pbsym_adaptive.argtypes = [P(_Grid), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_void_p, P(ctypes.c_int64), ctypes.c_int]
        lib.oracle_vb_voxels_adaptive.argtypes = [P(_Grid), ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                                  ctypes.c_void_p, ctypes.c_int]
        lib.oracle_point_sums_adaptive.argtypes = [P(_Grid), ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        for f in (lib.oracle_pbsym, lib.oracle_vb_voxels, lib.oracle_point_sums, lib.oracle_pbsym_adaptive,
                  lib.oracle_vb_voxels_adaptive, lib.oracle_point_sums_adaptive):
            f.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _threads(nthreads):
    if nthreads is None or nthreads < 1:
        return max(1, len(os.sched_getaffinity(0)))
    return int(nthreads)


def _points(xyt):
    a = np.ascontiguousarray(xyt, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("points must be an (n, 3) array of (x, y, t)")
    return a


def pbsym(xyt, grid: Grid, nthreads=None):
    """Alg. PB-SYM in FP64.  Returns (density[gx, gy, gt] float64, evals)."""
    pts = _points(xyt)
    out = np.empty((grid.gx, grid.gy, grid.gt), dtype=np.float64)
    ev = ctypes.c_int64(0)
    rc = _lib().oracle_pbsym(ctypes.byref(grid._c()), pts.ctypes.data, pts.shape[0],
                             out.ctypes.data, ctypes.byref(ev), _threads(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_pbsym failed ({rc})")
    return out, int(ev.value)


def vb_voxels(xyt, grid: Grid, voxels, nthreads=None):
    """Alg. VB evaluated at the (m, 3) integer voxel list ``voxels``."""
    pts = _points(xyt)
    vox = np.ascontiguousarray(voxels, dtype=np.int64).reshape(-1, 3)
    out = np.empty(vox.shape[0], dtype=np.float64)
    rc = _lib().oracle_vb_voxels(ctypes.byref(grid._c()), pts.ctypes.data, pts.shape[0],
                                 vox.ctypes.data, vox.shape[0], out.ctypes.data,
                                 _threads(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_vb_voxels failed ({rc})")
    return out


def point_sums(xyt, grid: Grid, nthreads=None):
    """Per point: (Ss, St, cs, ct) -- in-grid sums of ks and kt and the numbers
    of in-grid columns and rows inside the support."""
    pts = _points(xyt)
    n = pts.shape[0]
    Ss = np.empty(n, np.float64)
    St = np.empty(n, np.float64)
    cs = np.empty(n, np.int64)
    ct = np.empty(n, np.int64)
    rc = _lib().oracle_point_sums(ctypes.byref(grid._c()), pts.ctypes.data, n, Ss.ctypes.data,
                                  St.ctypes.data, cs.ctypes.data, ct.ctypes.data,
                                  _threads(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_point_sums failed ({rc})")
    return Ss, St, cs, ct


def exact_mass(xyt, grid: Grid, nthreads=None):
    """Total density times voxel volume implied by the per-point sums:
    sum_i Ss(i) St(i) / (n hs^2 ht) * sres^2 tres (exact up to rounding
    because grid clipping is a box and the kernel is separable)."""
    Ss, St, _, _ = point_sums(xyt, grid, nthreads)
    n = Ss.shape[0]
    return float(np.sum(Ss * St) / (n * grid.hs ** 2 * grid.ht) * grid.sres ** 2 * grid.tres)


def exact_evals(xyt, grid: Grid, nthreads=None):
    """Exact number of in-grid (voxel, point) pairs inside both supports."""
    _, _, cs, ct = point_sums(xyt, grid, nthreads)
    return int(np.sum(cs * ct))


def _np_ks(kernel, u, v):
    """Spatial factor of each pair on u^2 + v^2 < 1 (numpy; see stkde_oracle.h)."""
    r2 = u * u + v * v
    if kernel == KERNEL_QUARTIC:
        return 3.0 / np.pi * (1.0 - r2) ** 2
    if kernel == KERNEL_GAUSSIAN:
        return np.exp(-2.0 * r2) / (np.pi / 2.0 * (1.0 - np.exp(-2.0)))
    if kernel == KERNEL_PRINTED:
        return np.pi / 2.0 * (1.0 - u) ** 2 * (1.0 - v) ** 2
    return (2.0 / np.pi) * (1.0 - r2)


def _np_kt(kernel, w):
    """Temporal factor of each pair on |w| <= 1 (numpy)."""
    import math
    if kernel == KERNEL_QUARTIC:
        return 15.0 / 16.0 * (1.0 - w * w) ** 2
    if kernel == KERNEL_GAUSSIAN:
        return np.exp(-2.0 * w * w) / (math.sqrt(math.pi / 2.0) * math.erf(math.sqrt(2.0)))
    if kernel == KERNEL_PRINTED:
        return 0.75 * (1.0 - w) ** 2
    return 0.75 * (1.0 - w * w)


def vb_grid_numpy(xyt, grid: Grid):
    """Alg. VB over the whole grid, vectorised over points with numpy.  For
    tiny grids only (it holds a points x voxels-row temporary)."""
    pts = _points(xyt)
    fin = np.all(np.isfinite(pts), axis=1)
    n = pts.shape[0]
    p = pts[fin]
    off = 0.0 if grid.corner else 0.5
    out = np.zeros((grid.gx, grid.gy, grid.gt), dtype=np.float64)
    xs = grid.x0 + (np.arange(grid.gx) + off) * grid.sres
    ys = grid.y0 + (np.arange(grid.gy) + off) * grid.sres
    ts = grid.t0 + (np.arange(grid.gt) + off) * grid.tres
    for X, x in enumerate(xs):
        for Y, y in enumerate(ys):
            d = np.sqrt((p[:, 0] - x) ** 2 + (p[:, 1] - y) ** 2)
            ins = d < grid.hs
            if not np.any(ins):
                continue
            q = p[ins]
            u = (x - q[:, 0]) / grid.hs
            v = (y - q[:, 1]) / grid.hs
            ksv = _np_ks(grid.kernel, u, v)
            dt = ts[None, :] - q[:, 2][:, None]
            w = dt / grid.ht
            ktv = np.where(np.abs(dt) <= grid.ht, _np_kt(grid.kernel, np.clip(w, -1.0, 1.0)), 0.0)
            out[X, Y, :] = np.sum(ksv[:, None] * ktv, axis=0)
    return out / (n * grid.hs ** 2 * grid.ht)


# ------------------------------------------------ per-event bandwidths
def _bandwidths(hst, n):
    h = np.ascontiguousarray(hst, dtype=np.float64)
    if h.shape != (n, 2):
        raise ValueError("bandwidths must be an (n, 2) array of (hs_i, ht_i)")
    return h


def pbsym_adaptive(xyt, hst, grid: Grid, nthreads=None):
    """Alg. PB-SYM with a bandwidth pair per event (hst: (n, 2) of hs_i, ht_i
    in domain units; grid.hs / grid.ht are not used).  Returns (density, evals)."""
    pts = _points(xyt)
    h = _bandwidths(hst, pts.shape[0])
    out = np.empty((grid.gx, grid.gy, grid.gt), dtype=np.float64)
    ev = ctypes.c_int64(0)
    rc = _lib().oracle_pbsym_adaptive(ctypes.byref(grid._c()), pts.ctypes.data, h.ctypes.data,
                                      pts.shape[0], out.ctypes.data, ctypes.byref(ev),
                                      _threads(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_pbsym_adaptive failed ({rc})")
    return out, int(ev.value)


def vb_voxels_adaptive(xyt, hst, grid: Grid, voxels, nthreads=None):
    """Alg. VB with per-event bandwidths at the (m, 3) voxel list."""
    pts = _points(xyt)
    h = _bandwidths(hst, pts.shape[0])
    vox = np.ascontiguousarray(voxels, dtype=np.int64).reshape(-1, 3)
    out = np.empty(vox.shape[0], dtype=np.float64)
    rc = _lib().oracle_vb_voxels_adaptive(ctypes.byref(grid._c()), pts.ctypes.data, h.ctypes.data,
                                          pts.shape[0], vox.ctypes.data, vox.shape[0], out.ctypes.data,
                                          _threads(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_vb_voxels_adaptive failed ({rc})")
    return out


def point_sums_adaptive(xyt, hst, grid: Grid, nthreads=None):
    """Per event, with its own bandwidths: (Ss, St, cs, ct) as :func:`point_sums`."""
    pts = _points(xyt)
    n = pts.shape[0]
    h = _bandwidths(hst, n)
    Ss = np.empty(n, np.float64)
    St = np.empty(n, np.float64)
    cs = np.empty(n, np.int64)
    ct = np.empty(n, np.int64)
    rc = _lib().oracle_point_sums_adaptive(ctypes.byref(grid._c()), pts.ctypes.data, h.ctypes.data, n,
                                           Ss.ctypes.data, St.ctypes.data, cs.ctypes.data,
                                           ct.ctypes.data, _threads(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_point_sums_adaptive failed ({rc})")
    return Ss, St, cs, ct


def exact_mass_adaptive(xyt, hst, grid: Grid, nthreads=None):
    """sum_i Ss(i) St(i) / (n hs_i^2 ht_i) * sres^2 tres: the grid's mass,
    exact up to rounding (each event's clipping is a box)."""
    Ss, St, _, _ = point_sums_adaptive(xyt, hst, grid, nthreads)
    h = np.asarray(hst, dtype=np.float64)
    ok = np.isfinite(h).all(axis=1) & (h[:, 0] > 0) & (h[:, 1] > 0)
    w = np.zeros(len(h))
    w[ok] = 1.0 / (h[ok, 0] ** 2 * h[ok, 1])
    return float(np.sum(Ss * St * w) / len(h) * grid.sres ** 2 * grid.tres)


def exact_evals_adaptive(xyt, hst, grid: Grid, nthreads=None):
    """Exact number of in-grid (voxel, event) pairs inside the event's supports."""
    _, _, cs, ct = point_sums_adaptive(xyt, hst, grid, nthreads)
    return int(np.sum(cs * ct))


def vb_grid_numpy_adaptive(xyt, hst, grid: Grid):
    """Alg. VB with per-event bandwidths over a whole (tiny) grid, in numpy:
    every voxel centre against every event, each term over hs_i^2 ht_i."""
    pts = _points(xyt)
    h = _bandwidths(hst, pts.shape[0])
    n = pts.shape[0]
    ok = np.all(np.isfinite(pts), axis=1) & np.all(np.isfinite(h), axis=1) & (h[:, 0] > 0) & (h[:, 1] > 0)
    p, hs, ht = pts[ok], h[ok, 0], h[ok, 1]
    out = np.zeros((grid.gx, grid.gy, grid.gt), dtype=np.float64)
    off = 0.0 if grid.corner else 0.5
    ts = grid.t0 + (np.arange(grid.gt) + off) * grid.tres
    for X in range(grid.gx):
        x = grid.x0 + (X + off) * grid.sres
        for Y in range(grid.gy):
            y = grid.y0 + (Y + off) * grid.sres
            r2 = (p[:, 0] - x) ** 2 + (p[:, 1] - y) ** 2
            inside = np.sqrt(r2) < hs
            if not np.any(inside):
                continue
            ksv = _np_ks(grid.kernel, (x - p[inside, 0]) / hs[inside], (y - p[inside, 1]) / hs[inside])
            dt = ts[None, :] - p[inside, 2][:, None]
            hti = ht[inside][:, None]
            ktv = np.where(np.abs(dt) <= hti, _np_kt(grid.kernel, np.clip(dt / hti, -1.0, 1.0)), 0.0)
            wgt = 1.0 / (hs[inside] ** 2 * ht[inside])
            out[X, Y, :] = np.sum((ksv * wgt)[:, None] * ktv, axis=0)
    return out / n
