"""Python binding of the gfx950 space-time kernel density library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libstkde.so`` behind the C ABI of ``include/stkde.h``.  PyTorch
supplies device memory and the stream.  There is no CPU fallback: if the
library is missing, importing :func:`lib` raises.

The estimator (Sec. 2.1 of Saule et al., arXiv 1705.09366) is

    f[X][Y][T] = 1/(n hs^2 ht) sum_i ks(u, v) kt(w)

with Epanechnikov kernels ks = (2/pi)(1 - u^2 - v^2) on the unit disc and
kt = (3/4)(1 - w^2) on [-1, 1], evaluated at voxel centres; it is computed
by the point-based, symmetry-exploiting PB-SYM method (Sec. 3.2) organised
as an atomic-free gather over output tiles.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstkde.so")

STKDE_OK = 0
STKDE_ERR_INVALID_ARG = -1
STKDE_ERR_TOO_LARGE = -2
STKDE_ERR_WORKSPACE = -3
STKDE_ERR_HIP = -4
STKDE_ERR_UNSUPPORTED = -5

FLAG_KAHAN = 1
FLAG_MASS = 4
FLAG_POINT_STATS = 8
FLAG_ADAPTIVE = 16
FLAG_CORNER = 32
# Kernel pairs (include/stkde.h): flags |= kernel_flag(KERNEL_*)
KERNEL_EPANECHNIKOV, KERNEL_QUARTIC, KERNEL_GAUSSIAN, KERNEL_PRINTED = 0, 1, 2, 3


def kernel_flag(kernel: int) -> int:
    """The desc flag bits that select a kernel pair."""
    return (int(kernel) & 0xF) << 8

EXPORTED = ("stkde_plan", "stkde_plan_destroy", "stkde_workspace_bytes", "stkde_compute",
            "stkde_bin", "stkde_accumulate", "stkde_status_string", "stkde_version",
            "stkde_set_plan", "stkde_set_bytes", "stkde_set_build", "stkde_set_destroy",
            "stkde_batch_plan", "stkde_batch_workspace_bytes", "stkde_batch_run",
            "stkde_batch_capture", "stkde_batch_replay", "stkde_batch_destroy",
            "stkde_plan_profile", "stkde_plan_profile_read",
            "stkde_ablation_accumulate", "stkde_ablation_compute",
            "stkde_compute_adaptive", "stkde_bin_adaptive", "stkde_plan_capture", "stkde_plan_replay",
            "stkde_compute_noalloc", "stkde_batch_passes")

# Bytes of the library's own device scratch (stkde_compute_noalloc).
STATIC_SCRATCH_BYTES = 128 << 20

# Baselines of include/stkde_ablation.h (benchmarks and tests only).
ABLATION_SCATTER = 1
ABLATION_VOXEL = 2


class StkdeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class _Desc(ctypes.Structure):
    _fields_ = [("gx", ctypes.c_int64), ("gy", ctypes.c_int64), ("gt", ctypes.c_int64),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("t0", ctypes.c_double),
                ("sres", ctypes.c_double), ("tres", ctypes.c_double),
                ("hs", ctypes.c_double), ("ht", ctypes.c_double), ("flags", ctypes.c_uint32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("tile_t", ctypes.c_int32), ("cell_xy", ctypes.c_int32),
                ("cell_t", ctypes.c_int32), ("split_share", ctypes.c_int32),
                ("kahan_mode", ctypes.c_int32), ("operand_form", ctypes.c_int32)]


class _Item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("set", ctypes.c_void_p), ("d_set", ctypes.c_void_p),
                ("ox", ctypes.c_int64), ("oy", ctypes.c_int64), ("ot", ctypes.c_int64),
                ("d_out", ctypes.c_void_p), ("d_stats", ctypes.c_void_p)]


_LIB = None


def lib():
    """Load libstkde.so (built in-tree by ``build.py``); raise if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1705_09366_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.stkde_plan.argtypes = [P(_Desc), P(_Tuning), P(ctypes.c_void_p)]
        L.stkde_plan_destroy.argtypes = [ctypes.c_void_p]
        L.stkde_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int64, P(ctypes.c_size_t)]
        L.stkde_compute.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_void_p]
        L.stkde_bin.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_size_t, ctypes.c_void_p]
        L.stkde_compute_adaptive.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
        L.stkde_bin_adaptive.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p]
        L.stkde_accumulate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_void_p]
        L.stkde_set_plan.argtypes = [P(_Desc), P(_Tuning), ctypes.c_int64, P(ctypes.c_void_p)]
        L.stkde_set_bytes.argtypes = [ctypes.c_void_p, P(ctypes.c_size_t), P(ctypes.c_size_t)]
        L.stkde_set_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p]
        L.stkde_set_destroy.argtypes = [ctypes.c_void_p]
        L.stkde_batch_plan.argtypes = [P(_Item), ctypes.c_int32, P(ctypes.c_void_p)]
        L.stkde_batch_workspace_bytes.argtypes = [ctypes.c_void_p, P(ctypes.c_size_t)]
        L.stkde_batch_passes.argtypes = [ctypes.c_void_p, P(ctypes.c_int32)]
        L.stkde_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p]
        L.stkde_batch_capture.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        L.stkde_batch_replay.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.stkde_batch_destroy.argtypes = [ctypes.c_void_p]
        L.stkde_plan_profile.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.stkde_ablation_accumulate.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                                ctypes.c_void_p]
        L.stkde_ablation_compute.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]
        L.stkde_plan_profile_read.argtypes = [ctypes.c_void_p, P(ctypes.c_float), ctypes.c_int32,
                                              P(ctypes.c_int32)]
        L.stkde_plan_capture.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.stkde_plan_replay.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.stkde_compute_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        for name in EXPORTED:
            if name not in ("stkde_status_string", "stkde_version"):
                getattr(L, name).restype = ctypes.c_int
        L.stkde_status_string.argtypes = [ctypes.c_int]
        L.stkde_status_string.restype = ctypes.c_char_p
        L.stkde_version.restype = ctypes.c_int32
        _LIB = L
    return _LIB


def status_string(status: int) -> str:
    return lib().stkde_status_string(int(status)).decode()


@dataclass(frozen=True)
class Desc:
    """Problem description (Sec. 2.1, Table "Notations"): a gx x gy x gt
    grid of sres x sres x tres voxels cornered at (x0, y0, t0), bandwidths
    hs, ht in domain units."""
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
    flags: int = 0

    def _c(self):
        return _Desc(self.gx, self.gy, self.gt, self.x0, self.y0, self.t0, self.sres, self.tres,
                     self.hs, self.ht, self.flags)


@dataclass(frozen=True)
class Tuning:
    """Tuning of one plan (0 = library default): time rows per tile, bin
    edges, the split share of the work list, where compensated accumulation
    keeps its running pair (1 registers, 2 memory), and the matrix-core
    operands (0 two FP16 terms where the gather has that form, 1 FP32)."""
    tile_t: int = 0
    cell_xy: int = 0
    cell_t: int = 0
    split_share: int = 0
    kahan_mode: int = 0
    operand_form: int = 0

    def _c(self):
        return _Tuning(self.tile_t, self.cell_xy, self.cell_t, self.split_share, self.kahan_mode,
                       self.operand_form)


class Plan:
    """A plan for one grid and bandwidth pair: ``Plan(desc)(points)`` returns
    the FP32 density grid as a [gx, gy, gt] CUDA tensor."""

    def __init__(self, desc: Desc, tuning: Optional[Tuning] = None):
        self.desc = desc
        self.tuning = tuning
        h = ctypes.c_void_p()
        st = lib().stkde_plan(ctypes.byref(desc._c()),
                              ctypes.byref(tuning._c()) if tuning is not None else None,
                              ctypes.byref(h))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_plan")
        self._h = h
        self._ws = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().stkde_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def profile(self, capacity: int):
        """Record HIP events around the gather kernel of the next
        ``capacity`` computations (0 turns it off)."""
        st = lib().stkde_plan_profile(self._h, int(capacity))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_plan_profile")
        self._prof_cap = int(capacity)

    def profile_read(self):
        """Gather kernel durations (ms) of the recorded computations, in order."""
        cap = max(1, getattr(self, "_prof_cap", 0))
        buf = (ctypes.c_float * cap)()
        cnt = ctypes.c_int32(0)
        st = lib().stkde_plan_profile_read(self._h, buf, cap, ctypes.byref(cnt))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_plan_profile_read")
        return [float(buf[i]) for i in range(cnt.value)]

    def workspace_bytes(self, n: int) -> int:
        b = ctypes.c_size_t(0)
        st = lib().stkde_workspace_bytes(self._h, int(n), ctypes.byref(b))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_workspace_bytes")
        return int(b.value)

    def workspace(self, n: int, device=None):
        """A cached uint8 workspace tensor large enough for n points."""
        import torch
        need = self.workspace_bytes(n)
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self._ws is None or self._ws.numel() < need or self._ws.device != dev:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        return self._ws

    def compute_into(self, points, out, stats=None, workspace=None, stream=None):
        """Enqueue the computation on ``stream`` (default: torch's current
        stream).  points: [n, 3] float64 CUDA tensor; out: float32 CUDA tensor
        with gx*gy*gt elements; stats: optional float64 CUDA tensor of 8."""
        import torch
        n = int(points.shape[0])
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("points must be a [n, 3] float64 CUDA tensor")
        if not points.is_contiguous():
            raise ValueError("points must be contiguous")
        d = self.desc
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        if stats is not None and (stats.dtype != torch.float64 or stats.numel() < 8 or not stats.is_cuda):
            raise ValueError("stats must be a float64 CUDA tensor of 8 elements")
        ws = workspace if workspace is not None else self.workspace(n, points.device)
        base = ws.data_ptr()
        off = (-base) % 256
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        st = lib().stkde_compute(self._h, ctypes.c_void_p(points.data_ptr()), n,
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(base + off),
                                 ctypes.c_size_t(ws.numel() - off),
                                 ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                 ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_compute")
        return out

    def compute_noalloc(self, points, out, stats=None, stream=None):
        """As :meth:`compute_into`, with the library's own device scratch as
        the workspace (``stkde_compute_noalloc``): nothing is allocated, by
        the library or here.  Calls that may overlap on one GPU race."""
        import torch
        n = int(points.shape[0])
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 or points.shape[1] != 3 \
                or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor")
        d = self.desc
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        if stats is not None and (stats.dtype != torch.float64 or stats.numel() < 8 or not stats.is_cuda):
            raise ValueError("stats must be a float64 CUDA tensor of 8 elements")
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        st = lib().stkde_compute_noalloc(self._h, ctypes.c_void_p(points.data_ptr()), n,
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                         ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_compute_noalloc")
        return out

    def capture(self, points, out, stats=None, workspace=None):
        """Record one :meth:`compute_into` with these tensors as a HIP graph
        (``stkde_plan_capture``); :meth:`replay` launches it.  The tensors
        must stay alive while the graph is replayed; a replay reads the
        values ``points`` holds when it runs."""
        import torch
        n = int(points.shape[0])
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 or points.shape[1] != 3 \
                or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor")
        d = self.desc
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        if stats is not None and (stats.dtype != torch.float64 or stats.numel() < 8 or not stats.is_cuda):
            raise ValueError("stats must be a float64 CUDA tensor of 8 elements")
        ws = workspace if workspace is not None else self.workspace(n, points.device)
        p, nb = self._ws_args(ws)
        st = lib().stkde_plan_capture(self._h, ctypes.c_void_p(points.data_ptr()), n,
                                      ctypes.c_void_p(out.data_ptr()), p, nb,
                                      ctypes.c_void_p(stats.data_ptr()) if stats is not None else None)
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_plan_capture")
        self._graph_refs = (points, out, stats, ws)  # kept alive for the replays
        return out

    def replay(self, stream=None):
        """Launch the recorded graph on ``stream`` (default: the current one)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        st = lib().stkde_plan_replay(self._h, ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_plan_replay")

    def _ws_args(self, ws):
        base = ws.data_ptr()
        off = (-base) % 256
        return ctypes.c_void_p(base + off), ctypes.c_size_t(ws.numel() - off)

    def bin(self, points, workspace, stream=None):
        """Stage 1 (stkde_bin): bin the [n, 3] float64 points into workspace."""
        import torch
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 \
                or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor")
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        p, nb = self._ws_args(workspace)
        st = lib().stkde_bin(self._h, ctypes.c_void_p(points.data_ptr()), int(points.shape[0]), p, nb,
                             ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_bin")

    def accumulate(self, n, out, workspace, stats=None, stream=None):
        """Stage 2 (stkde_accumulate): gather and store the grid from a
        workspace that :meth:`bin` filled for the same n."""
        import torch
        d = self.desc
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        if stats is not None and (stats.dtype != torch.float64 or stats.numel() < 8 or not stats.is_cuda):
            raise ValueError("stats must be a float64 CUDA tensor of 8 elements")
        if stream is None:
            stream = torch.cuda.current_stream(out.device)
        p, nb = self._ws_args(workspace)
        st = lib().stkde_accumulate(self._h, int(n), ctypes.c_void_p(out.data_ptr()), p, nb,
                                    ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                    ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_accumulate")
        return out

    @staticmethod
    def _check_pairs(points, pairs):
        import torch
        n = int(points.shape[0])
        if pairs.dtype != torch.float64 or not pairs.is_cuda or tuple(pairs.shape) != (n, 2) \
                or not pairs.is_contiguous():
            raise ValueError("pairs must be a contiguous [n, 2] float64 CUDA tensor of (hs_i, ht_i)")

    def compute_adaptive_into(self, points, pairs, out, stats=None, workspace=None, stream=None):
        """Per-point bandwidths (plan with FLAG_ADAPTIVE): points [n, 3] and
        pairs [n, 2] (hs_i, ht_i) float64 CUDA tensors; as :meth:`compute_into`."""
        import torch
        n = int(points.shape[0])
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 \
                or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor")
        self._check_pairs(points, pairs)
        d = self.desc
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        if stats is not None and (stats.dtype != torch.float64 or stats.numel() < 8 or not stats.is_cuda):
            raise ValueError("stats must be a float64 CUDA tensor of 8 elements")
        ws = workspace if workspace is not None else self.workspace(n, points.device)
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        p, nb = self._ws_args(ws)
        st = lib().stkde_compute_adaptive(self._h, ctypes.c_void_p(points.data_ptr()),
                                          ctypes.c_void_p(pairs.data_ptr()), n,
                                          ctypes.c_void_p(out.data_ptr()), p, nb,
                                          ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                          ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_compute_adaptive")
        return out

    def compute_adaptive(self, points, pairs, stats=None):
        """The density grid with per-point bandwidths as a [gx, gy, gt] tensor."""
        import torch
        d = self.desc
        out = torch.empty((d.gx, d.gy, d.gt), dtype=torch.float32, device=points.device)
        return self.compute_adaptive_into(points, pairs, out, stats=stats)

    def bin_adaptive(self, points, pairs, workspace, stream=None):
        """Stage 1 with per-point bandwidths (stkde_bin_adaptive)."""
        import torch
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 \
                or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor")
        self._check_pairs(points, pairs)
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        p, nb = self._ws_args(workspace)
        st = lib().stkde_bin_adaptive(self._h, ctypes.c_void_p(points.data_ptr()),
                                      ctypes.c_void_p(pairs.data_ptr()), int(points.shape[0]), p, nb,
                                      ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_bin_adaptive")

    def ablation_accumulate(self, method: int, n, out, workspace, stream=None):
        """Baseline accumulation (stkde_ablation_accumulate): ABLATION_SCATTER
        or ABLATION_VOXEL over a workspace that :meth:`bin` filled for n."""
        import torch
        d = self.desc
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        if stream is None:
            stream = torch.cuda.current_stream(out.device)
        p, nb = self._ws_args(workspace)
        st = lib().stkde_ablation_accumulate(self._h, int(method), int(n), ctypes.c_void_p(out.data_ptr()),
                                             p, nb, ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_ablation_accumulate")
        return out

    def ablation_compute(self, method: int, points, out=None, stream=None):
        """Bin then run a baseline accumulation (stkde_ablation_compute)."""
        import torch
        d = self.desc
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 \
                or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor")
        if out is None:
            out = torch.empty((d.gx, d.gy, d.gt), dtype=torch.float32, device=points.device)
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != d.gx * d.gy * d.gt \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
        n = int(points.shape[0])
        ws = self.workspace(n, points.device)
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        p, nb = self._ws_args(ws)
        st = lib().stkde_ablation_compute(self._h, int(method), ctypes.c_void_p(points.data_ptr()), n,
                                          ctypes.c_void_p(out.data_ptr()), p, nb,
                                          ctypes.c_void_p(stream.cuda_stream))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_ablation_compute")
        return out

    def __call__(self, points, stats=None):
        import torch
        d = self.desc
        out = torch.empty((d.gx, d.gy, d.gt), dtype=torch.float32, device=points.device)
        return self.compute_into(points, out, stats=stats)


def _aligned(t):
    """(pointer, bytes) of a uint8 tensor from its first 256-byte boundary."""
    base = t.data_ptr()
    off = (-base) % 256
    return ctypes.c_void_p(base + off), ctypes.c_size_t(t.numel() - off)


def _stream_arg(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class BinnedSet:
    """A point set binned once on the device for a base grid (``stkde_set_*``):
    reusable by any number of :class:`Batch` items on the base grid or a
    window of it, with bandwidths up to ``base.hs``, ``base.ht``."""

    def __init__(self, base: Desc, n: int, tuning: Optional[Tuning] = None):
        if base.flags:
            raise ValueError("a set's base desc carries no flags")
        self.base = base
        self.n = int(n)
        h = ctypes.c_void_p()
        st = lib().stkde_set_plan(ctypes.byref(base._c()),
                                  ctypes.byref(tuning._c()) if tuning is not None else None,
                                  self.n, ctypes.byref(h))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_set_plan")
        self._h = h
        sb, cb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        st = lib().stkde_set_bytes(h, ctypes.byref(sb), ctypes.byref(cb))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_set_bytes")
        self.set_bytes, self.scratch_bytes = int(sb.value), int(cb.value)
        self.mem = None

    @property
    def handle(self):
        return self._h

    def build(self, points, scratch=None, stream=None):
        """Bin the [n, 3] float64 CUDA points into device memory held by this
        object (``self.mem``)."""
        import torch
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 \
                or points.shape[1] != 3 or not points.is_contiguous() or points.shape[0] != self.n:
            raise ValueError("points must be a contiguous [n, 3] float64 CUDA tensor of the set's n")
        if self.mem is None or self.mem.device != points.device:
            self.mem = torch.empty(self.set_bytes + 256, dtype=torch.uint8, device=points.device)
        if scratch is None:
            scratch = torch.empty(self.scratch_bytes + 256, dtype=torch.uint8, device=points.device)
        mp, mb = _aligned(self.mem)
        sp, sb = _aligned(scratch)
        st = lib().stkde_set_build(self._h, ctypes.c_void_p(points.data_ptr()), mp, mb, sp, sb,
                                   _stream_arg(stream, points.device))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_set_build")
        self._scratch = scratch  # kept until the stream has passed the build
        return self

    def device_ptr(self):
        if self.mem is None:
            raise RuntimeError("set not built")
        return _aligned(self.mem)[0]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().stkde_set_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Item:
    """One grid of a batch: ``plan`` gives the grid and bandwidths (its
    origin must be base voxel (ox, oy, ot) of the set), ``out`` the float32
    CUDA tensor it is written to, ``stats`` an optional float64 tensor of 8."""
    plan: "Plan"
    set: BinnedSet
    out: object
    ox: int = 0
    oy: int = 0
    ot: int = 0
    stats: object = None


class Batch:
    """Many grids in one work list and one persistent gather launch (per
    (tile_t, Kahan, operand form) group when the grids do not fit one
    multi-variant launch; ``stkde_batch_*``); optionally recorded once as a
    HIP graph and replayed.  ``allocate=False`` plans (and validates) only;
    :meth:`allocate` then provides the workspace."""

    def __init__(self, items, allocate: bool = True):
        import torch
        self.items = list(items)
        arr = (_Item * len(self.items))()
        for k, it in enumerate(self.items):
            d = it.plan.desc
            if it.out.dtype != torch.float32 or not it.out.is_cuda or not it.out.is_contiguous() \
                    or it.out.numel() != d.gx * d.gy * d.gt:
                raise ValueError("out must be a contiguous float32 CUDA tensor of gx*gy*gt elements")
            if it.stats is not None and (it.stats.dtype != torch.float64 or it.stats.numel() < 8
                                         or not it.stats.is_cuda):
                raise ValueError("stats must be a float64 CUDA tensor of 8 elements")
            arr[k] = _Item(it.plan.handle.value, it.set.handle.value, it.set.device_ptr().value,
                           it.ox, it.oy, it.ot, it.out.data_ptr(),
                           it.stats.data_ptr() if it.stats is not None else None)
        h = ctypes.c_void_p()
        st = lib().stkde_batch_plan(arr, len(self.items), ctypes.byref(h))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_batch_plan")
        self._h = h
        b = ctypes.c_size_t(0)
        st = lib().stkde_batch_workspace_bytes(h, ctypes.byref(b))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_batch_workspace_bytes")
        self.workspace_bytes = int(b.value)
        self.ws = None
        if allocate:
            self.allocate(self.items[0].out.device)

    def passes(self) -> int:
        """Passes (gather launches) a run enqueues (``stkde_batch_passes``)."""
        v = ctypes.c_int32(0)
        st = lib().stkde_batch_passes(self._h, ctypes.byref(v))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_batch_passes")
        return int(v.value)

    def allocate(self, device=None):
        import torch
        dev = device if device is not None else self.items[0].out.device
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        return self

    def run(self, stream=None):
        p, nb = _aligned(self.ws)
        st = lib().stkde_batch_run(self._h, p, nb, _stream_arg(stream, self.ws.device))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_batch_run")

    def capture(self):
        p, nb = _aligned(self.ws)
        st = lib().stkde_batch_capture(self._h, p, nb)
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_batch_capture")

    def replay(self, stream=None):
        st = lib().stkde_batch_replay(self._h, _stream_arg(stream, self.ws.device))
        if st != STKDE_OK:
            raise StkdeError(st, "stkde_batch_replay")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().stkde_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compute(points, desc: Desc, tuning: Optional[Tuning] = None, stats=None):
    """One-shot convenience: plan, compute, return the [gx, gy, gt] grid."""
    return Plan(desc, tuning)(points, stats=stats)
