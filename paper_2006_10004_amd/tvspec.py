"""Python binding of the tvspec C ABI (include/tvspec.h).

Argument marshalling only: every step of the decomposition runs in the HIP
kernels of libtvspec.so.  There is no CPU fallback; if the library is not
built, importing this module raises.

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch has already loaded (one runtime per process); torch is
used for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtvspec.so")

TVSPEC_OK = 0
TVSPEC_EINVAL = -1
TVSPEC_ENUMERIC = -2
TVSPEC_ENOMEM = -3
TVSPEC_EDEVICE = -4
TVSPEC_EBUSY = -5
TVSPEC_PENDING = 1
TVSPEC_PRECISION_F32 = 0
TVSPEC_PRECISION_F64 = 1
TVSPEC_PRECISION_MIXED = 2
PRECISIONS = {"f32": TVSPEC_PRECISION_F32, "f64": TVSPEC_PRECISION_F64, "mixed": TVSPEC_PRECISION_MIXED}
DEFAULT_PRECISION = "mixed"
TVSPEC_DEFAULT_TAU = 0.248
TVSPEC_PDHG_DEFAULT_STEP = 0.35355339059327373
TVSPEC_NSTATS = 4

EXPORTS = (
    "tvspec_decompose",
    "tvspec_decompose_dev",
    "tvspec_decompose_batch_dev",
    "tvspec_decompose_pdhg_dev",
    "tvspec_decompose_ex",
    "tvspec_decompose_noalloc_dev",
    "tvspec_default_options",
    "tvspec_dyadic_edges",
    "tvspec_timing_enable",
    "tvspec_timing_read",
    "tvspec_last_error",
    "tvspec_version",
    "tvspec_release",
    "tvspec_server_create",
    "tvspec_submit",
    "tvspec_poll",
    "tvspec_wait",
    "tvspec_server_info",
    "tvspec_server_destroy",
)


class _Request(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int), ("C", ctypes.c_int),
                ("dt", ctypes.c_double), ("K", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("band_edges", ctypes.c_void_p), ("n_bands", ctypes.c_int),
                ("bands", ctypes.c_void_p), ("S", ctypes.c_void_p), ("residual", ctypes.c_void_p),
                ("stats", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_ulonglong), ("admitted", ctypes.c_ulonglong),
                ("completed", ctypes.c_ulonglong), ("steps", ctypes.c_ulonglong),
                ("replays", ctypes.c_ulonglong), ("graph_builds", ctypes.c_ulonglong), ("buckets", ctypes.c_int),
                ("max_in_flight", ctypes.c_int), ("budget_bytes", ctypes.c_size_t),
                ("used_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t)]


class _Args(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int), ("C", ctypes.c_int),
                ("dt", ctypes.c_double), ("K", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("band_edges", ctypes.c_void_p), ("n_bands", ctypes.c_int),
                ("bands", ctypes.c_void_p), ("S", ctypes.c_void_p), ("residual", ctypes.c_void_p),
                ("stats", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("warm_start", ctypes.c_int), ("precision", ctypes.c_int), ("iters_per_launch", ctypes.c_int),
                ("device_ptrs", ctypes.c_int), ("stream", ctypes.c_void_p), ("tile_shape", ctypes.c_int)]


class _Report(ctypes.Structure):
    _fields_ = [("recon_err", ctypes.c_double), ("mean_err", ctypes.c_double), ("nonfinite", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


TVSPEC_SOLVER_CHAMBOLLE = 0
TVSPEC_SOLVER_PDHG = 1
SOLVERS = {"chambolle": TVSPEC_SOLVER_CHAMBOLLE, "pdhg": TVSPEC_SOLVER_PDHG}
TVSPEC_TILE_SQUARE = 0
TVSPEC_TILE_NARROW = 1
TILE_SHAPES = {"square": TVSPEC_TILE_SQUARE, "narrow": TVSPEC_TILE_NARROW}


class TvspecError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("tvspec error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("%s is not built (python -m paper_2006_10004_amd.build)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    i, d, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.tvspec_decompose.argtypes = [vp, i, i, i, d, i, i, vp, i, vp, vp, vp]
    lib.tvspec_decompose.restype = i
    lib.tvspec_decompose_dev.argtypes = [vp, i, i, i, d, i, i, vp, i, vp, vp, vp, vp, d, i, i, i, vp]
    lib.tvspec_decompose_dev.restype = i
    lib.tvspec_decompose_batch_dev.argtypes = [vp, i, i, i, i, i, vp, vp, vp, vp, vp, vp, vp, vp, d, i, i, i,
                                               vp]
    lib.tvspec_decompose_batch_dev.restype = i
    lib.tvspec_decompose_pdhg_dev.argtypes = [vp, i, i, i, d, i, i, vp, i, vp, vp, vp, vp, d, d, i, i, i, vp]
    lib.tvspec_decompose_pdhg_dev.restype = i
    lib.tvspec_decompose_noalloc_dev.argtypes = [vp, i, i, i, d, i, i, vp, i, vp, vp, vp, vp, d, i, i, i, vp]
    lib.tvspec_decompose_noalloc_dev.restype = i
    lib.tvspec_decompose_ex.argtypes = [ctypes.POINTER(_Args), ctypes.POINTER(_Options), ctypes.POINTER(_Report)]
    lib.tvspec_decompose_ex.restype = i
    lib.tvspec_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.tvspec_default_options.restype = None
    lib.tvspec_dyadic_edges.argtypes = [i, i, vp]
    lib.tvspec_dyadic_edges.restype = i
    lib.tvspec_timing_enable.argtypes = [i]
    lib.tvspec_timing_enable.restype = i
    lib.tvspec_timing_read.argtypes = [vp, vp, vp]
    lib.tvspec_timing_read.restype = i
    lib.tvspec_last_error.argtypes = []
    lib.tvspec_last_error.restype = ctypes.c_char_p
    lib.tvspec_version.argtypes = []
    lib.tvspec_version.restype = ctypes.c_char_p
    lib.tvspec_release.argtypes = []
    lib.tvspec_release.restype = None
    ull = ctypes.c_ulonglong
    lib.tvspec_server_create.argtypes = [ctypes.c_size_t, d, i, i, i, i, ctypes.POINTER(vp)]
    lib.tvspec_server_create.restype = i
    lib.tvspec_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(ull)]
    lib.tvspec_submit.restype = i
    lib.tvspec_poll.argtypes = [vp, ull, ctypes.POINTER(_Result)]
    lib.tvspec_poll.restype = i
    lib.tvspec_wait.argtypes = [vp, ull, ctypes.POINTER(_Result)]
    lib.tvspec_wait.restype = i
    lib.tvspec_server_info.argtypes = [vp, ctypes.POINTER(_ServerStats)]
    lib.tvspec_server_info.restype = i
    lib.tvspec_server_destroy.argtypes = [vp]
    lib.tvspec_server_destroy.restype = i
    return lib


_lib = _load()


def _check(rc: int):
    if rc != TVSPEC_OK:
        raise TvspecError(rc, tvspec_last_error())


def tvspec_last_error() -> str:
    return _lib.tvspec_last_error().decode()


def tvspec_version() -> str:
    return _lib.tvspec_version().decode()


def tvspec_release() -> None:
    _lib.tvspec_release()


def tvspec_timing_enable(on: bool) -> None:
    """Bracket every Chambolle kernel launch with hipEvents (benchmarks)."""
    _check(_lib.tvspec_timing_enable(1 if on else 0))


def tvspec_timing_read() -> dict:
    """Wait for the recorded launches; return and clear their summed kernel
    time (ms), launch count and pixel-iterations."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_longlong(0)
    pit = ctypes.c_longlong(0)
    _check(_lib.tvspec_timing_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pit)))
    return {"kernel_ms": ms.value, "launches": n.value, "pixel_iters": pit.value}


def tvspec_dyadic_edges(K: int, n_bands: int) -> list:
    """{0, 1, 2, 4, ..., 2^(B-2), K} (B = n_bands >= 2) or {0, K}."""
    e = (ctypes.c_int * (max(n_bands, 0) + 1))()
    _check(_lib.tvspec_dyadic_edges(int(K), int(n_bands), e))
    return list(e)


def _edges_array(edges):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32))
    if e.ndim != 1 or e.size < 2:
        raise ValueError("band_edges must be a 1-D sequence of n_bands+1 ints")
    return e


def _outputs(out, B, C, H, W, K, dev):
    """New output tensors, or a check of caller-provided ones."""
    want = {"bands": (B, C, H, W), "S": (C, K), "residual": (C, H, W), "stats": (TVSPEC_NSTATS,)}
    if out is None:
        return {k: torch.empty(shp, dtype=torch.float64, device=dev) for k, shp in want.items()}
    for k, shp in want.items():
        t = out[k]
        if tuple(t.shape) != shp or t.dtype != torch.float64 or t.device != dev or not t.is_contiguous():
            raise ValueError("out[%r] must be a contiguous float64 %s tensor on %s" % (k, shp, dev))
    return out


def tvspec_decompose(f: np.ndarray, dt: float, K: int, inner_iters: int, band_edges):
    """Host entry point (synchronous, default options).

    f: (C,H,W) or (H,W) float32 numpy array.  Returns dict of numpy arrays
    bands (B,C,H,W), S (C,K), residual (C,H,W)."""
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    f = np.ascontiguousarray(f, dtype=np.float32)
    C, H, W = f.shape
    e = _edges_array(band_edges)
    B = e.size - 1
    bands = np.empty((B, C, H, W), dtype=np.float64)
    S = np.empty((C, K), dtype=np.float64)
    res = np.empty((C, H, W), dtype=np.float64)
    _check(_lib.tvspec_decompose(f.ctypes.data, H, W, C, float(dt), int(K), int(inner_iters),
                                 e.ctypes.data, B, bands.ctypes.data, S.ctypes.data, res.ctypes.data))
    return {"bands": bands, "S": S, "residual": res}


def tvspec_decompose_dev(f: torch.Tensor, dt: float, K: int, inner_iters: int, band_edges,
                         tau: float = TVSPEC_DEFAULT_TAU, warm_start: bool = False,
                         precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0,
                         stream: torch.cuda.Stream | None = None, out: dict | None = None):
    """Device entry point: f is a (C,H,W) or (H,W) float32 tensor on a GPU.

    Enqueues on `stream` (default: torch's current stream) and returns
    without waiting.  Returns dict of device tensors bands (B,C,H,W), S (C,K),
    residual (C,H,W) and stats (4,) = [recon_err, mean_err, n_nonfinite, 0].
    `out` may pass preallocated tensors of those shapes."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda:
        raise TypeError("f must be a GPU tensor")
    if f.dtype != torch.float32:
        raise TypeError("f must be float32")
    if f.dim() == 2:
        f = f.unsqueeze(0)
    if f.dim() != 3:
        raise ValueError("f must be (C,H,W) or (H,W)")
    f = f.contiguous()
    C, H, W = f.shape
    e = _edges_array(band_edges)
    B = e.size - 1
    prec = PRECISIONS[precision]
    dev = f.device
    out = _outputs(out, B, C, H, W, int(K), dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(_lib.tvspec_decompose_dev(
            f.data_ptr(), H, W, C, float(dt), int(K), int(inner_iters), e.ctypes.data, B,
            out["bands"].data_ptr(), out["S"].data_ptr(), out["residual"].data_ptr(),
            out["stats"].data_ptr(), float(tau), 1 if warm_start else 0, prec,
            int(iters_per_launch), ctypes.c_void_p(st.cuda_stream)))
    return out


def tvspec_decompose_noalloc_dev(f: torch.Tensor, dt: float, K: int, inner_iters: int, band_edges, out: dict,
                                 tau: float = TVSPEC_DEFAULT_TAU, warm_start: bool = False,
                                 precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0,
                                 stream: torch.cuda.Stream | None = None):
    """Allocation-free variant of tvspec_decompose_dev: the library uses its
    fixed per-device scratch array and allocates nothing.  `out` must pass
    preallocated output tensors (bands (B,C,H,W), S (C,K), residual (C,H,W),
    stats (4,) float64 on f's device); they are returned."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32:
        raise TypeError("f must be a float32 GPU tensor")
    if f.dim() == 2:
        f = f.unsqueeze(0)
    if f.dim() != 3 or not f.is_contiguous():
        raise ValueError("f must be a contiguous (C,H,W) or (H,W) tensor")
    if out is None:
        raise ValueError("the allocation-free entry point needs preallocated outputs")
    C, H, W = f.shape
    e = _edges_array(band_edges)
    B = e.size - 1
    dev = f.device
    out = _outputs(out, B, C, H, W, int(K), dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(_lib.tvspec_decompose_noalloc_dev(
            f.data_ptr(), H, W, C, float(dt), int(K), int(inner_iters), e.ctypes.data, B,
            out["bands"].data_ptr(), out["S"].data_ptr(), out["residual"].data_ptr(),
            out["stats"].data_ptr(), float(tau), 1 if warm_start else 0, PRECISIONS[precision],
            int(iters_per_launch), ctypes.c_void_p(st.cuda_stream)))
    return out


def tvspec_decompose_pdhg_dev(f: torch.Tensor, dt: float, K: int, inner_iters: int, band_edges,
                              tau: float = 0.0, sigma: float = 0.0, warm_start: bool = False,
                              precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0,
                              stream: torch.cuda.Stream | None = None, out: dict | None = None):
    """As tvspec_decompose_dev, with the Chambolle-Pock primal-dual ROF solver
    (primal step tau, dual step sigma; 0, 0 = 1/sqrt(8) each)."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32:
        raise TypeError("f must be a float32 GPU tensor")
    if f.dim() == 2:
        f = f.unsqueeze(0)
    if f.dim() != 3:
        raise ValueError("f must be (C,H,W) or (H,W)")
    f = f.contiguous()
    C, H, W = f.shape
    e = _edges_array(band_edges)
    B = e.size - 1
    dev = f.device
    out = _outputs(out, B, C, H, W, int(K), dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(_lib.tvspec_decompose_pdhg_dev(
            f.data_ptr(), H, W, C, float(dt), int(K), int(inner_iters), e.ctypes.data, B,
            out["bands"].data_ptr(), out["S"].data_ptr(), out["residual"].data_ptr(),
            out["stats"].data_ptr(), float(tau), float(sigma), 1 if warm_start else 0,
            PRECISIONS[precision], int(iters_per_launch), ctypes.c_void_p(st.cuda_stream)))
    return out


def tvspec_default_options() -> dict:
    """The options tvspec_decompose_ex uses when given none."""
    o = _Options()
    _lib.tvspec_default_options(ctypes.byref(o))
    return {k: getattr(o, k) for k, _ in _Options._fields_}


def tvspec_decompose_ex(f, dt: float, K: int, inner_iters: int, band_edges, solver: str = "chambolle",
                        tau: float = 0.0, sigma: float = 0.0, warm_start: bool = False,
                        precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0,
                        stream: torch.cuda.Stream | None = None, report: bool = True, out: dict | None = None,
                        tile_shape: str = "square"):
    """tvspec_decompose_ex: f is a (C,H,W)/(H,W) float32 numpy array (host
    buffers, synchronous) or GPU tensor (device buffers on `stream`);
    tile_shape "square" (32 x 32) or "narrow" (32 x 16) for the Chambolle
    tile kernel.

    Returns (outputs, report): outputs as tvspec_decompose (numpy) or
    tvspec_decompose_dev (tensors, with stats); report a dict of recon_err,
    mean_err, nonfinite, device_ms, total_ms, or None with report=False."""
    e = _edges_array(band_edges)
    B = e.size - 1
    o = _Options()
    _lib.tvspec_default_options(ctypes.byref(o))
    o.solver = SOLVERS[solver]
    o.tau = float(tau)
    o.sigma = float(sigma)
    o.warm_start = 1 if warm_start else 0
    o.precision = PRECISIONS[precision]
    o.iters_per_launch = int(iters_per_launch)
    o.tile_shape = TILE_SHAPES[tile_shape]
    if isinstance(f, torch.Tensor):
        if not f.is_cuda or f.dtype != torch.float32:
            raise TypeError("a tensor f must be a float32 GPU tensor")
        if f.dim() == 2:
            f = f.unsqueeze(0)
        if f.dim() != 3:
            raise ValueError("f must be (C,H,W) or (H,W)")
        f = f.contiguous()
        C, H, W = f.shape
        dev = f.device
        outs = _outputs(out, B, C, H, W, int(K), dev)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        o.device_ptrs = 1
        o.stream = st.cuda_stream
        args = _Args(f.data_ptr(), H, W, C, float(dt), int(K), int(inner_iters), e.ctypes.data, B,
                     outs["bands"].data_ptr(), outs["S"].data_ptr(), outs["residual"].data_ptr(),
                     outs["stats"].data_ptr())
    else:
        f = np.asarray(f)
        if f.ndim == 2:
            f = f[None]
        f = np.ascontiguousarray(f, dtype=np.float32)
        C, H, W = f.shape
        outs = {"bands": np.empty((B, C, H, W), dtype=np.float64), "S": np.empty((C, K), dtype=np.float64),
                "residual": np.empty((C, H, W), dtype=np.float64),
                "stats": np.empty((TVSPEC_NSTATS,), dtype=np.float64)}
        o.device_ptrs = 0
        args = _Args(f.ctypes.data, H, W, C, float(dt), int(K), int(inner_iters), e.ctypes.data, B,
                     outs["bands"].ctypes.data, outs["S"].ctypes.data, outs["residual"].ctypes.data,
                     outs["stats"].ctypes.data)
        dev = None
    rep = _Report() if report else None
    if dev is not None:
        with torch.cuda.device(dev):
            rc = _lib.tvspec_decompose_ex(ctypes.byref(args), ctypes.byref(o),
                                          ctypes.byref(rep) if rep is not None else None)
    else:
        rc = _lib.tvspec_decompose_ex(ctypes.byref(args), ctypes.byref(o),
                                      ctypes.byref(rep) if rep is not None else None)
    _check(rc)
    return outs, ({k: getattr(rep, k) for k, _ in _Report._fields_} if rep is not None else None)


def tvspec_decompose_batch_dev(f: torch.Tensor, dt, K, inner_iters: int, band_edges,
                               tau: float = TVSPEC_DEFAULT_TAU, warm_start: bool = False,
                               precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0,
                               stream: torch.cuda.Stream | None = None):
    """Batched device entry point: f is a (B,C,H,W) float32 GPU tensor; dt and K
    are length-B sequences, band_edges a length-B sequence of edge lists.

    Returns a list of B dicts (views into shared output tensors) with bands
    (n_bands_b,C,H,W), S (C,K_b), residual (C,H,W) and stats (4,)."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32 or f.dim() != 4:
        raise TypeError("f must be a (B,C,H,W) float32 GPU tensor")
    f = f.contiguous()
    B, C, H, W = f.shape
    dt_a = np.ascontiguousarray(np.asarray(dt, dtype=np.float64))
    K_a = np.ascontiguousarray(np.asarray(K, dtype=np.int32))
    if dt_a.shape != (B,) or K_a.shape != (B,) or len(band_edges) != B:
        raise ValueError("dt, K and band_edges need one entry per image")
    edges = [_edges_array(e) for e in band_edges]
    nb = np.ascontiguousarray(np.array([e.size - 1 for e in edges], dtype=np.int32))
    edges_cat = np.ascontiguousarray(np.concatenate(edges).astype(np.int32))
    dev = f.device
    bands = torch.empty((int(nb.sum()) * C * H * W,), dtype=torch.float64, device=dev)
    S = torch.empty((int(C * K_a.sum()),), dtype=torch.float64, device=dev)
    res = torch.empty((B, C, H, W), dtype=torch.float64, device=dev)
    stats = torch.empty((B, TVSPEC_NSTATS), dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(_lib.tvspec_decompose_batch_dev(
            f.data_ptr(), B, H, W, C, int(inner_iters), dt_a.ctypes.data, K_a.ctypes.data,
            edges_cat.ctypes.data, nb.ctypes.data, bands.data_ptr(), S.data_ptr(), res.data_ptr(),
            stats.data_ptr(), float(tau), 1 if warm_start else 0, PRECISIONS[precision],
            int(iters_per_launch), ctypes.c_void_p(st.cuda_stream)))
    out = []
    bo = so = 0
    for b in range(B):
        nbb, Kb = int(nb[b]), int(K_a[b])
        out.append({
            "bands": bands[bo:bo + nbb * C * H * W].view(nbb, C, H, W),
            "S": S[so:so + C * Kb].view(C, Kb),
            "residual": res[b],
            "stats": stats[b],
        })
        bo += nbb * C * H * W
        so += C * Kb
    return out


def tvspec_server_create(budget_bytes: int, tau: float = TVSPEC_DEFAULT_TAU, warm_start: bool = False,
                         precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0,
                         use_graphs: bool = True) -> ctypes.c_void_p:
    """Create a server on the current device; returns its handle."""
    h = ctypes.c_void_p()
    _check(_lib.tvspec_server_create(int(budget_bytes), float(tau), 1 if warm_start else 0,
                                     PRECISIONS[precision], int(iters_per_launch), 1 if use_graphs else 0,
                                     ctypes.byref(h)))
    return h


def tvspec_submit(handle, f_ptr: int, H: int, W: int, C: int, dt: float, K: int, inner_iters: int,
                  band_edges, bands_ptr: int, S_ptr: int, residual_ptr: int, stats_ptr: int) -> int:
    """Queue a request given device pointers; returns its ticket."""
    e = _edges_array(band_edges)
    req = _Request(f_ptr, int(H), int(W), int(C), float(dt), int(K), int(inner_iters), e.ctypes.data,
                   e.size - 1, bands_ptr, S_ptr, residual_ptr, stats_ptr)
    t = ctypes.c_ulonglong(0)
    _check(_lib.tvspec_submit(handle, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def _result(rc, r):
    if rc == TVSPEC_PENDING:
        return None
    _check(rc)
    return {"queue_ms": r.queue_ms, "latency_ms": r.latency_ms}


def tvspec_poll(handle, ticket: int):
    """None while pending, else {queue_ms, latency_ms} (the ticket is retired)."""
    r = _Result()
    return _result(_lib.tvspec_poll(handle, ctypes.c_ulonglong(ticket), ctypes.byref(r)), r)


def tvspec_wait(handle, ticket: int):
    """Block until complete; {queue_ms, latency_ms} (the ticket is retired)."""
    r = _Result()
    return _result(_lib.tvspec_wait(handle, ctypes.c_ulonglong(ticket), ctypes.byref(r)), r)


def tvspec_server_info(handle) -> dict:
    st = _ServerStats()
    _check(_lib.tvspec_server_info(handle, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in _ServerStats._fields_}


def tvspec_server_destroy(handle) -> None:
    _check(_lib.tvspec_server_destroy(handle))


class Server:
    """Continuous-batching decomposition server on the current device
    (tvspec_server_create and friends).

    submit() queues a (C,H,W) or (H,W) float32 GPU tensor and returns a ticket
    and the output tensors it will fill; poll() / wait() report completion.
    The binding keeps the request's tensors alive until its ticket completes.
    Results equal tvspec_decompose_dev's with the server's options."""

    def __init__(self, budget_bytes: int, tau: float = TVSPEC_DEFAULT_TAU, warm_start: bool = False,
                 precision: str = DEFAULT_PRECISION, iters_per_launch: int = 0, use_graphs: bool = True):
        self._h = tvspec_server_create(budget_bytes, tau, warm_start, precision, iters_per_launch, use_graphs)
        self._live = {}
        # tensors of failed tickets: work enqueued before the failure may
        # still read or write them until tvspec_server_destroy has
        # synchronised the server's streams, so they are kept until close()
        self._graveyard = []

    def submit(self, f: torch.Tensor, dt: float, K: int, inner_iters: int, band_edges, sync: bool = True,
               out: dict | None = None):
        """Queue one image.  With sync=True (default) torch's current stream is
        synchronised first, so that work writing f (and the allocation of the
        outputs) is complete before the server's streams use them.  Returns
        (ticket, outputs) with outputs a dict of bands (B,C,H,W), S (C,K),
        residual (C,H,W) and stats (4,) device tensors (`out` may pass
        preallocated ones of those shapes)."""
        if self._h is None:
            raise RuntimeError("server is closed")
        if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32:
            raise TypeError("f must be a float32 GPU tensor")
        if f.dim() == 2:
            f = f.unsqueeze(0)
        if f.dim() != 3:
            raise ValueError("f must be (C,H,W) or (H,W)")
        f = f.contiguous()
        C, H, W = f.shape
        e = _edges_array(band_edges)
        B = e.size - 1
        dev = f.device
        out = _outputs(out, B, C, H, W, int(K), dev)
        if sync:
            torch.cuda.current_stream(dev).synchronize()
        t = tvspec_submit(self._h, f.data_ptr(), H, W, C, dt, K, inner_iters, e, out["bands"].data_ptr(),
                          out["S"].data_ptr(), out["residual"].data_ptr(), out["stats"].data_ptr())
        self._live[t] = (f, out)
        return t, out

    def _bury(self, ticket):
        t = self._live.pop(ticket, None)
        if t is not None:
            self._graveyard.append(t)

    def poll(self, ticket: int):
        """None while pending; {queue_ms, latency_ms} once complete."""
        try:
            r = tvspec_poll(self._h, ticket)
        except TvspecError:
            self._bury(ticket)
            raise
        if r is not None:
            self._live.pop(ticket, None)
        return r

    def wait(self, ticket: int):
        """Block until the ticket completes; {queue_ms, latency_ms}."""
        try:
            r = tvspec_wait(self._h, ticket)
        except TvspecError:
            self._bury(ticket)
            raise
        self._live.pop(ticket, None)
        return r

    def info(self) -> dict:
        return tvspec_server_info(self._h)

    def close(self) -> None:
        if self._h is not None:
            h, self._h = self._h, None
            try:
                tvspec_server_destroy(h)
            finally:
                self._live.clear()
                self._graveyard.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
