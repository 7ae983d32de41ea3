"""Python binding of the exact Tukey-depth library (libtd.so, gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI of ``include/td.h``.  PyTorch supplies device memory
and the current stream.  There is no CPU fallback: if the library is not
built, or no GPU is visible, calls raise.

    import torch, paper_1409_3901_amd as td
    counts = td.depth(X, Z)                  # int32, counts[q] = n * D_n(Z_q)
    counts = td.depth(X, Z, precision="plain")
    outs = td.depth_batched([(X1, Z1), (X2, Z2)])
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libtd.so")

TD_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported request", 3: "out of device memory",
          4: "HIP runtime error", 5: "some queries failed (see device_status)", 6: "no HIP device",
          7: "call too large for the static workspace"}
PRECISION = {"plain": 0, "fp64": 0, "filtered": 1, "fp32": 1, "exact": 2}
SWEEP = {"auto": 0, "bucket": 0, "bitonic": 1}
METHOD = {"rcom": 0, "adia": 1, "vertex": 2}
DEV_BITS = {1: "nonfinite", 2: "no_valid_subset", 4: "defer_overflow", 8: "exact_range",
            16: "degeneracy_limit", 32: "not_general"}
MAX_P = 8
MAX_N = 1024


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("filter_scale", ctypes.c_double),
        ("force_exact", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("deferred_capacity", ctypes.c_int64),
        ("sweep", ctypes.c_int32),
        ("prune", ctypes.c_int32),
        ("method", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("subsets_swept", ctypes.c_uint64),
        ("fp64_rechecks", ctypes.c_uint64),
        ("deferred_subsets", ctypes.c_uint64),
        ("exact_predicates", ctypes.c_uint64),
        ("degenerate_subsets", ctypes.c_uint64),
        ("invalid_subsets", ctypes.c_uint64),
        ("device_status", ctypes.c_int32),
        ("prep_ms", ctypes.c_float),
        ("subset_ms", ctypes.c_float),
        ("exact_ms", ctypes.c_float),
        ("finalize_ms", ctypes.c_float),
        ("total_ms", ctypes.c_float),
        ("walked_sweeps", ctypes.c_uint64),
        ("pruned_subsets", ctypes.c_uint64),
        ("exact_subsets", ctypes.c_uint64),
        ("adia_evaluations", ctypes.c_uint64),
        ("adia_candidates", ctypes.c_uint64),
        ("f64_items", ctypes.c_uint64),
        ("adia_rcom_queries", ctypes.c_uint64),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("p", ctypes.c_int32),
        ("Z", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("counts", ctypes.c_void_p),
    ]


# exported symbols of include/td.h
SYMBOLS = ["td_default_options", "td_depth", "td_depth_ex", "td_depth_batched", "td_depth_noalloc",
           "td_get_stats", "td_autotune", "td_tuning_save", "td_tuning_load", "td_status_string", "td_release",
           "td_version"]

_lib = None


class TDError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s: %s (%d)" % (what, STATUS.get(code, "unknown"), code))
        self.code = code


def load():
    """Load libtd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtd.so is not built (%s); run __graft_entry__.build() "
                           "or python -m paper_1409_3901_amd._build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.td_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.td_default_options.restype = ctypes.c_int
    lib.td_depth.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int64, vp, vp]
    lib.td_depth.restype = ctypes.c_int
    lib.td_depth_ex.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int64, vp,
                                ctypes.POINTER(Options), vp]
    lib.td_depth_ex.restype = ctypes.c_int
    lib.td_depth_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int64, vp,
                                     ctypes.POINTER(Options), vp]
    lib.td_depth_noalloc.restype = ctypes.c_int
    lib.td_depth_batched.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Options), vp]
    lib.td_depth_batched.restype = ctypes.c_int
    lib.td_get_stats.argtypes = [ctypes.POINTER(Stats)]
    lib.td_get_stats.restype = ctypes.c_int
    lib.td_autotune.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(Options), vp]
    lib.td_autotune.restype = ctypes.c_int
    lib.td_tuning_save.argtypes = [ctypes.c_char_p]
    lib.td_tuning_save.restype = ctypes.c_int
    lib.td_tuning_load.argtypes = [ctypes.c_char_p]
    lib.td_tuning_load.restype = ctypes.c_int
    lib.td_status_string.argtypes = [ctypes.c_int]
    lib.td_status_string.restype = ctypes.c_char_p
    lib.td_release.argtypes = []
    lib.td_release.restype = None
    lib.td_version.argtypes = []
    lib.td_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def options(precision="filtered", autotune=True, chunk=0, grid_blocks=0, filter_scale=1.0,
            force_exact=False, timing=False, deferred_capacity=0, sweep="auto", prune=True,
            method="rcom") -> Options:
    lib = load()
    o = Options()
    lib.td_default_options(ctypes.byref(o))
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.autotune = 1 if autotune else 0
    o.chunk = int(chunk)
    o.grid_blocks = int(grid_blocks)
    o.filter_scale = float(filter_scale)
    o.force_exact = 1 if force_exact else 0
    o.timing = 1 if timing else 0
    o.deferred_capacity = int(deferred_capacity)
    o.sweep = SWEEP[sweep] if isinstance(sweep, str) else int(sweep)
    o.prune = 1 if prune else 0
    o.method = METHOD[method] if isinstance(method, str) else int(method)
    return o


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _check_tensor(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous 2-D tensor" % name)


def depth(X, Z, stream=None, out=None, **opts):
    """Depth counts n * D_n(Z_q) of the rows of Z w.r.t. the rows of X.

    X: (n, p) float64 CUDA tensor, Z: (m, p) float64 CUDA tensor.
    Returns an int32 CUDA tensor of length m (-1 marks a failed query)."""
    import torch
    lib = load()
    _check_tensor(X, "X")
    _check_tensor(Z, "Z")
    n, p = X.shape
    m, pz = Z.shape
    if pz != p:
        raise ValueError("X and Z have different dimensions")
    if out is None:
        out = torch.empty(m, dtype=torch.int32, device=X.device)
    o = options(**opts)
    rc = lib.td_depth_ex(ctypes.c_void_p(X.data_ptr()), n, p, ctypes.c_void_p(Z.data_ptr()), m,
                         ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream_ptr(stream))
    if rc != TD_OK:
        raise TDError(rc, "td_depth_ex")
    return out


def depth_noalloc(X, Z, out, stream=None, **opts):
    """As ``depth`` through td_depth_noalloc: the library allocates nothing
    (its workspace is a static device array); ``out`` (int32, length m, on
    the device) must be given."""
    lib = load()
    _check_tensor(X, "X")
    _check_tensor(Z, "Z")
    n, p = X.shape
    m, pz = Z.shape
    if pz != p:
        raise ValueError("X and Z have different dimensions")
    o = options(**opts)
    rc = lib.td_depth_noalloc(ctypes.c_void_p(X.data_ptr()), n, p, ctypes.c_void_p(Z.data_ptr()), m,
                              ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream_ptr(stream))
    if rc != TD_OK:
        raise TDError(rc, "td_depth_noalloc")
    return out


def depth_batched(problems, stream=None, **opts):
    """Depth counts for a list of (X, Z) pairs in one graph launch."""
    import torch
    lib = load()
    arr = (Problem * len(problems))()
    outs = []
    for i, (X, Z) in enumerate(problems):
        _check_tensor(X, "X")
        _check_tensor(Z, "Z")
        out = torch.empty(Z.shape[0], dtype=torch.int32, device=X.device)
        outs.append(out)
        arr[i].X = X.data_ptr()
        arr[i].n = X.shape[0]
        arr[i].p = X.shape[1]
        arr[i].Z = Z.data_ptr()
        arr[i].m = Z.shape[0]
        arr[i].counts = out.data_ptr()
    o = options(**opts)
    rc = lib.td_depth_batched(arr, len(problems), ctypes.byref(o), _stream_ptr(stream))
    if rc != TD_OK:
        raise TDError(rc, "td_depth_batched")
    return outs


def get_stats() -> dict:
    """Counters and stage timings of the last call (synchronises)."""
    lib = load()
    s = Stats()
    rc = lib.td_get_stats(ctypes.byref(s))
    if rc not in (TD_OK, 5):
        raise TDError(rc, "td_get_stats")
    d = {k: getattr(s, k) for k, _ in Stats._fields_}
    d["device_status_bits"] = [v for b, v in DEV_BITS.items() if s.device_status & b]
    return d


def autotune(p: int, n: int, stream=None, **opts):
    lib = load()
    o = options(**opts)
    rc = lib.td_autotune(int(p), int(n), ctypes.byref(o), _stream_ptr(stream))
    if rc != TD_OK:
        raise TDError(rc, "td_autotune")


def tuning_save(path: str):
    """Write the current device's tuned launch shapes to a text file."""
    rc = load().td_tuning_save(os.fsencode(path))
    if rc != TD_OK:
        raise TDError(rc, "td_tuning_save")


def tuning_load(path: str):
    """Read launch shapes written by tuning_save into the current device's
    cache (the file must come from a device with the same CU count)."""
    rc = load().td_tuning_load(os.fsencode(path))
    if rc != TD_OK:
        raise TDError(rc, "td_tuning_load")


def release():
    if _lib is not None:
        _lib.td_release()


def subsets(n: int, p: int) -> int:
    """Number of (p-2)-subsets swept for n observations (none for p = 1)."""
    return math.comb(n, p - 2) if p >= 2 else 0
