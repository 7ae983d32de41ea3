"""CPU oracle for the exact Tukey depth count (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, loads or calls anything here.

* ``depth_counts`` -- the paper's first algorithm made exact (C++/OpenMP,
  ``td_oracle.cpp``): the arbiter at workload scale.
* ``depth_adia``   -- the paper's adaptive algorithm (Algorithm 3), step by
  step, with exact subset values.
* ``depth_range``  -- the same loop restricted to a range of subset ranks (a
  bounded sample, used to time the oracle).
* ``depth_vertex`` -- the critical-direction route in C++ (tiny inputs).
* ``enumerate_subsets`` -- the subset ranks as the depth loop visits them.
* ``brute``        -- independent pure-Python exact arbiters.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import brute  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

EXACT_ONLY = 1


def build(force: bool = True) -> str:
    """Compile the C++ oracle with g++ (OpenMP)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               os.path.join(_HERE, "td_oracle.cpp"), "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=False)
    lib = ctypes.CDLL(_SO)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_depth.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64,
                                 i64p, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_depth.restype = ctypes.c_int
    lib.oracle_depth_range.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_uint64,
                                       ctypes.c_uint64, i64p, u64p, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_depth_range.restype = ctypes.c_int
    lib.oracle_depth_vertex.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, dp, i64p]
    lib.oracle_depth_vertex.restype = ctypes.c_int
    lib.oracle_binom.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.oracle_binom.restype = ctypes.c_uint64
    lib.oracle_depth_adia.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, i64p, i64p,
                                      ctypes.c_int32, ctypes.c_int32]
    lib.oracle_depth_adia.restype = ctypes.c_int
    lib.oracle_enumerate.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_enumerate.restype = ctypes.c_int64
    _lib = lib
    return lib


def _arr(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def depth_counts(X, Z, threads: int | None = None, exact_only: bool = False) -> np.ndarray:
    """Exact depth counts n*D_n(Z_q) for every query row of Z."""
    lib = _load()
    X, Xp = _arr(X)
    Z, Zp = _arr(np.atleast_2d(Z))
    n, p = X.shape
    m = Z.shape[0]
    out = np.zeros(m, dtype=np.int64)
    rc = lib.oracle_depth(Xp, n, p, Zp, m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          int(threads or default_threads()), EXACT_ONLY if exact_only else 0)
    if rc != 0:
        raise ValueError("oracle_depth failed with code %d" % rc)
    return out


def depth_range(X, z, r0: int, r1: int, threads: int | None = None, exact_only: bool = False):
    """(n0 + min over subsets of lexicographic rank in [r0, r1), number swept)."""
    lib = _load()
    X, Xp = _arr(X)
    z, zp = _arr(np.asarray(z).reshape(-1))
    n, p = X.shape
    out = ctypes.c_int64(0)
    sw = ctypes.c_uint64(0)
    rc = lib.oracle_depth_range(Xp, n, p, zp, int(r0), int(r1), ctypes.byref(out), ctypes.byref(sw),
                                int(threads or default_threads()), EXACT_ONLY if exact_only else 0)
    if rc != 0:
        raise ValueError("oracle_depth_range failed with code %d" % rc)
    return int(out.value), int(sw.value)


def depth_adia(X, Z, threads: int | None = None, exact_only: bool = False):
    """Depth counts by the paper's adaptive algorithm (Algorithm 3) and the
    number of Step 5 candidate points per query (-1: Algorithm 1 was used)."""
    lib = _load()
    X, Xp = _arr(X)
    Z, Zp = _arr(np.atleast_2d(Z))
    n, p = X.shape
    m = Z.shape[0]
    out = np.zeros(m, dtype=np.int64)
    ks = np.zeros(m, dtype=np.int64)
    i64 = ctypes.POINTER(ctypes.c_int64)
    rc = lib.oracle_depth_adia(Xp, n, p, Zp, m, out.ctypes.data_as(i64), ks.ctypes.data_as(i64),
                               int(threads or default_threads()), EXACT_ONLY if exact_only else 0)
    if rc != 0:
        raise ValueError("oracle_depth_adia failed with code %d" % rc)
    return out, ks


def depth_vertex(X, z) -> int:
    lib = _load()
    X, Xp = _arr(X)
    z, zp = _arr(np.asarray(z).reshape(-1))
    n, p = X.shape
    out = ctypes.c_int64(0)
    rc = lib.oracle_depth_vertex(Xp, n, p, zp, ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_depth_vertex failed with code %d" % rc)
    return int(out.value)


def binom(n: int, k: int) -> int:
    return int(_load().oracle_binom(n, k))


def enumerate_subsets(n: int, k: int, r0: int = 0, r1: int | None = None, chunk: int = 256) -> np.ndarray:
    """The k-subsets of lexicographic rank [r0, r1) as the depth loop visits
    them (rows of k indices, rank order)."""
    lib = _load()
    total = binom(n, k)
    r1 = total if r1 is None else min(int(r1), total)
    cnt = max(0, r1 - int(r0))
    out = np.zeros((cnt, max(k, 1)), dtype=np.int32)
    got = lib.oracle_enumerate(int(n), int(k), int(r0), int(r1), int(chunk),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if got != cnt:
        raise ValueError("oracle_enumerate returned %d, expected %d" % (got, cnt))
    return out[:, :k]
