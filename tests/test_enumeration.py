"""Enumeration pins (the index set of (p-2)-subsets in Section 2, looped over
by Algorithm 1, Step 1): every subset is visited exactly once, by the
oracle's lexicographic enumerator and by the kernels' colex unranking.

* Oracle: the ranks [r0, r1) are visited in chunks (unrank at the chunk
  start, then successor steps); the visited sequence must be the
  lexicographic order of ``itertools.combinations`` for every n <= 30 and
  every chunk size tried, including ranges that start and end inside a
  chunk.  ``depth_range`` over all ranks equals ``depth_counts``, a split
  into ranges gives the same minimum, and the visited count is counted, not
  assumed.
* Kernels: ``tests/colex_check.hip`` runs the device unranking code on the
  host over every rank for n <= 30 and sampled ranks up to n = 1024.
"""
import itertools
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_oracle_lex_enumeration_exhaustive(k):
    for n in range(k, 31 if k <= 3 else 25):
        ref = np.array(list(itertools.combinations(range(n), k)), dtype=np.int32).reshape(math.comb(n, k), k)
        assert len(ref) == oracle.binom(n, k)
        for chunk in (1, 7, 256):
            got = oracle.enumerate_subsets(n, k, chunk=chunk)
            assert np.array_equal(got, ref), (n, k, chunk)


def test_oracle_lex_enumeration_ranges():
    rng = np.random.default_rng(1)
    for n, k in [(30, 3), (30, 4), (20, 6), (12, 6)]:
        ref = np.array(list(itertools.combinations(range(n), k)), dtype=np.int32)
        total = len(ref)
        for _ in range(10):
            r0 = int(rng.integers(0, total))
            r1 = int(rng.integers(r0, total + 1))
            got = oracle.enumerate_subsets(n, k, r0, r1, chunk=int(rng.integers(1, 300)))
            assert np.array_equal(got, ref[r0:r1]), (n, k, r0, r1)


def test_depth_range_full_and_split():
    X, Z = workloads.c1()
    rng = np.random.default_rng(2)
    X4 = rng.standard_normal((25, 4))
    Z4 = np.vstack([0.2 * rng.standard_normal((2, 4)), X4[:1]])
    for X_, Z_ in [(X, Z[:4]), (X4, Z4)]:
        full = oracle.depth_counts(X_, Z_)
        n, p = X_.shape
        for q in range(Z_.shape[0]):
            n0 = int(np.sum(np.all(X_ == Z_[q], axis=1)))
            total = math.comb(n - n0, p - 2)
            v, swept = oracle.depth_range(X_, Z_[q], 0, total)
            assert (v, swept) == (int(full[q]), total)
            # past the end: clipped
            v2, swept2 = oracle.depth_range(X_, Z_[q], 0, total + 1000)
            assert (v2, swept2) == (v, total)
            cuts = sorted(set([0, total] + [int(c) for c in rng.integers(0, total, size=3)]))
            parts = [oracle.depth_range(X_, Z_[q], a, b) for a, b in zip(cuts[:-1], cuts[1:])]
            assert sum(s for _, s in parts) == total
            assert min(v for v, s in parts if v >= 0) == int(full[q])
            # an empty range visits nothing and has no minimum
            assert oracle.depth_range(X_, Z_[q], 5, 5) == (-1, 0)


def test_kernel_colex_unranking(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "colex_check")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", os.path.join(HERE, "colex_check.hip"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok ")
    assert int(r.stdout.split()[1]) > 10**6
