"""Exactness on degenerate inputs: the filtered path (with its float64 and
exact tiers) must equal the oracle on data that is far from general position.

Both filtered sweeps are covered: the bucketed sweep (default) and the full
bitonic sort.

Families: small integer lattices (exact angle ties, points inside span(x_I),
linearly dependent subsets, queries on sample points), points duplicated along
their own rays, data of deficient rank, and lattices with 1e-12 jitter (near
ties that float arithmetic cannot order).  The plain float64 kernel carries
no such guarantee and is not checked here.
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), **kw)
    return c.cpu().numpy().astype(np.int64)


def _check(td, dev, X, Z, **kw):
    exp = oracle.depth_counts(X, Z)
    got = run(td, dev, X, Z, **kw)
    return got, exp


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_lattice_small(td, dev, p, sweep):
    rng = np.random.default_rng(100 + p)
    bad = []
    for t in range(40):
        n = int(rng.integers(p + 1, 13))
        X, Z = workloads.lattice_small(rng, p, n, R=2)
        got, exp = _check(td, dev, X, Z, sweep=sweep)
        if got[0] != exp[0]:
            bad.append((t, n, int(got[0]), int(exp[0])))
    assert not bad, bad


@pytest.mark.parametrize("p", [3, 4, 5])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_ray_duplicated(td, dev, p, sweep):
    rng = np.random.default_rng(200 + p)
    bad = []
    for t in range(20):
        X, Z = workloads.ray_duplicated(rng, p, int(rng.integers(3, 7)))
        got, exp = _check(td, dev, X, Z, sweep=sweep)
        if got[0] != exp[0]:
            bad.append((t, int(got[0]), int(exp[0])))
    assert not bad, bad


@pytest.mark.parametrize("p,rank", [(3, 2), (4, 3), (4, 2), (5, 4), (5, 3)])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_rank_deficient(td, dev, p, rank, sweep):
    rng = np.random.default_rng(300 + 10 * p + rank)
    bad = []
    for t in range(15):
        X, Z = workloads.rank_deficient(rng, p, int(rng.integers(p + 1, 12)), rank)
        got, exp = _check(td, dev, X, Z, sweep=sweep)
        if got[0] != exp[0]:
            bad.append((t, int(got[0]), int(exp[0])))
    assert not bad, bad


@pytest.mark.parametrize("p", [3, 4, 5])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_near_degenerate(td, dev, p, sweep):
    rng = np.random.default_rng(400 + p)
    bad = []
    for t in range(20):
        X, Z = workloads.near_degenerate(rng, p, int(rng.integers(p + 2, 14)))
        got, exp = _check(td, dev, X, Z, sweep=sweep)
        if got[0] != exp[0]:
            bad.append((t, int(got[0]), int(exp[0])))
    assert not bad, bad


@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_lattice_medium_many_queries(td, dev, sweep):
    """A 3-D lattice cloud with every sample point as a query: long tie runs
    and many points inside span(x_I) at once."""
    rng = np.random.default_rng(7)
    X = rng.integers(-3, 4, size=(60, 3)).astype(np.float64)
    Z = X[:20].copy()
    got, exp = _check(td, dev, X, Z, sweep=sweep)
    assert np.array_equal(got, exp), (got, exp)


@pytest.mark.parametrize("mode", ["fp64_everywhere", "exact_everywhere"])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_forced_fallback(td, dev, mode, sweep):
    """Every float32 decision re-checked (filter_scale = inf) or every subset
    through the exact tier: the counts must not change."""
    rng = np.random.default_rng(13)
    kw = {"filter_scale": float("inf")} if mode == "fp64_everywhere" else {"force_exact": True}
    for p, n in [(3, 40), (4, 30), (5, 20)]:
        X = rng.standard_normal((n, p))
        Z = np.vstack([rng.standard_normal((2, p)), X[:1]])
        got, exp = _check(td, dev, X, Z, sweep=sweep, **kw)
        assert np.array_equal(got, exp), (p, n, got, exp)
    for p in (3, 4):
        X, Z = workloads.lattice_small(rng, p, 10, R=2)
        got, exp = _check(td, dev, X, Z, sweep=sweep, **kw)
        assert np.array_equal(got, exp), (p, got, exp)


@pytest.mark.parametrize("scale", [16.0, 512.0, 8192.0])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_widened_float32_radii(td, dev, scale, sweep):
    """float32 key intervals widened by `scale` next to float64 re-checks of
    the points that then fail the float32 check: clusters of intervals whose
    widths differ by orders of magnitude, the case in which the grouping
    must order intervals by their lower ends.  Counts must not change."""
    rng = np.random.default_rng(int(scale) + 5)
    cases = [workloads.c1()]
    for p, n in [(3, 60), (4, 45), (5, 25)]:
        X = rng.standard_normal((n, p))
        cases.append((X, np.vstack([0.3 * rng.standard_normal((2, p)), X[:1]])))
    for p in (3, 4, 5):
        cases.append(workloads.near_degenerate(rng, p, 12))
        cases.append(workloads.lattice_small(rng, p, 11, R=2))
    bad = []
    for t, (X, Z) in enumerate(cases):
        got, exp = _check(td, dev, X, Z, sweep=sweep, filter_scale=scale)
        if not np.array_equal(got, exp):
            bad.append((t, X.shape, got.tolist(), exp.tolist()))
    assert not bad, bad


def test_rank_too_low_is_flagged(td, dev):
    """Centred data spanning at most p-3 dimensions is outside what the GPU
    path handles: the query reports -1 and a status bit, never a wrong count."""
    rng = np.random.default_rng(17)
    X, Z = workloads.rank_deficient(rng, 5, 9, 1)
    got = run(td, dev, X, Z)
    st = td.get_stats()
    exp = oracle.depth_counts(X, Z)
    assert got[0] == -1 or got[0] == exp[0]
    if got[0] == -1:
        assert "no_valid_subset" in st["device_status_bits"]
