"""Pruning (td_options.prune) leaves every count unchanged.

With pruning the library bounds the minimum before the subsets by the closed
halfspace counts of the directions +-(X_j - z) (Algorithm 3, Step 2(a)), lets
the bucketed sweep skip subsets that cannot go below that bound, and skips
the remaining subsets of a query once a term of 0 is reached.  These tests
compare pruned and unpruned runs with each other and with the oracle, on
cases where the bound is loose, where it equals the depth, and where it is 0.
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), **kw)
    out = c.cpu().numpy().astype(np.int64)
    return out, td.get_stats()


@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_c1_pruned_equals_unpruned_and_oracle(td, dev, sweep):
    X, Z = workloads.c1()
    a, _ = run(td, dev, X, Z, sweep=sweep, prune=True)
    b, sb = run(td, dev, X, Z, sweep=sweep, prune=False)
    exp = oracle.depth_counts(X, Z)
    assert np.array_equal(a, exp), (a, exp)
    assert np.array_equal(b, exp), (b, exp)
    assert sb["pruned_subsets"] == 0


@pytest.mark.parametrize("p,n", [(3, 300), (4, 1000), (5, 300)])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_outside_hull_is_pruned(td, dev, p, n, sweep):
    """Queries outside the hull have depth 0: once a subset reports 0 the rest
    of the query's subsets are skipped, and the count stays 0."""
    rng = np.random.default_rng(100 + p)
    X = rng.standard_normal((n, p))
    Z = np.vstack([workloads.outside_hull_query(X, rng) for _ in range(4)])
    a, sa = run(td, dev, X, Z, sweep=sweep, prune=True)
    b, sb = run(td, dev, X, Z, sweep=sweep, prune=False)
    assert np.all(a == 0) and np.all(b == 0), (a, b)
    assert sb["pruned_subsets"] == 0
    total = 4 * workloads_subsets(n, p)
    assert sa["subsets_swept"] + sa["pruned_subsets"] + sa["deferred_subsets"] <= total
    # at p = 3 a query has only n subsets, a batch or two that all start
    # before any term is known; the larger cases have many batches per query
    if p >= 4:
        assert sa["pruned_subsets"] > 0


def workloads_subsets(n, p):
    import math
    return math.comb(n, p - 2)


@pytest.mark.parametrize("p", [3, 4, 5])
@pytest.mark.parametrize("with_center", [False, True])
def test_symmetric_bound_attained(td, dev, p, with_center):
    """For {z +- v_k} every direction +-v_j has the closed count k (+1 with z
    in the sample) or more, and the depth is exactly that: the bound from the
    directions can equal the minimum, which must then still be returned."""
    rng = np.random.default_rng(7 * p + with_center)
    k = 60
    X, Z = workloads.symmetric(rng, p, k, with_center=with_center)
    a, _ = run(td, dev, X, Z, prune=True)
    b, _ = run(td, dev, X, Z, prune=False)
    exp = k + (1 if with_center else 0)
    assert a[0] == exp and b[0] == exp, (a, b, exp)


@pytest.mark.parametrize("p", [3, 4, 5])
def test_degenerate_lattice_pruned_vs_oracle(td, dev, p):
    """Lattices with exact ties, points inside span(x_I) and queries on sample
    points, pruned and unpruned, against the oracle."""
    rng = np.random.default_rng(300 + p)
    for _ in range(3):
        X, Z = workloads.lattice_small(rng, p, 12, R=2)
        exp = oracle.depth_counts(X, Z)
        a, _ = run(td, dev, X, Z, prune=True)
        b, _ = run(td, dev, X, Z, prune=False)
        assert np.array_equal(a, exp), (p, a, exp)
        assert np.array_equal(b, exp), (p, b, exp)


def test_c5_low_depth_queries_pruned(td, dev):
    """The stress lattice: its uniform lattice queries have depth 0 or close to
    it.  Pruned and unpruned counts agree on every query."""
    X, Z = workloads.c5()
    a, sa = run(td, dev, X, Z, prune=True)
    b, sb = run(td, dev, X, Z, prune=False)
    assert np.array_equal(a, b), (a, b)
    assert sb["pruned_subsets"] == 0
    if np.any(a == 0):
        assert sa["pruned_subsets"] > 0


def test_batched_pruned_equals_unpruned(td, dev):
    rng = np.random.default_rng(11)
    probs = []
    for p in (3, 4, 5):
        X = rng.standard_normal((150, p))
        Z = np.vstack([rng.standard_normal((3, p)), workloads.outside_hull_query(X, rng)])
        probs.append((to_dev(X, dev), to_dev(Z, dev)))
    a = [c.cpu().numpy() for c in td.depth_batched(probs, prune=True)]
    b = [c.cpu().numpy() for c in td.depth_batched(probs, prune=False)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y), (x, y)
        assert x[-1] == 0


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
@pytest.mark.parametrize("prec", ["filtered", "bitonic", "plain"])
def test_every_subset_accounted_unpruned(td, dev, cfg, prec):
    """With pruning off, the subset kernels visit every (p-2)-subset of every
    query once: swept + deferred (+ invalid in the plain tier, which finds
    dependent subsets itself; in the filtered tiers they are among the
    deferred) = sum over queries of C(n', p-2), n' the observations
    different from the query (equality, the index set of Section 2)."""
    from conftest import PREC_OPTS
    X, Z = workloads.config(cfg)
    n, p = X.shape
    total = 0
    for q in range(Z.shape[0]):
        n0 = int(np.sum(np.all(X == Z[q], axis=1)))
        total += workloads_subsets(n - n0, p)
    _, st = run(td, dev, X, Z, prune=False, **PREC_OPTS[prec])
    assert st["pruned_subsets"] == 0
    assert st["device_status"] == 0
    got = st["subsets_swept"] + st["deferred_subsets"] + (st["invalid_subsets"] if prec == "plain" else 0)
    assert got == total, (got, total, st)
