"""The depth of every observation of a sample (the queries are the sample
itself, so every query has n0 >= 1): the workload of the paper's real-data
experiments (Section 5.1, p in {3, 4}, n in {64, 200, 500}), on seeded
stand-ins of the same shapes, through the single call and the batched call."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import PREC_OPTS, to_dev

pytestmark = pytest.mark.gpu

# (kind, p, n) of the paper's table of per-observation timings
FULL = [("scores", 3, 64), ("scores", 4, 64), ("returns", 3, 200), ("returns", 4, 200),
        ("returns", 3, 500)]
LARGEST = ("returns", 4, 500)


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(Z, dev), **kw)
    return c.cpu().numpy().astype(np.int64)


def duplicates(X):
    """n0 of each observation: how many rows equal it."""
    return np.array([int(np.sum(np.all(X == x, axis=1))) for x in X])


def check_bounds(X, got):
    """Properties at any size: an observation lies in the sample, so its
    count is at least its multiplicity n0; and a generic hyperplane through
    it splits the other n - n0 points, so one closed side holds at most
    n0 + (n - n0) / 2 of them."""
    n0 = duplicates(X)
    n = X.shape[0]
    assert np.all(got >= n0)
    assert np.all(2 * got <= n + n0)


@pytest.mark.parametrize("prec", ["filtered", "bitonic"])
@pytest.mark.parametrize("kind,p,n", FULL)
def test_every_observation(td, dev, prec, kind, p, n):
    X, Z = workloads.observations(kind, p, n)
    got = run(td, dev, X, Z, **PREC_OPTS[prec])
    assert td.get_stats()["device_status"] == 0
    exp = oracle.depth_counts(X, Z)
    assert np.array_equal(got, exp), (int(np.sum(got != exp)),)
    check_bounds(X, got)


def test_every_observation_largest(td, dev):
    """p = 4, n = 500: all 500 observations on the GPU, the oracle on a
    seeded sample of them, the bounds on all, and the bitonic sweep equal to
    the bucketed one everywhere."""
    kind, p, n = LARGEST
    X, Z = workloads.observations(kind, p, n)
    got = run(td, dev, X, Z)
    assert td.get_stats()["device_status"] == 0
    check_bounds(X, got)
    idx = np.sort(np.random.default_rng(11).choice(n, 8, replace=False))
    exp = oracle.depth_counts(X, Z[idx])
    assert np.array_equal(got[idx], exp), (got[idx], exp)
    other = run(td, dev, X, Z, **PREC_OPTS["bitonic"])
    assert np.array_equal(got, other), (int(np.sum(got != other)),)


def test_every_observation_batched(td, dev):
    """All six samples in one batched call (one graph launch) give the
    single call's counts."""
    cases = FULL + [LARGEST]
    data = [workloads.observations(k, p, n) for k, p, n in cases]
    probs = [(to_dev(X, dev), to_dev(Z, dev)) for X, Z in data]
    outs = td.depth_batched(probs)
    for (X, Z), o, case in zip(data, outs, cases):
        single = run(td, dev, X, Z)
        got = o.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, single), (case, int(np.sum(got != single)))
        check_bounds(X, got)
