"""p = 2: Algorithm 2 on its own (the index set of (p-2)-subsets holds only
the empty set), one sweep of every query's n' points.  The p2 workload puts
1023 points in the sweep of a sample-point query and 1024 in the others;
the filtered tier sorts every p = 2 sweep in full, and no p = 2 sweep may go
to the exact tier."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from conftest import PREC_OPTS, to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("prec", ["filtered", "bitonic", "plain"])
def test_p2_workload_vs_stored_oracle(td, dev, prec):
    with open(os.path.join(GOLD, "p2.json")) as f:
        g = json.load(f)["counts"]
    X, Z = workloads.p2()
    exp = np.array([g[str(q)] for q in range(Z.shape[0])])
    got = td.depth(to_dev(X, dev), to_dev(Z, dev), **PREC_OPTS[prec]).cpu().numpy()
    st = td.get_stats()
    assert st["device_status"] == 0
    if prec != "plain":
        assert st["deferred_subsets"] == 0, st
        # every p = 2 sweep takes the full sort: none is walked
        assert st["walked_sweeps"] == 0, st
        assert st["subsets_swept"] == Z.shape[0], st
    assert np.array_equal(got, exp), int(np.sum(got != exp))


@pytest.mark.parametrize("n", [1023, 1024])
def test_p2_full_sweep_degenerate(td, dev, n):
    """Exact ties at the full sweep width: integer points of [-200, 200]^2
    (several on some lines through the query) with eight points doubled
    along their rays from the origin, queried at the origin, off the
    lattice, and at a sample point.  (A lattice as small as [-6, 6]^2 puts
    hundreds of points on one line through the query, beyond the exact
    tier's runs, which is reported as degeneracy_limit.)"""
    rng = np.random.default_rng(n)
    X = rng.integers(-200, 201, size=(n, 2)).astype(np.float64)
    X[n - 8:] = 2.0 * X[:8]
    Z = np.vstack([[0.0, 0.0], [0.5, 0.25], X[3]])
    exp = oracle.depth_counts(X, Z)
    got = td.depth(to_dev(X, dev), to_dev(Z, dev)).cpu().numpy()
    assert td.get_stats()["device_status"] == 0
    assert np.array_equal(got, exp), (got, exp)
