"""Failure reporting and the negative control.

Every data-dependent failure must come back as counts[q] = -1 with its bit in
td_stats.device_status, never as a wrong count, and every kernel must still
exit normally: the conditions are produced from the host (inputs, options),
not by faulting anything.  The negative control (filter_scale = 0: float32
decisions trusted without their error bound) must show that the parity
checks can fail: on exactly degenerate data it has to give wrong counts.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), **kw)
    return c.cpu().numpy().astype(np.int64), td.get_stats()


def test_nonfinite_query(td, dev):
    """NaN / Inf in a query: that query fails, the others are exact."""
    rng = np.random.default_rng(50)
    X = rng.standard_normal((40, 4))
    Z = rng.standard_normal((4, 4))
    Z[1, 2] = np.nan
    Z[3, 0] = np.inf
    got, st = run(td, dev, X, Z)
    assert got[1] == -1 and got[3] == -1
    assert "nonfinite" in st["device_status_bits"]
    ok = [0, 2]
    assert np.array_equal(got[ok], oracle.depth_counts(X, Z[ok]))


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_sample(td, dev, bad):
    """NaN / Inf in X: every query of that sample fails."""
    rng = np.random.default_rng(51)
    X = rng.standard_normal((30, 3))
    X[7, 1] = bad
    Z = rng.standard_normal((3, 3))
    got, st = run(td, dev, X, Z)
    assert np.all(got == -1)
    assert "nonfinite" in st["device_status_bits"]


def test_nonfinite_in_batch_leaves_other_problems_exact(td, dev):
    rng = np.random.default_rng(52)
    X1 = rng.standard_normal((30, 3))
    Z1 = rng.standard_normal((2, 3))
    X2 = rng.standard_normal((25, 4))
    X2[0, 0] = np.nan
    Z2 = rng.standard_normal((2, 4))
    outs = td.depth_batched([(to_dev(X1, dev), to_dev(Z1, dev)), (to_dev(X2, dev), to_dev(Z2, dev))])
    assert np.array_equal(outs[0].cpu().numpy(), oracle.depth_counts(X1, Z1))
    assert np.all(outs[1].cpu().numpy() == -1)


def test_defer_overflow(td, dev):
    """Every subset sent to the exact tier with room for one deferred entry:
    the queries whose entries did not fit fail."""
    rng = np.random.default_rng(53)
    X = rng.standard_normal((30, 4))
    Z = rng.standard_normal((2, 4))
    got, st = run(td, dev, X, Z, force_exact=True, deferred_capacity=1, prune=False)
    assert np.all(got == -1), got
    assert "defer_overflow" in st["device_status_bits"]
    assert st["deferred_subsets"] > 1
    # the same call with room for every subset is exact
    got, st = run(td, dev, X, Z, force_exact=True, prune=False)
    assert np.array_equal(got, oracle.depth_counts(X, Z))
    assert st["device_status"] == 0


@pytest.mark.parametrize("online", [20, 24])
def test_degeneracy_limit(td, dev, online):
    """p = 3 with `online` points on one line through the query: a subset
    on that line has all of them inside its span, more than the exact tier's
    hitting-set search takes.  The answer is the exact count or -1 with the
    degeneracy bit, never another value."""
    rng = np.random.default_rng(54 + online)
    v = np.array([1.0, 2.0, -1.0])
    t = np.concatenate([np.arange(1, online // 2 + 1), -np.arange(1, online - online // 2 + 1)]).astype(float)
    line = t[:, None] * v[None, :]
    gen = rng.integers(-4, 5, size=(5, 3)).astype(float)
    X = np.vstack([line, gen])
    Z = np.zeros((1, 3))
    exp = oracle.depth_counts(X, Z)
    for prune in (True, False):
        got, st = run(td, dev, X, Z, prune=prune)
        if got[0] == -1:
            assert "degeneracy_limit" in st["device_status_bits"], st
        else:
            assert got[0] == exp[0], (got, exp)
            assert st["device_status"] == 0


def test_exact_range(td, dev):
    """The exact integer copy of the centred data needs more than 125 bits:
    points duplicated along their rays from the origin, and a query at
    (2^-140, 0, 0).  Centred in float64 the pairs stay exactly on one ray;
    exactly, they do not.  float64 cannot decide them, so the call fails with
    the exact-range bit, never with a wrong count."""
    rng = np.random.default_rng(56)
    flagged = 0
    for t in range(6):
        X, Z0 = workloads.ray_duplicated(rng, 3, 12)
        X = X - Z0                      # integers: exact
        Z = np.zeros_like(Z0)
        Z[0, 0] = 2.0 ** -140
        exp = oracle.depth_counts(X, Z)
        got, st = run(td, dev, X, Z, prune=False)
        if got[0] == -1:
            assert "exact_range" in st["device_status_bits"], st
            flagged += 1
        else:
            assert got[0] == exp[0], (t, got, exp)
    assert flagged > 0


def _c5_golden():
    counts = {}
    for name in sorted(os.listdir(GOLD)):
        if name.startswith("c5") and name.endswith(".json"):
            with open(os.path.join(GOLD, name)) as f:
                counts.update({int(k): v for k, v in json.load(f)["counts"].items()})
    return counts


def test_stress_lattice_certified_and_uncertified(td, dev):
    """The mapped lattice stress workload with the filter certified (exact
    counts required) and with filter_scale = 0, the float32 keys taken
    without any margin (recorded).  The uncertified counts come out exact
    here as well: the float64 re-order of overlapping mixed clusters and the
    exact tier still run, and points swept that should have been left out
    (members of I, points inside span(x_I)) only raise a subset's count, so
    the minimum over subsets survives whenever some minimising subset is
    unaffected.  The control that must fail is the ray-duplicated family
    below.  Pruning is off, so the bound from the directions +-x_j (which
    does not depend on the filter) cannot hide wrong sweeps."""
    X, Z = workloads.c5()
    g = _c5_golden()
    qs = sorted(g)
    exp = np.array([g[q] for q in qs])
    for sweep in ("auto", "bitonic"):
        good, st = run(td, dev, X, Z[qs], sweep=sweep, prune=False)
        assert np.array_equal(good, exp), (sweep, good, exp)
        if sweep == "auto":
            # the map's condition number leaves float32 uncertified often:
            # the bucketed kernel hands most work items to its float64 pass
            assert st["f64_items"] > 0 and st["fp64_rechecks"] > 0, st
        bad, _ = run(td, dev, X, Z[qs], sweep=sweep, prune=False, filter_scale=0.0)
        print(sweep, "stress lattice, filter_scale=0:", bad.tolist(), "expected", exp.tolist(),
              "mismatches", int(np.sum(bad != exp)))


@pytest.mark.parametrize("prune", [True, False])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_negative_control_ray_duplicated(td, dev, sweep, prune):
    """Points duplicated along their rays from the query: every subset holding
    one copy has the other inside its span.  Certified, the counts are exact;
    with filter_scale = 0 the copies are swept like ordinary points and some
    counts must come out wrong (the parity checks can fail)."""
    rng = np.random.default_rng(57)
    wrong = 0
    for t in range(20):
        X, Z = workloads.ray_duplicated(rng, 4, int(rng.integers(4, 8)))
        exp = oracle.depth_counts(X, Z)
        got, _ = run(td, dev, X, Z, sweep=sweep, prune=prune)
        assert got[0] == exp[0]
        bad, _ = run(td, dev, X, Z, sweep=sweep, prune=prune, filter_scale=0.0)
        wrong += int(bad[0] != exp[0])
    print("uncertified mismatches:", wrong, "of 20")
    assert wrong >= 1


def test_float64_pass_accounts_every_subset_once(td, dev):
    """The mapped lattice sends most work items of the bucketed kernel to its
    float64 pass (the first pass hands over the marked subsets of a batch and
    the rest of the item, which the pass cuts into units shared by all
    waves).  Without pruning, every subset is still swept or deferred exactly
    once: the two counters add up to sum_q C(n'_q, p-2) (the invalid subsets
    of the filtered tier are deferred ones the exact tier found dependent)."""
    X, Z = workloads.c5()
    g = _c5_golden()
    qs = sorted(g)[:6]
    got, st = run(td, dev, X, Z[qs], prune=False)
    assert np.array_equal(got, [g[q] for q in qs]), got
    assert st["f64_items"] > 100, st
    total = sum(math.comb(int(np.sum(~np.all(X == Z[q], axis=1))), X.shape[1] - 2) for q in qs)
    assert st["subsets_swept"] + st["deferred_subsets"] == total, (st, total)
    assert st["invalid_subsets"] <= st["deferred_subsets"]
    # with pruning, the subsets skipped once a minimum reached 0 (counted in
    # both passes) complete the account
    got, st = run(td, dev, X, Z[qs])
    assert np.array_equal(got, [g[q] for q in qs]), got
    acc = st["subsets_swept"] + st["pruned_subsets"] + st["deferred_subsets"]
    assert acc == total, (st, total)
