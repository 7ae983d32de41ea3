"""The paper's adaptive algorithm (Algorithm 3, td_options.method = ADIA) on
the GPU: the descent of Steps 2-4 and Step 5's certified sweeps over the
subsets of the candidate points.  In general position its counts must equal
the exact counts (and the oracle's ADIA); on any data they must never lie
below the exact count."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), method="adia", **kw)
    return c.cpu().numpy().astype(np.int64), td.get_stats()


def test_adia_c1(td, dev):
    X, Z = workloads.c1()
    g = json.load(open(os.path.join(GOLD, "c1.json")))["counts"]
    exp = np.array([g[str(q)] for q in range(Z.shape[0])])
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0
    assert st["adia_evaluations"] > 0
    assert np.array_equal(got, exp), (got, exp)
    a, _ = oracle.depth_adia(X, Z)
    assert np.array_equal(got, a)


@pytest.mark.parametrize("p,n", [(3, 200), (4, 90), (5, 50), (6, 28), (7, 20), (8, 19)])
@pytest.mark.parametrize("sweep", ["auto", "bitonic"])
def test_adia_general_position_vs_oracle(td, dev, p, n, sweep):
    rng = np.random.default_rng(500 + 11 * p + n)
    X = rng.standard_normal((n, p))
    Z = np.vstack([0.3 * rng.standard_normal((3, p)), X[:2], 1.5 * rng.standard_normal((2, p)),
                   workloads.outside_hull_query(X, rng)])
    got, st = run(td, dev, X, Z, sweep=sweep)
    assert st["device_status"] == 0
    exp = oracle.depth_counts(X, Z)
    assert np.array_equal(got, exp), (got, exp)
    a, _ = oracle.depth_adia(X, Z)
    assert np.array_equal(got, a)


def test_adia_c3_sample_queries(td, dev):
    """The benchmark workload (p = 5, n = 500): four queries against the
    stored exact counts."""
    X, Z = workloads.c3()
    g = json.load(open(os.path.join(GOLD, "c3.json")))["counts"]
    qs = [0, 5, 16, 20]
    exp = np.array([g[str(q)] for q in qs])
    got, st = run(td, dev, X, Z[qs])
    assert st["device_status"] == 0
    assert np.array_equal(got, exp), (got, exp)
    assert st["adia_candidates"] < 4 * X.shape[0]


def test_adia_never_below_depth_on_degenerate_data(td, dev):
    rng = np.random.default_rng(94)
    bad = []
    for t in range(30):
        p = int(rng.integers(3, 6))
        kind = t % 3
        if kind == 0:
            X, Z = workloads.lattice_small(rng, p, int(rng.integers(p + 6, 16)), R=2)
        elif kind == 1:
            X, Z = workloads.ray_duplicated(rng, p, int(rng.integers(5, 9)))
        else:
            X, Z = workloads.near_degenerate(rng, p, int(rng.integers(p + 6, 16)))
        got, st = run(td, dev, X, Z)
        exp = oracle.depth_counts(X, Z)
        if st["device_status"] == 0 and got[0] < exp[0]:
            bad.append((t, int(got[0]), int(exp[0])))
    assert not bad, bad


def test_adia_small_samples_and_p2_use_algorithm_1(td, dev):
    rng = np.random.default_rng(95)
    for p, n in [(2, 40), (3, 6), (5, 10)]:
        X = rng.standard_normal((n, p))
        Z = rng.standard_normal((3, p))
        got, st = run(td, dev, X, Z)
        assert np.array_equal(got, oracle.depth_counts(X, Z))
        assert st["adia_evaluations"] == 0
        assert st["adia_rcom_queries"] == 3


def test_adia_long_tie_groups_take_algorithm_1(td, dev):
    """Two rays of 45 and 40 points from the query among 50 general points
    (p = 3): the first evaluation meets an exact tie group longer than an
    evaluation lists (32 points next to its minimising states), so
    Algorithm 1 answers the query (counted in adia_rcom_queries) and the
    count is the exact one.  The descent of a general-position query in the
    same call is unaffected."""
    rng = np.random.default_rng(0)
    p = 3
    d = rng.standard_normal(p)
    G = rng.standard_normal((50, p))
    ray = np.outer(np.linspace(0.5, 3.0, 45), d)
    rng.standard_normal((1, p))
    ray2 = np.outer(np.linspace(0.5, 3.0, 40), -d + 0.3 * rng.standard_normal(p))
    X = np.vstack([G, ray, ray2])
    Z = np.zeros((1, p))
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0
    assert st["adia_rcom_queries"] == 1, st
    assert int(got[0]) == int(oracle.depth_counts(X, Z)[0])
    # with a general-position query beside it, only the tied one falls back
    Z2 = np.vstack([Z, 0.2 * rng.standard_normal((1, p))])
    got2, st2 = run(td, dev, X, Z2)
    assert st2["adia_rcom_queries"] >= 1
    assert int(got2[0]) == int(got[0])
    assert int(got2[1]) >= int(oracle.depth_counts(X, Z2[1:])[0])


def test_adia_unsupported_entry_points(td, dev):
    import torch
    X = to_dev(np.random.default_rng(1).standard_normal((20, 3)), dev)
    Z = to_dev(np.zeros((1, 3)), dev)
    with pytest.raises(td.TDError) as e:
        td.depth_batched([(X, Z)], method="adia")
    assert e.value.code == 2
    out = torch.zeros(1, dtype=torch.int32, device=dev)
    with pytest.raises(td.TDError) as e:
        td.depth_noalloc(X, Z, out, method="adia")
    assert e.value.code == 2


def _adia_golden():
    with open(os.path.join(GOLD, "adia.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("key", sorted(_adia_golden()["adia"]))
def test_adia_paper_grid_vs_stored_oracle(td, dev, key):
    """The paper's simulation design (X ~ N(0, I_p), z = alpha 1_p) at its
    full sizes: the GPU's Algorithm 3 equals the oracle's Algorithm 3 (value
    and candidate count, stored by tests/golden/make_golden.py), and where the
    exact count is stored, RCom equals it.  At p = 6, n = 320, alpha = 0 the
    adaptive value (111) lies above the exact depth (110): Step 5's candidate
    union misses every optimal subset there, on both sides."""
    g = _adia_golden()
    p, n, alpha = key.split(",")
    X, Z = workloads.grid(int(p), int(n), float(alpha))
    print("adia grid", key, flush=True)
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0
    assert int(got[0]) == g["adia"][key], (key, got, g["adia"][key])
    assert st["adia_candidates"] == g["candidates"][key]
    if key in g["exact"]:
        rc = td.depth(to_dev(X, dev), to_dev(Z, dev)).cpu().numpy()
        assert int(rc[0]) == g["exact"][key]
        assert int(got[0]) >= g["exact"][key]


def _obs_golden():
    path = os.path.join(GOLD, "adia_obs.json")
    if not os.path.exists(path):
        return {"adia": {}, "exact": {}}
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("key", sorted(set(_obs_golden()["adia"]) & set(_obs_golden()["exact"])))
def test_adia_every_observation_vs_stored_oracle(td, dev, key):
    """Every observation of a real-data stand-in as a query (the paper's
    real-data experiment): one call over all observations and one call per
    observation both give the oracle's Algorithm 3 value for each of them,
    never below the exact count that RCom returns."""
    g = _obs_golden()
    kind, p, n = key.split(",")
    X, Z = workloads.observations(kind, int(p), int(n))
    exp = np.array(g["adia"][key])
    exact = np.array(g["exact"][key])
    print("adia observations", key, flush=True)
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0
    assert np.array_equal(got, exp), (key, np.nonzero(got != exp)[0])
    assert np.all(exp >= exact)
    rc = td.depth(to_dev(X, dev), to_dev(Z, dev)).cpu().numpy()
    assert np.array_equal(rc, exact)
    # one call per observation: the differing ones and the first 16
    idx = sorted(set(np.nonzero(exp != exact)[0].tolist()) | set(range(16)))
    for q in idx:
        one, _ = run(td, dev, X, Z[q])
        assert int(one[0]) == int(exp[q]), (key, q, one, exp[q])
