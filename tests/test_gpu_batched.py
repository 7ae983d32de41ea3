"""Batched persistent launches (one captured HIP graph per class set) and the
autotuner: counts must equal the per-query path and the oracle, for every
launch shape, and stay equal over graph replays."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from conftest import PREC_OPTS, to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _small_batch(seed, num=24):
    rng = np.random.default_rng(seed)
    probs = []
    for d in range(num):
        p = int(rng.integers(2, 7))
        n = int(rng.integers(max(p + 1, 8), 70 if p < 6 else 30))
        if d % 3 == 0:
            X, Z = workloads.lattice_small(rng, p, min(n, 12), R=2)
            Z = np.vstack([Z, X[:1]])
        else:
            X = rng.standard_normal((n, p))
            Z = np.vstack([rng.standard_normal((3, p)), X[:1]])
        probs.append((X, Z))
    return probs


def test_batched_small_uneven_vs_oracle(td, dev):
    probs = _small_batch(21)
    outs = td.depth_batched([(to_dev(X, dev), to_dev(Z, dev)) for X, Z in probs])
    for (X, Z), o in zip(probs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.depth_counts(X, Z)), (X.shape,)


def test_batched_graph_replay_and_equal_to_single(td, dev):
    """Same class set three times (the graph is captured once and replayed
    with new data); every replay equals the per-query path."""
    for seed in (31, 32, 33):
        rng = np.random.default_rng(seed)
        probs = []
        for p, n in [(3, 90), (4, 70), (5, 40), (3, 200), (4, 130)]:
            X = rng.standard_normal((n, p))
            probs.append((X, np.vstack([rng.standard_normal((2, p)), X[:1]])))
        dprobs = [(to_dev(X, dev), to_dev(Z, dev)) for X, Z in probs]
        outs = td.depth_batched(dprobs)
        for (Xd, Zd), o in zip(dprobs, outs):
            single = td.depth(Xd, Zd)
            assert np.array_equal(o.cpu().numpy(), single.cpu().numpy())


@pytest.mark.parametrize("prec", ["plain", "filtered", "bitonic"])
def test_batched_precisions(td, dev, prec):
    probs = _small_batch(41, num=10)
    probs = [(X, Z) for X, Z in probs if X.shape[0] > 12]   # general position only
    outs = td.depth_batched([(to_dev(X, dev), to_dev(Z, dev)) for X, Z in probs], **PREC_OPTS[prec])
    for (X, Z), o in zip(probs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.depth_counts(X, Z))


def test_launch_shapes_do_not_change_counts(td, dev):
    """Determinism: every chunk / grid the autotuner may pick gives the same
    counts, and so do repeated runs."""
    X, Z = workloads.c1()
    rng = np.random.default_rng(3)
    X2 = rng.standard_normal((300, 4))
    Z2 = np.vstack([rng.standard_normal((3, 4)), X2[:2]])
    ref1 = oracle.depth_counts(X, Z)
    ref2 = oracle.depth_counts(X2, Z2)
    for chunk in (64, 128, 512):
        for grid in (17, 256, 2048):
            for prec in ("plain", "filtered", "bitonic"):
                a = td.depth(to_dev(X, dev), to_dev(Z, dev), chunk=chunk, grid_blocks=grid, **PREC_OPTS[prec])
                b = td.depth(to_dev(X2, dev), to_dev(Z2, dev), chunk=chunk, grid_blocks=grid, **PREC_OPTS[prec])
                assert np.array_equal(a.cpu().numpy(), ref1)
                assert np.array_equal(b.cpu().numpy(), ref2)


def test_autotune_then_depth(td, dev):
    td.autotune(4, 300)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 4))
    Z = np.vstack([rng.standard_normal((2, 4)), X[:1]])
    got = td.depth(to_dev(X, dev), to_dev(Z, dev))
    assert np.array_equal(got.cpu().numpy(), oracle.depth_counts(X, Z))


def c4_golden():
    """Stored oracle counts of the batched workload, merged over the files
    c4.json (the budget subsample) and c4.<part>.json (e.g. the p = 5
    datasets with n > 512 in c4.wide.json)."""
    g = {}
    for name in sorted(os.listdir(GOLD)):
        if name == "c4.json" or (name.startswith("c4.") and name.endswith(".json")):
            with open(os.path.join(GOLD, name)) as f:
                g.update(json.load(f)["counts"])
    return g


def test_c4_subsample_golden(td, dev):
    """All 256 datasets of the batched workload in one graph launch; the
    queries the oracle could afford (stored subsample, plus two queries per
    wide p = 5 kernel class) must match, the rest must satisfy
    d <= n0 + floor(n'/2) and d >= 0."""
    g = c4_golden()
    assert g, "c4 golden files missing"
    data = workloads.c4()
    dprobs = [(to_dev(X, dev), to_dev(Z, dev)) for X, Z in data]
    outs = [o.cpu().numpy() for o in td.depth_batched(dprobs)]
    bad = [(k, outs[int(k.split(":")[0])][int(k.split(":")[1])], v) for k, v in g.items()
           if outs[int(k.split(":")[0])][int(k.split(":")[1])] != v]
    assert not bad, bad[:10]
    for (X, Z), o in zip(data, outs):
        for q in range(Z.shape[0]):
            n0 = int(np.sum(np.all(X == Z[q], axis=1)))
            assert 0 <= o[q] <= n0 + (X.shape[0] - n0) // 2


def _class_n(K):
    """Smallest sample size whose sort width is 64 K (K a power of two) or,
    for 10, 12, 14 points per lane, the first size of that range."""
    return {1: 30, 2: 65, 4: 129, 8: 257, 16: 897, 10: 513, 12: 641, 14: 769}[K]


def test_batched_more_than_forty_classes(td, dev):
    """One call whose problems fall into 47 (p, points-per-lane) classes:
    p = 2..6 with 1, 2, 4, 8, 16 points per lane and 10, 12, 14 (bucketed
    sweep), p = 7 up to 8 and p = 8 up to 4.  Every problem has a query
    outside the hull (depth 0, which the pruning settles quickly) and the
    small ones a deep query checked against the oracle."""
    rng = np.random.default_rng(47)
    probs, deep = [], []
    classes = [(p, K) for p in range(2, 7) for K in (1, 2, 4, 8, 16, 10, 12, 14)]
    classes += [(7, K) for K in (1, 2, 4, 8)] + [(8, K) for K in (1, 2, 4)]
    assert len(classes) == 47
    for p, K in classes:
        n = max(_class_n(K), p + 2)
        X = rng.standard_normal((n, p))
        Z = workloads.outside_hull_query(X, rng)
        cheap = K <= 2 and p <= 6 or K == 1
        if cheap:
            Z = np.vstack([Z, 0.2 * rng.standard_normal((1, p))])
        probs.append((X, Z))
        deep.append(cheap)
    outs = td.depth_batched([(to_dev(X, dev), to_dev(Z, dev)) for X, Z in probs])
    st = td.get_stats()
    assert st["device_status"] == 0, st
    for (X, Z), o, c in zip(probs, outs, deep):
        o = o.cpu().numpy()
        assert o[0] == 0, (X.shape, o)
        if c:
            assert o[1] == oracle.depth_counts(X, Z[1:2])[0], (X.shape, o)


def test_batched_exact_tier_takes_each_deferred_subset_once(td, dev):
    """Four p = 5 problems whose kernels hold 10, 12, 14 and 16 points per
    lane share the sort width 1024.  A point duplicated along its ray from
    the query sends the subsets holding it to the exact tier; each deferred
    subset must be taken up by exactly one exact-tier launch, and the counts
    must equal the single calls'."""
    rng = np.random.default_rng(48)
    probs = []
    for n in (600, 700, 850, 1000):
        X = rng.standard_normal((n, 5))
        z = 0.2 * rng.standard_normal(5)
        X[1] = z + 2.0 * (X[0] - z)
        probs.append((X, np.vstack([z, 0.3 * rng.standard_normal((1, 5))])))
    dprobs = [(to_dev(X, dev), to_dev(Z, dev)) for X, Z in probs]
    outs = td.depth_batched(dprobs, prune=False)
    st = td.get_stats()
    assert st["device_status"] == 0, st
    assert st["deferred_subsets"] > 0
    assert st["exact_subsets"] == st["deferred_subsets"], st
    for (Xd, Zd), o in zip(dprobs, outs):
        single = td.depth(Xd, Zd, prune=False)
        s1 = td.get_stats()
        assert s1["exact_subsets"] == s1["deferred_subsets"]
        assert np.array_equal(o.cpu().numpy(), single.cpu().numpy())
