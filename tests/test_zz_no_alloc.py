"""td_depth_noalloc: the allocation-free variant of td_depth_ex (workspace in
a static device array) gives the same counts as td_depth_ex, on calls in a
row that reuse the array with a smaller input the second time, and rejects a
call larger than the array with TD_ERR_TOO_LARGE before launching anything."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _noalloc(td, dev, X, Z, **kw):
    import torch
    Xd, Zd = to_dev(X, dev), to_dev(np.atleast_2d(Z), dev)
    out = torch.full((Zd.shape[0],), -7, dtype=torch.int32, device=dev)
    td.depth_noalloc(Xd, Zd, out, **kw)
    got = out.cpu().numpy().astype(np.int64)
    return got, td.get_stats()


def _alloc(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), **kw)
    return c.cpu().numpy().astype(np.int64)


def test_noalloc_equals_depth_ex_twice_shrinking(td, dev):
    rng = np.random.default_rng(71)
    X1 = rng.standard_normal((300, 5))
    Z1 = np.vstack([0.3 * rng.standard_normal((6, 5)), X1[:2]])
    X2 = rng.standard_normal((60, 4))
    Z2 = np.vstack([0.3 * rng.standard_normal((2, 4)), X2[:1]])
    for kw in ({}, {"sweep": "bitonic"}, {"precision": "plain"}):
        a1, s1 = _noalloc(td, dev, X1, Z1, **kw)
        assert s1["device_status"] == 0
        assert s1["subsets_swept"] + s1["deferred_subsets"] + s1["pruned_subsets"] > 0
        b1 = _alloc(td, dev, X1, Z1, **kw)
        assert np.array_equal(a1, b1), (kw, a1, b1)
        a2, _ = _noalloc(td, dev, X2, Z2, **kw)
        b2 = _alloc(td, dev, X2, Z2, **kw)
        assert np.array_equal(a2, b2), (kw, a2, b2)
        assert np.array_equal(a2, oracle.depth_counts(X2, Z2))


def test_noalloc_degenerate_and_small_cases(td, dev):
    """The exact tier (deferred subsets in the static list), p = 1, p = 2,
    a query equal to every sample point's copy, and c1 against the oracle."""
    rng = np.random.default_rng(72)
    cases = [workloads.c1()]
    for p in (3, 4):
        cases.append(workloads.lattice_small(rng, p, 12, R=2))
        cases.append(workloads.ray_duplicated(rng, p, 6))
    X = rng.standard_normal((50, 1))
    cases.append((X, np.vstack([X[:2], [[0.0]]])))
    X = rng.standard_normal((70, 2))
    cases.append((X, np.vstack([X[:1], 0.1 * rng.standard_normal((2, 2))])))
    for X, Z in cases:
        a, st = _noalloc(td, dev, X, Z)
        b = _alloc(td, dev, X, Z)
        assert np.array_equal(a, b), (X.shape, a, b)
        assert np.array_equal(a, oracle.depth_counts(X, Z)), (X.shape, a)
        a, _ = _noalloc(td, dev, X, Z, force_exact=True)
        assert np.array_equal(a, b), (X.shape, a, b)


def test_noalloc_too_large_is_rejected(td, dev):
    import torch
    rng = np.random.default_rng(73)
    # p = 5, n = 1024: about 180 KB of per-query arrays, 2000 queries need
    # 368 MB, more than the 128 MiB array
    X = rng.standard_normal((1024, 5))
    Z = rng.standard_normal((2000, 5))
    out = torch.zeros(2000, dtype=torch.int32, device=dev)
    with pytest.raises(td.TDError) as e:
        td.depth_noalloc(to_dev(X, dev), to_dev(Z, dev), out)
    assert e.value.code == 7
    assert int(out.abs().sum().item()) == 0
    # the array still serves the next call
    X2 = rng.standard_normal((40, 3))
    Z2 = rng.standard_normal((3, 3))
    a, _ = _noalloc(td, dev, X2, Z2)
    assert np.array_equal(a, oracle.depth_counts(X2, Z2))
