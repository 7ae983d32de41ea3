"""The edges of the supported range against the oracle: the largest
dimensions (p = 7, 8, where a subset has 5 or 6 members and the sort classes
run at one or two waves per SIMD) and the largest sample (n = 1024, the full
sort width, where p = 2 puts 1024 points in one sweep)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from conftest import PREC_OPTS, to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

PRECS = ["filtered", "bitonic", "plain"]


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), **kw)
    return c.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p,n", [(7, 8), (7, 13), (7, 20), (8, 9), (8, 14), (8, 17)])
def test_largest_dimensions(td, dev, prec, p, n):
    rng = np.random.default_rng(40 + 3 * p + n)
    X = rng.standard_normal((n, p))
    Z = np.vstack([rng.standard_normal((2, p)), X[:1], 4.0 * rng.standard_normal((1, p))])
    exp = oracle.depth_counts(X, Z)
    got = run(td, dev, X, Z, **PREC_OPTS[prec])
    assert np.array_equal(got, exp), (got, exp)


@pytest.mark.parametrize("prec", ["filtered", "bitonic"])
@pytest.mark.parametrize("p", [7, 8])
def test_largest_dimensions_lattice(td, dev, prec, p):
    """Exact ties and points inside span(x_I) at the largest dimensions."""
    rng = np.random.default_rng(70 + p)
    X, Z = workloads.lattice_small(rng, p, 12, R=1)
    exp = oracle.depth_counts(X, Z)
    got = run(td, dev, X, Z, **PREC_OPTS[prec])
    assert np.array_equal(got, exp), (got, exp)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [2, 3])
def test_largest_sample(td, dev, prec, p):
    rng = np.random.default_rng(90 + p)
    X = rng.standard_normal((1024, p))
    Z = np.vstack([rng.standard_normal((2, p)), X[5:6], 3.0 * rng.standard_normal((1, p))])
    exp = oracle.depth_counts(X, Z)
    got = run(td, dev, X, Z, **PREC_OPTS[prec])
    st = td.get_stats()
    assert st["device_status"] == 0
    assert np.array_equal(got, exp), (got, exp)


# Samples of 512 < n <= 896 at p <= 6 run the bucketed kernel with 10, 12 or
# 14 points per lane instead of 16 (n up to 640, 768, 896); every end of those
# ranges, and 897, the first sample back on 16.
@pytest.mark.parametrize("p,n", [(3, 513), (3, 640), (3, 641), (3, 768), (3, 769), (3, 896), (3, 897),
                                 (4, 513), (4, 640), (4, 641), (4, 768), (4, 769), (4, 896), (4, 897)])
def test_narrow_points_per_lane(td, dev, p, n):
    rng = np.random.default_rng(200 + 7 * p + n)
    X = rng.standard_normal((n, p))
    X[-3:] = X[:3]   # duplicated observations (n0 = 2 for the sample queries)
    Z = np.vstack([rng.standard_normal((2, p)), X[:1], X[n // 2:n // 2 + 1], 3.0 * rng.standard_normal((1, p))])
    exp = oracle.depth_counts(X, Z)
    got = run(td, dev, X, Z)
    assert td.get_stats()["device_status"] == 0
    assert np.array_equal(got, exp), (got, exp)


def _wide_golden():
    with open(os.path.join(GOLD, "wide.json")) as f:
        return json.load(f)["counts"]


@pytest.mark.parametrize("name", sorted(workloads.WIDE_CASES))
@pytest.mark.parametrize("prec", ["filtered", "bitonic"])
def test_wide_classes_vs_stored_oracle(td, dev, name, prec):
    """Samples at the ends of the kernel classes (p = 5: n = 640, the last
    sample on 10 points per lane, and n = 768, the last on 12; p = 6: n = 270,
    8 points per lane) against stored oracle counts, both filtered sweeps."""
    g = _wide_golden()
    X, Z = workloads.wide(name)
    qs = [q for q in range(Z.shape[0]) if "%s:%d" % (name, q) in g]
    assert qs, "no stored count for %s" % name
    exp = np.array([g["%s:%d" % (name, q)] for q in qs])
    got = run(td, dev, X, Z[qs], **PREC_OPTS[prec])
    assert td.get_stats()["device_status"] == 0
    assert np.array_equal(got, exp), (got, exp)


@pytest.mark.parametrize("n", [600, 700, 850])
def test_narrow_points_per_lane_p5(td, dev, n):
    """p = 5: the bucketed kernel (10, 12 and 14 points per lane) against the
    full bitonic sort and the plain float64 tier (16 points per lane), which
    order the points independently of it."""
    rng = np.random.default_rng(n + 1)
    X = rng.standard_normal((n, 5))
    Z = np.vstack([0.2 * rng.standard_normal((2, 5)), X[:1], 2.5 * rng.standard_normal((1, 5))])
    a = run(td, dev, X, Z)
    assert td.get_stats()["device_status"] == 0
    b = run(td, dev, X, Z, **PREC_OPTS["bitonic"])
    c = run(td, dev, X, Z, **PREC_OPTS["plain"])
    assert np.array_equal(a, b), (a, b)
    assert np.array_equal(a, c), (a, c)


def test_narrow_points_per_lane_p6(td, dev):
    """p = 6, n = 520 (10 points per lane), one central query: bucketed
    against bitonic."""
    rng = np.random.default_rng(520)
    X = rng.standard_normal((520, 6))
    Z = np.zeros((1, 6))
    a = run(td, dev, X, Z)
    assert td.get_stats()["device_status"] == 0
    b = run(td, dev, X, Z, **PREC_OPTS["bitonic"])
    assert np.array_equal(a, b), (a, b)
