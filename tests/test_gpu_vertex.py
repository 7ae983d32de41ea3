"""The vertex-form check on the GPU (td_options.method = VERTEX): Proposition
1 with r = p - 1, every hyperplane through the query and p - 1 sample points,
each side decision certified in float64.  On data in general position its
counts must equal the oracle's and the RCom path's; on lattice data a query
either agrees or declines with TD_DEV_NOT_GENERAL, never another value."""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def run(td, dev, X, Z, **kw):
    c = td.depth(to_dev(X, dev), to_dev(np.atleast_2d(Z), dev), method="vertex", **kw)
    return c.cpu().numpy().astype(np.int64), td.get_stats()


def nprime(X, z):
    return int(np.sum(~np.all(X == z, axis=1)))


def test_vertex_c1(td, dev):
    X, Z = workloads.c1()
    g = json.load(open(os.path.join(GOLD, "c1.json")))["counts"]
    exp = np.array([g[str(q)] for q in range(Z.shape[0])])
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0, st
    assert np.array_equal(got, exp), (got, exp)
    # every (p-1)-subset of every query swept once
    assert st["subsets_swept"] == sum(math.comb(nprime(X, z), 2) for z in Z)


@pytest.mark.parametrize("p,n", [(2, 200), (3, 150), (4, 80), (5, 40), (6, 24), (7, 16), (8, 14)])
def test_vertex_general_position_vs_oracle_and_rcom(td, dev, p, n):
    rng = np.random.default_rng(900 + 7 * p + n)
    X = rng.standard_normal((n, p))
    Z = np.vstack([0.3 * rng.standard_normal((3, p)), X[:2]])
    print("vertex p=%d n=%d" % (p, n), flush=True)
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0, st
    exp = oracle.depth_counts(X, Z)
    assert np.array_equal(got, exp), (got, exp)
    rcom = td.depth(to_dev(X, dev), to_dev(Z, dev)).cpu().numpy()
    assert np.array_equal(got, rcom)


@pytest.mark.parametrize("p,n", [(3, 700), (4, 600), (2, 1024)])
def test_vertex_sixteen_points_per_lane(td, dev, p, n):
    """n > 512 at p <= 4: 16 points per lane."""
    rng = np.random.default_rng(960 + p)
    X = rng.standard_normal((n, p))
    Z = np.vstack([0.2 * rng.standard_normal((2, p)), X[:1]])
    got, st = run(td, dev, X, Z)
    assert st["device_status"] == 0, st
    assert np.array_equal(got, oracle.depth_counts(X, Z)), got


def test_vertex_c3_queries(td, dev):
    X, Z = workloads.c3()
    g = json.load(open(os.path.join(GOLD, "c3.json")))["counts"]
    qs = [0, 7, 16, 25]
    got, st = run(td, dev, X, Z[qs])
    assert st["device_status"] == 0, st
    assert np.array_equal(got, [g[str(q)] for q in qs]), got


@pytest.mark.parametrize("p", [2, 3, 4])
def test_vertex_lattice_declines_or_agrees(td, dev, p):
    rng = np.random.default_rng(930 + p)
    X, Z = workloads.lattice_small(rng, p, 40)
    got, st = run(td, dev, X, Z)
    exp = oracle.depth_counts(X, Z)
    assert np.all((got == exp) | (got == -1)), (got, exp)
    assert np.any(got == -1)
    assert "not_general" in st["device_status_bits"]


def test_vertex_limits_and_statuses(td, dev):
    rng = np.random.default_rng(940)
    # p = 1: the closed form
    X = rng.standard_normal((50, 1))
    got, _ = run(td, dev, X, np.array([[0.1], [X[3, 0]]]))
    assert np.array_equal(got, oracle.depth_counts(X, np.array([[0.1], [X[3, 0]]])))
    # n' < p - 1: no hyperplane through p - 1 points
    X = np.vstack([np.zeros((3, 4)), rng.standard_normal((2, 4))])
    got, st = run(td, dev, X, np.zeros((1, 4)))
    assert got[0] == -1 and "no_valid_subset" in st["device_status_bits"]
    # a non-finite query fails alone
    X = rng.standard_normal((30, 3))
    Z = rng.standard_normal((2, 3))
    Z[1, 0] = np.nan
    got, st = run(td, dev, X, Z)
    assert got[1] == -1 and "nonfinite" in st["device_status_bits"]
    assert got[0] == oracle.depth_counts(X, Z[:1])[0]
    # n above 512 is not supported by the check at p >= 5
    X = rng.standard_normal((600, 5))
    with pytest.raises(td.TDError) as e:
        run(td, dev, X, np.zeros((1, 5)))
    assert e.value.code == 2
    # nor by the batched and allocation-free entry points
    Xd, Zd = to_dev(X[:100], dev), to_dev(np.zeros((1, 5)), dev)
    with pytest.raises(td.TDError) as e:
        td.depth_batched([(Xd, Zd)], method="vertex")
    assert e.value.code == 2
    out = torch.zeros(1, dtype=torch.int32, device=Xd.device)
    with pytest.raises(td.TDError) as e:
        td.depth_noalloc(Xd, Zd, out, method="vertex")
    assert e.value.code == 2
