"""The stored expected counts (tests/golden, written by make_golden.py from
the oracle only): they cover the kernel classes the parity tests need, and
every stored count respects bounds that hold for any input:
0 <= d <= n0 + floor(n'/2) (a direction and its negation split the
nonzero points)."""
import json
import os

import numpy as np

import workloads

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(prefix):
    g = {}
    for name in sorted(os.listdir(GOLD)):
        if (name == prefix + ".json" or name.startswith(prefix + ".")) and name.endswith(".json"):
            with open(os.path.join(GOLD, name)) as f:
                g.update(json.load(f)["counts"])
    return g


def _bound(X, z):
    n0 = int(np.sum(np.all(X == z, axis=1)))
    return n0 + (X.shape[0] - n0) // 2


def test_c4_wide_classes_covered():
    """At least two stored queries for each p = 5 kernel class holding 10,
    12 and 14 points per lane (512 < n <= 896)."""
    data = workloads.c4()
    per = {10: 0, 12: 0, 14: 0}
    g = _load("c4")
    for k, v in g.items():
        d, q = (int(t) for t in k.split(":"))
        X, Z = data[d]
        assert 0 <= v <= _bound(X, Z[q]), (k, v)
        n, p = X.shape
        if p == 5 and 512 < n <= 896:
            per[(n + 127) // 128 * 2] += 1
    assert min(per.values()) >= 2, per


def test_wide_cases_covered():
    g = _load("wide")
    for name in workloads.WIDE_CASES:
        X, Z = workloads.wide(name)
        keys = [k for k in g if k.startswith(name + ":")]
        assert keys, name
        for k in keys:
            q = int(k.split(":")[1])
            assert 0 <= g[k] <= _bound(X, Z[q]), (k, g[k])


def test_config_goldens_within_bounds():
    for cfg in ("c1", "c2", "c3"):
        X, Z = workloads.config(cfg)
        for k, v in _load(cfg).items():
            assert 0 <= v <= _bound(X, Z[int(k)]), (cfg, k, v)


def test_adia_grid_covered():
    """adia.json: Algorithm 3's value and candidate count for every case of
    workloads.ADIA_GRID_CASES, each at or above the exact count where that is
    stored, and within the bound that holds for any count."""
    with open(os.path.join(GOLD, "adia.json")) as f:
        g = json.load(f)
    for p, n, alpha in workloads.ADIA_GRID_CASES:
        key = "%d,%d,%.1f" % (p, n, alpha)
        X, Z = workloads.grid(p, n, alpha)
        assert key in g["adia"] and key in g["candidates"], key
        assert 0 <= g["adia"][key] <= _bound(X, Z[0])
        assert p - 2 <= g["candidates"][key] <= n
        if key in g["exact"]:
            assert g["exact"][key] <= g["adia"][key]


def test_adia_observations_covered():
    """adia_obs.json: for every observation of the real-data stand-ins, the
    exact count and Algorithm 3's value, never below it, both within the
    bound; every observation is a sample point, so n0 >= 1 and the depth
    count is at least 1."""
    with open(os.path.join(GOLD, "adia_obs.json")) as f:
        g = json.load(f)
    keys = {("scores", 3, 64), ("scores", 4, 64), ("returns", 3, 200), ("returns", 4, 200), ("returns", 4, 500)}
    for kind, p, n in keys:
        key = "%s,%d,%d" % (kind, p, n)
        X, Z = workloads.observations(kind, p, n)
        a, e = g["adia"][key], g["exact"][key]
        assert len(a) == len(e) == n, key
        for q in range(n):
            assert 1 <= e[q] <= a[q] <= _bound(X, Z[q]), (key, q, e[q], a[q])
