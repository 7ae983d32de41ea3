"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each pin is independent of the oracle's own code path:
  * p = 1 closed form min(#{X <= z}, #{X >= z}) (Section 3),
  * p = 2 exhaustive search over the circle (the definition, equation (1)),
  * the critical-direction route (equation (4)) in exact Python integers
    and in C++, on tiny inputs with heavy degeneracy (the paper validates its
    algorithms by agreement of independent methods, Section 5.1),
  * closed forms: exactly antipodal sets, queries outside the hull (vanishing
    at infinity, Section 1), duplication, affine invariance under exact
    integer maps, permutation invariance,
  * bounds: any direction gives an upper bound (definition), and
    d <= n0 + floor(n'/2),
  * the exact-only mode equals the filtered mode (the float64 filter never
    changes a decision).
A plausible slip in the oracle (a dropped correction term, a wrong sign or
fold, ungrouped ties, a transposed operand) fails at least one of these:
ungrouped ties and the literal (p-2) correction are caught by the lattice and
ray-duplicated families (see test_literal_variants_fail).
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import brute


def test_p1_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(1, 30))
        X = rng.integers(-3, 4, size=(n, 1)).astype(float)
        z = np.array([float(rng.integers(-3, 4))])
        assert oracle.depth_counts(X, z[None])[0] == brute.depth_p1(X, z)


def test_p2_angular_brute_force():
    rng = np.random.default_rng(2)
    for _ in range(300):
        n = int(rng.integers(1, 14))
        X, Z = workloads.lattice_small(rng, 2, n, R=3)
        assert oracle.depth_counts(X, Z)[0] == brute.depth_angular_p2(X, Z[0])


@pytest.mark.parametrize("p", [2, 3, 4])
def test_vertex_route_python_lattice(p):
    rng = np.random.default_rng(30 + p)
    for _ in range(120 if p < 4 else 60):
        n = int(rng.integers(p + 1, 10 if p < 4 else 8))
        X, Z = workloads.lattice_small(rng, p, n, R=2)
        a = oracle.depth_counts(X, Z)[0]
        assert a == brute.depth_vertex(X, Z[0])
        assert a == oracle.depth_vertex(X, Z[0])


@pytest.mark.parametrize("p", [3, 4, 5])
def test_vertex_route_degenerate_families(p):
    rng = np.random.default_rng(40 + p)
    for t in range(25):
        if t % 3 == 0:
            X, Z = workloads.ray_duplicated(rng, p, int(rng.integers(2, 5)))
        elif t % 3 == 1:
            X, Z = workloads.rank_deficient(rng, p, int(rng.integers(p, 9)), int(rng.integers(1, p)))
        else:
            X, Z = workloads.near_degenerate(rng, p, int(rng.integers(p + 1, 9)))
        a = oracle.depth_counts(X, Z)[0]
        assert a == oracle.depth_vertex(X, Z[0])
        if X.shape[0] <= 8:
            assert a == brute.depth_vertex(X, Z[0])


def test_exact_only_equals_filtered():
    rng = np.random.default_rng(5)
    for p in (3, 4, 5):
        X = rng.standard_normal((30, p))
        Z = np.vstack([rng.standard_normal((2, p)), X[:1]])
        assert np.array_equal(oracle.depth_counts(X, Z), oracle.depth_counts(X, Z, exact_only=True))
    for p in (3, 4):
        X, Z = workloads.lattice_small(rng, p, 11, R=2)
        assert np.array_equal(oracle.depth_counts(X, Z), oracle.depth_counts(X, Z, exact_only=True))


def test_symmetric_closed_form():
    rng = np.random.default_rng(6)
    for p, k in [(3, 80), (4, 50), (5, 25), (6, 12)]:
        for center in (False, True):
            X, Z = workloads.symmetric(rng, p, k, with_center=center)
            assert oracle.depth_counts(X, Z)[0] == k + (1 if center else 0)


def test_outside_hull_is_zero():
    rng = np.random.default_rng(7)
    for p in (2, 3, 4, 5):
        X = rng.standard_normal((60, p))
        assert oracle.depth_counts(X, workloads.outside_hull_query(X, rng))[0] == 0


def test_duplication_scales():
    rng = np.random.default_rng(8)
    for p in (3, 4):
        X = rng.standard_normal((18, p))
        Z = np.vstack([rng.standard_normal((2, p)), X[:1]])
        d1 = oracle.depth_counts(X, Z)
        for k in (2, 3):
            assert np.array_equal(oracle.depth_counts(workloads.duplicated(X, k), Z), k * d1)


def test_affine_invariance_exact_integer_maps():
    rng = np.random.default_rng(9)
    for p in (3, 4, 5):
        X, Z = workloads.lattice_small(rng, p, 12, R=3)
        U = workloads.unimodular(rng, p, steps=6)
        A = np.array(U, dtype=np.int64) * 3
        b = rng.integers(-5, 6, size=p)
        Xm = (X.astype(np.int64) @ A.T + b).astype(np.float64)
        Zm = (Z.astype(np.int64) @ A.T + b).astype(np.float64)
        assert oracle.depth_counts(Xm, Zm)[0] == oracle.depth_counts(X, Z)[0]


def test_c5_map_invariance():
    """The mapped stress data has the depths of its pre-map lattice."""
    X, Z, info = workloads.c5(return_premap=True)
    X0 = info["X0"].astype(np.float64)
    Z0 = info["Z0"].astype(np.float64)
    rng = np.random.default_rng(10)
    idx = rng.choice(len(X0), 30, replace=False)
    for q in (0, 3, 9):
        assert (oracle.depth_counts(X[idx], Z[q:q + 1])[0]
                == oracle.depth_counts(X0[idx], Z0[q:q + 1])[0])


def test_permutation_invariance():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((25, 4))
    Z = rng.standard_normal((3, 4))
    perm = rng.permutation(25)
    assert np.array_equal(oracle.depth_counts(X, Z), oracle.depth_counts(X[perm], Z))


def test_upper_bounds():
    rng = np.random.default_rng(12)
    for p in (3, 4, 5):
        X = rng.standard_normal((40, p))
        Z = np.vstack([rng.standard_normal((3, p)), X[:2]])
        d = oracle.depth_counts(X, Z)
        U = rng.standard_normal((3000, p))
        for q in range(Z.shape[0]):
            x = X - Z[q]
            dirs = np.vstack([U, x, -x])
            assert d[q] <= brute.upper_bound_directions(X, Z[q], dirs)
            n0 = int(np.sum(np.all(x == 0, axis=1)))
            assert d[q] <= n0 + (X.shape[0] - n0) // 2


def test_centerpoint_bound_at_symmetry_centre():
    """Soft check: for a centrally symmetric law the centre is deep, at least
    the centerpoint bound ceil(n/(p+1))."""
    rng = np.random.default_rng(13)
    for p in (3, 4):
        X, Z = workloads.symmetric(rng, p, 20)
        assert oracle.depth_counts(X, Z)[0] >= int(np.ceil(X.shape[0] / (p + 1)))


def test_literal_variants_fail():
    """Negative control: the literal steps of the paper (correction p-2 for
    all points inside span(x_I), per-element updates inside tie runs) differ
    from the exact count on degenerate data, so the pins above can see such a
    slip."""
    from oracle import literal
    rng = np.random.default_rng(14)
    diffs = 0
    for _ in range(40):
        X, Z = workloads.ray_duplicated(rng, 3, 4)
        diffs += int(literal.depth_literal(X, Z[0]) != oracle.depth_counts(X, Z)[0])
    assert diffs > 0


# ---------------------------------------------------------- Algorithm 3 (ADIA)
def test_adia_oracle_equals_depth_in_general_position():
    """The paper reports the exact depth from its adaptive algorithm in all
    its experiments (general position); the oracle's ADIA must agree with the
    exact count on such data, across dimensions and depths (shallow, deep,
    sample points, outside the hull)."""
    rng = np.random.default_rng(91)
    for p, n in [(3, 120), (4, 60), (5, 36), (6, 22)]:
        X = rng.standard_normal((n, p))
        Z = np.vstack([0.3 * rng.standard_normal((3, p)), X[:2], 1.5 * rng.standard_normal((2, p)),
                       workloads.outside_hull_query(X, rng)])
        got, ks = oracle.depth_adia(X, Z)
        exp = oracle.depth_counts(X, Z)
        assert np.array_equal(got, exp), (p, n, got, exp)
        # Step 5 looks at fewer points than the sample for shallow queries
        assert np.all(ks[ks >= 0] <= n)


def test_adia_oracle_never_below_depth():
    """ADIA's value is attained by some subset, so it is never below the
    depth, whatever the data (degenerate families)."""
    rng = np.random.default_rng(92)
    for t in range(40):
        p = int(rng.integers(3, 6))
        kind = t % 3
        if kind == 0:
            X, Z = workloads.lattice_small(rng, p, int(rng.integers(p + 6, 16)), R=2)
        elif kind == 1:
            X, Z = workloads.ray_duplicated(rng, p, int(rng.integers(5, 9)))
        else:
            X, Z = workloads.near_degenerate(rng, p, int(rng.integers(p + 6, 16)))
        got, _ = oracle.depth_adia(X, Z)
        exp = oracle.depth_counts(X, Z)
        assert got[0] >= exp[0], (t, got, exp)


def test_adia_oracle_small_samples_use_algorithm_1():
    """n <= 2p or p < 3: the paper's advice is Algorithm 1 (reported with
    ksize -1), so the count is the exact one."""
    rng = np.random.default_rng(93)
    for p, n in [(2, 30), (3, 6), (5, 10)]:
        X = rng.standard_normal((n, p))
        Z = rng.standard_normal((2, p))
        got, ks = oracle.depth_adia(X, Z)
        assert np.array_equal(got, oracle.depth_counts(X, Z))
        assert np.all(ks == -1)
