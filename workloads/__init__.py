"""Seeded synthetic inputs for the Tukey-depth hot path.

This module only draws random numbers and arranges them into arrays of the
shapes the experiments use; it contains none of the depth arithmetic, so both
the HIP path and the CPU oracle can consume its output without sharing any
method code.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``
(PCG64); arrays are float64, row-major, one observation per row.

Workloads (sizes follow the paper's simulation design, Section 5.2, and the
headline configurations of this project):

* ``c1`` : p=3, n=100 points from N(0, I_3), m=10 queries from N(0, I_3).
* ``c2`` : p=4, n=1000 points from N(0, S) with S_ij = 0.5^|i-j|; 100 queries
           from the same law plus 10 queries from 5x that law (shallow points).
* ``c3`` : p=5, n=500 points from a multivariate Student-t with 3 degrees of
           freedom (identity scale); 16 queries are exact copies of sample
           points, 16 are drawn from N(0, I_5).
* ``c4`` : 256 datasets, p uniform in {3,4,5}, n uniform in [50, 800],
           points from N(0, I_p) or U[-1,1]^p (fair coin), 8 queries each
           from the same law.
* ``c5`` : p=6, n=200 points of the integer lattice {-20..20}^6 with planted
           structure (points on a lattice hyperplane and on a 3-flat), 16
           queries (8 sample points, 8 lattice points), then an exact integer
           affine map with 2-norm condition number in [5e5, 2e6], scaled by
           the odd integer 65521.  All mapped coordinates are integers below
           2^40, so the map is exact in float64 and exact ties survive; about
           30% of centred coordinates exceed 2^24, so float32 rounding is
           real.
* ``p2`` : p=2, n=1024 points from N(0, I_2), m=1024 queries (512 sample
           points, 512 from N(0, I_2)): one sweep of 1023 or 1024 points per
           query (Algorithm 2 on its own).
* ``grid``: the paper's speed-comparison design: N(0, I_p), z = alpha * 1_p.
* ``observations``: the depth of every observation (queries = the sample) on
           seeded stand-ins with the shapes of the paper's two real data sets
           (Section 5.1; the data themselves are not available): ``"scores"``,
           64 rows of four strongly correlated scores that rise from column to
           column, rounded to 0.01; ``"returns"``, 500 rows of four weakly
           correlated heavy-tailed (Student-t, 4 degrees of freedom) daily
           returns of scale 0.015, rounded to 1e-6.  As in the paper, p = 3
           uses the first three columns and a smaller n the first n rows.

Degenerate families for parity tests (small n, heavy exact degeneracy):
``lattice_small``, ``ray_duplicated``, ``rank_deficient``, ``near_degenerate``,
``symmetric``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "c1", "c2", "c3", "c4", "c5", "p2", "grid", "observations", "config",
    "lattice_small", "ray_duplicated", "rank_deficient", "near_degenerate",
    "symmetric", "duplicated", "outside_hull_query", "unimodular", "wide",
    "WIDE_CASES", "ADIA_GRID_CASES",
]


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def c1(seed: int = 0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((100, 3))
    Z = rng.standard_normal((10, 3))
    return _f64(X), _f64(Z)


def c2(seed: int = 2):
    rng = np.random.default_rng(seed)
    p = 4
    S = np.array([[0.5 ** abs(i - j) for j in range(p)] for i in range(p)])
    L = np.linalg.cholesky(S)
    X = rng.standard_normal((1000, p)) @ L.T
    Zin = rng.standard_normal((100, p)) @ L.T
    Zout = 5.0 * (rng.standard_normal((10, p)) @ L.T)
    return _f64(X), _f64(np.vstack([Zin, Zout]))


def c3(seed: int = 3):
    rng = np.random.default_rng(seed)
    n, p = 500, 5
    G = rng.standard_normal((n, p))
    W = rng.chisquare(3, size=n)
    X = G / np.sqrt(W / 3.0)[:, None]
    idx = rng.choice(n, 16, replace=False)
    Zs = X[idx].copy()
    Zg = rng.standard_normal((16, p))
    return _f64(X), _f64(np.vstack([Zs, Zg]))


def c4(seed: int = 4, num: int = 256, queries: int = 8):
    """List of (X, Z) pairs of uneven n and p."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(num):
        p = int(rng.integers(3, 6))
        n = int(rng.integers(50, 801))
        law = int(rng.integers(0, 2))
        if law == 0:
            X = rng.standard_normal((n, p))
            Z = rng.standard_normal((queries, p))
        else:
            X = rng.uniform(-1.0, 1.0, size=(n, p))
            Z = rng.uniform(-1.0, 1.0, size=(queries, p))
        out.append((_f64(X), _f64(Z)))
    return out


def p2(seed: int = 7):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((1024, 2))
    idx = rng.choice(1024, 512, replace=False)
    Z = np.vstack([X[idx], rng.standard_normal((512, 2))])
    return _f64(X), _f64(Z)


def unimodular(rng, p: int, steps: int = 12):
    """Random integer matrix with determinant +-1: a signed permutation
    times a product of integer shears I + c E_ij (c in {-2..2}, i != j)."""
    U = np.eye(p, dtype=object)
    for _ in range(steps):
        i, j = rng.choice(p, 2, replace=False)
        c = int(rng.integers(-2, 3))
        E = np.eye(p, dtype=object)
        E[i, j] = c
        U = U.dot(E)
    perm = rng.permutation(p)
    signs = rng.choice([-1, 1], size=p)
    P = np.zeros((p, p), dtype=object)
    for r in range(p):
        P[r, perm[r]] = int(signs[r])
    return P.dot(U)


def c5(seed: int = 5, return_premap: bool = False):
    """Near-degenerate lattice stress case (see module docstring).

    Structure planted before the map (coordinates in {-20..20}^6):
      * 156 i.i.d. uniform lattice points,
      * 28 points on the lattice hyperplane {v_6 = 7}: with a query on that
        hyperplane, every subset drawn from it sees the rest of it as one
        exactly tied angular run,
      * 16 points on the 3-flat {v_4 = -5, v_5 = 3, v_6 = 7} (inside the
        hyperplane): with a query on it, subsets holding three of its points
        see the others inside their own span (degenerate subsets).
    Queries: 3 sample points on the flat, 3 on the hyperplane (off the
    flat), 2 i.i.d. sample points, 8 uniform lattice points.
    The affine map T(v) = A v + b is exact integer arithmetic; A =
    U1 diag(1,1,1,1,1,2^k) U2 with unimodular U1, U2, and k chosen so that
    cond_2(A) lands in [5e5, 2e6].
    """
    rng = np.random.default_rng(seed)
    p = 6
    iid = rng.integers(-20, 21, size=(156, p))
    hyp = rng.integers(-20, 21, size=(28, p))
    hyp[:, 5] = 7
    flat = rng.integers(-20, 21, size=(16, p))
    flat[:, 3] = -5
    flat[:, 4] = 3
    flat[:, 5] = 7
    X0 = np.vstack([iid, hyp, flat]).astype(np.int64)
    order = rng.permutation(len(X0))
    X0 = X0[order]
    inv = np.argsort(order)
    # positions (after the shuffle) of each planted group
    pos_iid = inv[:156]
    pos_hyp = inv[156:184]
    pos_flat = inv[184:200]
    qsel = np.concatenate([
        rng.choice(pos_flat, 3, replace=False),
        rng.choice(pos_hyp, 3, replace=False),
        rng.choice(pos_iid, 2, replace=False),
    ])
    Z0 = np.vstack([X0[qsel], rng.integers(-20, 21, size=(8, p))]).astype(np.int64)

    # exact affine map with a prescribed condition number
    for _ in range(200):
        U1 = unimodular(rng, p)
        U2 = unimodular(rng, p)
        chosen = None
        for k in range(0, 40):
            D = np.diag([1, 1, 1, 1, 1, 2 ** k]).astype(object)
            A = U1.dot(D).dot(U2)
            c = np.linalg.cond(A.astype(np.float64))
            if 5e5 <= c <= 2e6:
                chosen = (A, k, c)
                break
            if c > 2e6:
                break
        if chosen is not None:
            break
    A, k, cond = chosen
    # an odd integer scale lifts many centred coordinates above 2^24 so that
    # float32 rounding is real, while every value stays an exact float64
    A = A * 65521
    b = np.array([int(v) for v in rng.integers(-1000, 1001, size=p)], dtype=object)

    def T(V):
        V = V.astype(object)
        out = V.dot(A.T) + b
        return out

    Xm = T(X0)
    Zm = T(Z0)
    big = max(abs(int(v)) for v in np.concatenate([Xm.ravel(), Zm.ravel()]))
    assert big < 2 ** 40, big
    X = _f64(np.array(Xm, dtype=np.float64))
    Z = _f64(np.array(Zm, dtype=np.float64))
    # every value is an exactly representable integer
    assert np.all(X == np.array(Xm, dtype=np.float64))
    if return_premap:
        return X, Z, dict(X0=X0, Z0=Z0, A=A, b=b, k=k, cond=cond)
    return X, Z


def grid(p: int, n: int, alpha: float, seed: int = 0):
    """Paper's simulation design: X ~ N(0, I_p), z = alpha * 1_p."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p))
    Z = np.full((1, p), float(alpha))
    return _f64(X), _f64(Z)


def observations(kind: str, p: int, n: int, seed: int = 6):
    """Sample whose every observation is a query (Z = X).  ``kind`` is
    ``"scores"`` (up to 64 rows) or ``"returns"`` (up to 500 rows); p <= 4."""
    rng = np.random.default_rng(seed)
    if kind == "scores":
        rows = 64
        S = np.full((4, 4), 0.8) + 0.2 * np.eye(4)
        mu = np.array([0.0, 0.5, 1.0, 1.5])
        A = mu + 2.0 * rng.standard_normal((rows, 4)) @ np.linalg.cholesky(S).T
        A = np.round(A, 2)
    elif kind == "returns":
        rows = 500
        rng = np.random.default_rng(seed + 1)
        S = np.full((4, 4), 0.1) + 0.9 * np.eye(4)
        G = rng.standard_normal((rows, 4)) @ np.linalg.cholesky(S).T
        W = rng.chisquare(4.0, size=(rows, 1))
        A = np.round(0.015 * G / np.sqrt(W / 4.0), 6)
    else:
        raise KeyError(kind)
    if not (1 <= p <= 4 and 1 <= n <= rows):
        raise ValueError("observations(%r): p <= 4 and n <= %d" % (kind, rows))
    X = _f64(A[:n, :p])
    return X, X.copy()


# Samples sized at the ends of the kernel classes that hold 10, 12 or 14
# points per lane (p = 5, 512 < n <= 896) and of the 8-points-per-lane class
# at p = 6 (260 < n <= 516): name -> (p, n, seed).
WIDE_CASES = {
    "p5n640": (5, 640, 640),
    "p5n768": (5, 768, 768),
    "p6n270": (6, 270, 270),
}


def wide(name: str):
    """N(0, I_p) sample of one of ``WIDE_CASES`` with two queries: a deep
    point 0.3 * N(0, I_p) and a sample point (n0 = 1)."""
    p, n, seed = WIDE_CASES[name]
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p))
    Z = np.vstack([0.3 * rng.standard_normal((1, p)), X[n // 3:n // 3 + 1]])
    return _f64(X), _f64(Z)


# Grid cases (p, n, alpha) whose Algorithm 3 counts are stored: the deep
# query at p = 6, n = 320 is one where the paper's adaptive algorithm stops
# above the depth.
ADIA_GRID_CASES = [(6, 320, 0.0), (6, 320, 0.4), (5, 640, 0.0), (5, 640, 0.4), (4, 640, 0.8)]


def config(name: str):
    name = name.lower()
    if name == "c1":
        return c1()
    if name == "c2":
        return c2()
    if name == "c3":
        return c3()
    if name == "c5":
        return c5()
    if name == "c4":
        return c4()
    if name == "p2":
        return p2()
    raise KeyError(name)


# ---------------------------------------------------------------- degenerate
def lattice_small(rng, p: int, n: int, R: int = 2, z_mode: str = "mixed"):
    """n points of {-R..R}^p; the query is a lattice point of {-1..1}^p or a
    sample point (z_mode 'lattice' / 'sample' / 'mixed' = coin flip)."""
    X = rng.integers(-R, R + 1, size=(n, p)).astype(np.float64)
    mode = z_mode
    if mode == "mixed":
        mode = "sample" if rng.integers(0, 2) else "lattice"
    if mode == "sample":
        z = X[rng.integers(0, n)].copy()
    else:
        z = rng.integers(-1, 2, size=p).astype(np.float64)
    return _f64(X), _f64(z[None, :])


def ray_duplicated(rng, p: int, n_base: int, R: int = 3):
    """Each base point relative to the query is repeated at 2x along its ray,
    so every subset holding one copy sees the other inside its span."""
    z = rng.integers(-2, 3, size=p).astype(np.float64)
    V = rng.integers(-R, R + 1, size=(n_base, p)).astype(np.float64)
    V = V[np.any(V != 0, axis=1)]
    X = np.vstack([z + V, z + 2.0 * V])
    return _f64(X), _f64(z[None, :])


def rank_deficient(rng, p: int, n: int, rank: int, R: int = 3):
    """Points whose differences from the query span only `rank` dimensions."""
    z = rng.integers(-2, 3, size=p).astype(np.float64)
    B = rng.integers(-2, 3, size=(rank, p)).astype(np.float64)
    C = rng.integers(-R, R + 1, size=(n, rank)).astype(np.float64)
    X = z + C @ B
    return _f64(X), _f64(z[None, :])


def near_degenerate(rng, p: int, n: int, R: int = 2, jitter: float = 1e-12):
    """Lattice points with a tiny float jitter on some coordinates: near ties
    that only exact predicates can order."""
    X = rng.integers(-R, R + 1, size=(n, p)).astype(np.float64)
    mask = rng.random((n, p)) < 0.3
    X = X + mask * rng.choice([-1.0, 1.0], size=(n, p)) * jitter * rng.integers(1, 4, size=(n, p))
    z = rng.integers(-1, 2, size=p).astype(np.float64)
    return _f64(X), _f64(z[None, :])


def symmetric(rng, p: int, k: int, with_center: bool = False):
    """2k points z +- v_j (v_j != 0) around a query z; the depth count is
    exactly k (plus one if z itself is a sample point).  z and v_j lie on the
    grid 2^-20 Z with |.| < 2^10, so z +- v_j is exact in float64 and the pairs
    are exactly antipodal about z."""
    z = np.round(rng.standard_normal(p) * 2.0**20) / 2.0**20
    V = np.round(rng.standard_normal((k, p)) * 2.0**20) / 2.0**20
    V[np.all(V == 0, axis=1), 0] = 2.0**-20
    X = np.vstack([z + V, z - V])
    if with_center:
        X = np.vstack([X, z[None, :]])
    X = X[rng.permutation(len(X))]
    return _f64(X), _f64(z[None, :])


def duplicated(X, times: int):
    return _f64(np.repeat(X, times, axis=0))


def outside_hull_query(X, rng):
    """A query beyond the largest value of a random coordinate."""
    c = int(rng.integers(0, X.shape[1]))
    z = X.mean(axis=0)
    z[c] = X[:, c].max() + 1.0
    return _f64(z[None, :])
