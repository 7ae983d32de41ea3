"""Small exact arbiters for the Tukey depth count (pure Python, exact ints).

TEST INFRASTRUCTURE ONLY: used by tests to pin the C++ oracle; never by the
product path.  Shares no code with the HIP path or with ``td_oracle.cpp``.

* ``depth_vertex``  -- the critical-direction route (equation (4), the
  p-1 subset form of Proposition 1): the optimum of the closed-halfspace count
  is attained next to an extreme ray of an open cone of the central hyperplane
  arrangement {u : u'x_i = 0}; such a ray is normal to p-1 independent points;
  next to it the count is the strict count plus the depth, inside the
  hyperplane, of the points lying on it.  O(n^p), tiny inputs only.
* ``depth_angular_p2`` -- p = 2 by brute force over the circle (the definition,
  equation (1)): every direction between two consecutive critical directions is
  generic; take the bisector of each consecutive pair and count.
* ``depth_p1`` -- p = 1 closed form min(#{X <= z}, #{X >= z}) (Section 3).
* ``upper_bound_directions`` -- the definition (equation (1)) evaluated at given directions: any
  direction gives an upper bound.
All inputs are floats; they are converted exactly with ``fractions.Fraction``
and scaled to integers by the common denominator.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


def _exact_centered(X, z):
    X = np.asarray(X, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64).reshape(-1)
    rows = [[Fraction(float(v)) - Fraction(float(c)) for v, c in zip(r, z)] for r in X]
    den = 1
    for r in rows:
        for v in r:
            den = den * v.denominator // math.gcd(den, v.denominator)
    return [[int(v * den) for v in r] for r in rows]


def _det(M):
    """Exact determinant of a small square integer matrix (Laplace)."""
    s = len(M)
    if s == 0:
        return 1
    if s == 1:
        return M[0][0]
    if s == 2:
        return M[0][0] * M[1][1] - M[0][1] * M[1][0]
    tot = 0
    for j in range(s):
        a = M[0][j]
        if a == 0:
            continue
        sub = [row[:j] + row[j + 1:] for row in M[1:]]
        tot += (-1) ** j * a * _det(sub)
    return tot


def _rank_rows(V, d):
    """Rank of integer vectors V (in Z^d) and a row set with a nonzero
    maximal minor (fraction-free elimination on a copy)."""
    basis = []
    for v in V:
        if len(basis) == d:
            break
        cand = basis + [v]
        s = len(cand)
        for rows in itertools.combinations(range(d), s):
            M = [[cand[c][r] for c in range(s)] for r in rows]
            if _det(M) != 0:
                basis = cand
                break
    r = len(basis)
    if r == 0:
        return 0, ()
    for rows in itertools.combinations(range(d), r):
        M = [[basis[c][rr] for c in range(r)] for rr in rows]
        if _det(M) != 0:
            return r, rows
    raise AssertionError("unreachable")


def _depth0(V, d):
    """min over generic u of #{v : u.v < 0} for nonzero integer vectors."""
    if not V:
        return 0
    r, rows = _rank_rows(V, d)
    if r < d:
        V = [[v[i] for i in rows] for v in V]
        d = r
    if d == 1:
        pos = sum(1 for v in V if v[0] > 0)
        return min(pos, len(V) - pos)
    best = len(V)
    for J in itertools.combinations(range(len(V)), d - 1):
        # generalised cross product: u_i = det[v_J | e_i]
        u = []
        for i in range(d):
            M = [[V[J[c]][rr] for c in range(d - 1)] + [1 if rr == i else 0] for rr in range(d)]
            u.append(_det(M))
        if not any(u):
            continue
        drop = next(i for i in range(d) if u[i] != 0)
        pos = neg = 0
        on = []
        for v in V:
            s = sum(a * b for a, b in zip(u, v))
            if s > 0:
                pos += 1
            elif s < 0:
                neg += 1
            else:
                on.append([v[i] for i in range(d) if i != drop])
        best = min(best, min(pos, neg) + _depth0(on, d - 1))
    return best


def depth_vertex(X, z):
    """Exact depth count n*D_n(z) by the critical-direction route."""
    x = _exact_centered(X, z)
    n0 = sum(1 for r in x if not any(r))
    W = [r for r in x if any(r)]
    d = len(x[0]) if x else 0
    return n0 + _depth0(W, d)


def depth_p1(X, z):
    X = np.asarray(X, dtype=np.float64).reshape(-1)
    z = float(np.asarray(z).reshape(-1)[0])
    return int(min(np.sum(X <= z), np.sum(X >= z)))


def depth_angular_p2(X, z):
    """p = 2: exact brute force over the circle.

    The count #{i : u.x_i < 0} is constant on the open arcs between the
    critical directions (normals of the x_i); the bisector of two consecutive
    distinct critical directions lies inside such an arc.  Points equal to z
    lie on every line and add n0."""
    x = _exact_centered(X, z)
    n0 = sum(1 for r in x if not any(r))
    W = [r for r in x if any(r)]
    if not W:
        return n0
    crit = []
    for a, b in W:
        crit.append((-b, a))
        crit.append((b, -a))

    def half(v):  # 0 for angle in [0, pi), 1 for [pi, 2pi)
        return 0 if (v[1] > 0 or (v[1] == 0 and v[0] > 0)) else 1

    def key_less(u, v):
        hu, hv = half(u), half(v)
        if hu != hv:
            return hu < hv
        return u[0] * v[1] - u[1] * v[0] > 0

    import functools

    def cmp(u, v):
        if key_less(u, v):
            return -1
        if key_less(v, u):
            return 1
        return 0

    crit = sorted(set(crit), key=functools.cmp_to_key(cmp))
    best = len(W)
    L = len(crit)
    for i in range(L):
        u, v = crit[i], crit[(i + 1) % L]
        nu = u[0] * u[0] + u[1] * u[1]
        nv = v[0] * v[0] + v[1] * v[1]
        cr = u[0] * v[1] - u[1] * v[0]
        if cr > 0:
            # arc shorter than pi: a positive combination lies strictly inside
            w = (u[0] * nv + v[0] * nu, u[1] * nv + v[1] * nu)
        elif cr < 0 or (u[0] * v[0] + u[1] * v[1]) < 0:
            # arc of pi or more: u turned by +90 degrees lies strictly inside
            w = (-u[1], u[0])
        else:
            continue  # same direction: empty arc
        cnt = sum(1 for a, b in W if w[0] * a + w[1] * b < 0)
        best = min(best, cnt)
    return n0 + best


def upper_bound_directions(X, z, U):
    """min over the directions u in U of #{i : u'(X_i - z) <= 0}: an upper
    bound of the depth count (the definition, equation (1))."""
    X = np.asarray(X, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64).reshape(-1)
    D = X - z
    best = X.shape[0]
    for u in U:
        best = min(best, int(np.sum(D @ u <= 0)))
    return best
