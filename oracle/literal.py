"""The paper's first algorithm taken literally in float64 (documentation and
negative controls only; TEST INFRASTRUCTURE, never used by the product path).

Algorithm 1: for every (p-2)-subset, an orthonormal basis of the complement
(here from a complete QR factorisation), projections y_i, then Algorithm 2 on
them: drop y = 0, theta = -y1/y2, L_i = [y2 <= 0], S1 = sum L, S0 = min(S1,
m - S1), sort theta ascending and update S1 after every element, M_min the
smallest S0 seen; the bivariate count is M_min + n - m; the result is
N_min - (p-2).  In general position this equals the exact count; on
degenerate data it can differ (in-span points, tie runs), which the tests use
to show that the pins can detect such a slip.
"""
from __future__ import annotations

import itertools

import numpy as np


def depth_literal(X, z) -> int:
    X = np.asarray(X, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64).reshape(-1)
    x = X - z
    n, p = x.shape
    if p < 3:
        raise ValueError("the literal algorithm is stated for p >= 3")
    nmin = n
    for I in itertools.combinations(range(n), p - 2):
        A = x[list(I)].T
        Q, _ = np.linalg.qr(A, mode="complete")
        E = Q[:, p - 2:]
        y = x @ E
        keep = ~np.all(y == 0.0, axis=1)
        yt = y[keep]
        m = yt.shape[0]
        with np.errstate(divide="ignore", invalid="ignore"):
            theta = -yt[:, 0] / yt[:, 1]
        L = (yt[:, 1] <= 0).astype(int)
        S1 = int(L.sum())
        Mmin = min(S1, m - S1)
        for j in np.argsort(theta, kind="stable"):
            S1 = S1 + 1 if L[j] == 0 else S1 - 1
            Mmin = min(Mmin, S1, m - S1)
        nmin = min(nmin, Mmin + n - m)
    return int(nmin - (p - 2))
