"""The grouping rule the filtered and exact tiers use to find states of the
circular sweep among uncertain keys (Algorithm 2, Step 1(e), with keys known
only up to an interval).

Every swept point carries an interval [lo, hi] that holds its exact angular
position.  The kernels sort the points by the interval's lower end; a point
whose lower end exceeds every earlier upper end starts a new cluster, and the
boundary before it is a state of the sweep.  A cluster whose points all have
one fold sign contributes only its end state (every inner order reaches it);
a cluster holding both signs is put in exact order and grouped by equal
positions.  This file models that procedure on the CPU and checks it against
the sweep over the exact positions.  It also shows why the order matters:
with the intervals ordered by their centres, a later and wider interval can
reach below a boundary taken as a gap, and the count comes out too high or
too low (the fixed cases below).
"""
import numpy as np


def clusters(lo, hi, order):
    out = []
    pm = -np.inf
    for e in order:
        if not out or lo[e] > pm:
            out.append([])
        out[-1].append(e)
        pm = max(pm, hi[e])
    return out


def kernel_min(lo, hi, pos, sign, order, m):
    """min(S, m - S) over the states the procedure visits.  S starts at the
    number of points folded with sign -1 and moves by each point's sign."""
    S = int(np.sum(sign < 0))
    best = min(S, m - S)
    for c in clusters(lo, hi, list(order)):
        if len(set(sign[c].tolist())) == 1:
            S += int(np.sum(sign[c]))
            best = min(best, S, m - S)
        else:
            cc = sorted(c, key=lambda e: pos[e])
            for i, e in enumerate(cc):
                S += int(sign[e])
                if i + 1 == len(cc) or pos[cc[i + 1]] != pos[e]:
                    best = min(best, S, m - S)
    return best


def exact_min(pos, sign, m):
    """The sweep over exact positions, states between distinct positions."""
    order = np.argsort(pos, kind="stable")
    S = int(np.sum(sign < 0))
    best = min(S, m - S)
    for k, e in enumerate(order):
        S += int(sign[e])
        if k + 1 == len(order) or pos[order[k + 1]] != pos[e]:
            best = min(best, S, m - S)
    return best


def by_lower(lo, hi):
    return np.argsort(lo, kind="stable")


def by_centre(lo, hi):
    return np.argsort((lo + hi) / 2, kind="stable")


CASES = [
    # (lo, hi, exact position, sign): centre order over- and under-counts
    ([-12.07, 9.46, 6.87, 3.21, -8.83, 1.8], [5.92, 18.13, 7.45, 8.88, 6.52, 29.77],
     [3.0, 11.0, 7.0, 7.5, 2.0, 3.0], [1, -1, -1, -1, 1, 1]),
    ([12.74, 25.86, 23.48, 16.03], [41.2, 27.36, 23.69, 22.1],
     [14.5, 27.0, 23.5, 17.0], [-1, -1, -1, 1]),
]


def test_fixed_cases():
    for lo, hi, pos, sign in CASES:
        lo, hi, pos, sign = map(np.asarray, (lo, hi, pos, sign))
        assert np.all(lo <= pos) and np.all(pos <= hi)
        m = len(pos)
        e = exact_min(pos, sign, m)
        assert kernel_min(lo, hi, pos, sign, by_lower(lo, hi), m) == e
        assert kernel_min(lo, hi, pos, sign, by_centre(lo, hi), m) != e


def test_lower_end_order_with_mixed_radii():
    rng = np.random.default_rng(7)
    wrong_centre = 0
    for _ in range(20000):
        m = int(rng.integers(2, 10))
        pos = rng.integers(0, 30, size=m).astype(float) + rng.choice([0.0, 0.5], size=m)
        # radii over two orders of magnitude, as float32 keys next to float64
        # re-checks give
        rad = 10.0 ** rng.uniform(-1.0, 1.3, size=m)
        off = rng.uniform(-1.0, 1.0, size=m) * rad
        lo, hi = pos + off - rad, pos + off + rad
        sign = rng.choice([-1, 1], size=m)
        e = exact_min(pos, sign, m)
        assert kernel_min(lo, hi, pos, sign, by_lower(lo, hi), m) == e
        wrong_centre += kernel_min(lo, hi, pos, sign, by_centre(lo, hi), m) != e
    assert wrong_centre > 0


def test_equal_radii_orders_agree():
    """With one radius for every point the two orders coincide: the defect
    needs radii that differ."""
    rng = np.random.default_rng(8)
    for _ in range(2000):
        m = int(rng.integers(2, 10))
        pos = rng.integers(0, 20, size=m).astype(float)
        r = 1.5
        off = rng.uniform(-1, 1, size=m) * r
        lo, hi = pos + off - r, pos + off + r
        sign = rng.choice([-1, 1], size=m)
        e = exact_min(pos, sign, m)
        assert kernel_min(lo, hi, pos, sign, by_centre(lo, hi), m) == e
        assert kernel_min(lo, hi, pos, sign, by_lower(lo, hi), m) == e
