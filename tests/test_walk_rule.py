"""The bucketed sweep's walk over the points gathered in exact order
(Algorithm 2, Step 1(e), on the runs of buckets whose states may dip below
the bound), in its two forms: the one-lane walk of the float64 pass, which
takes the clusters in turn with the running minimum of the states after
them, and the first pass's parallel form, which decides every cluster at
once against the minimum of all those states.  The states after a cluster
do not depend on the order inside it, so that minimum is a valid bound for
every cluster, and no lower than the running one: wherever the one-lane
walk settles a sweep, the parallel form must return the same value, and it
may settle more sweeps (a cluster with both fold signs whose states cannot
go below min(U, ubound, best) needs no inner order).  This file models both
on the CPU over random gathered lists."""
import random

KBIG = 0x7FFFFFFF
KCLUSTER = 64


def fside(s, m):
    return min(s, m - s)


def one_lane(entries, m, U, ub):
    """entries: (lo, hi, negative fold, run, state at the run's left end),
    sorted by lo with the runs contiguous and increasing."""
    best = KBIG
    k, g = 0, len(entries)
    while k < g:
        run, s, a = entries[k][3], entries[k][4], k
        while a < g and entries[a][3] == run:
            mhi = entries[a][1]
            npos = 0 if entries[a][2] else 1
            b = a
            while b + 1 < g and entries[b + 1][3] == run and entries[b + 1][0] <= mhi:
                b += 1
                mhi = max(mhi, entries[b][1])
                npos += 0 if entries[b][2] else 1
            c = b - a + 1
            mixed = 0 < npos < c
            dip = min(s - npos, m - (s + (c - npos)))
            if mixed and dip < min(min(U, ub), best):
                return "defer" if c > KCLUSTER else "need64"
            s += c - 2 * npos
            best = min(best, fside(s, m))
            a = b + 1
        k = a
    return min(U, best)


def parallel(entries, m, U, ub):
    g = len(entries)
    start, maxhi = [], {}
    for e, (lo, hi, _, run, _) in enumerate(entries):
        start.append(e == 0 or entries[e - 1][3] != run or lo > maxhi[run])
        maxhi[run] = max(maxhi.get(run, -1), hi)
    send, cnt, npos = [], [], []
    runsum, c, n = {}, 0, 0
    for e, (_, _, neg, run, srun) in enumerate(entries):
        runsum[run] = runsum.get(run, 0) + (1 if neg else -1)
        if start[e]:
            c = n = 0
        c += 1
        n += 0 if neg else 1
        send.append(srun + runsum[run])
        cnt.append(c)
        npos.append(n)
    end = [e == g - 1 or start[e + 1] for e in range(g)]
    best = min([fside(send[e], m) for e in range(g) if end[e]] + [KBIG])
    bound = min(min(U, ub), best)
    need = big = False
    for e in range(g):
        if not end[e] or npos[e] in (0, cnt[e]):
            continue
        s0 = send[e] - (cnt[e] - 2 * npos[e])
        if min(s0 - npos[e], m - (s0 + (cnt[e] - npos[e]))) < bound:
            need = True
            big = big or cnt[e] > KCLUSTER
    if big:
        return "defer"
    if need:
        return "need64"
    return min(U, best)


def _case(rng):
    m = rng.randint(5, 60)
    entries, x = [], 0
    for r in range(rng.randint(1, 4)):
        run = 3 * r + rng.randint(0, 2)
        srun = rng.randint(0, m)
        for _ in range(rng.randint(1, 8)):
            x += rng.randint(0, 3)
            entries.append((x, x + rng.randint(0, 4), rng.random() < 0.5, run, srun))
        x += 10
    return entries, m, rng.randint(0, m), rng.randint(0, m + 5)


def test_parallel_walk_equals_one_lane_walk_where_it_settles():
    rng = random.Random(11)
    settled = extra = 0
    for _ in range(30000):
        entries, m, U, ub = _case(rng)
        a, b = one_lane(entries, m, U, ub), parallel(entries, m, U, ub)
        if isinstance(a, int):
            assert b == a, (entries, m, U, ub, a, b)
            settled += 1
        elif b != a:
            extra += 1
    assert settled > 5000 and extra > 0


def test_parallel_walk_single_sign_runs_are_exact():
    """Runs whose clusters all have one fold sign: both forms give the
    minimum over the states after the clusters."""
    rng = random.Random(12)
    for _ in range(2000):
        entries, m, U, ub = _case(rng)
        entries = [(lo, hi, True, run, s) for lo, hi, _, run, s in entries]
        a, b = one_lane(entries, m, U, ub), parallel(entries, m, U, ub)
        assert a == b and isinstance(a, int)
