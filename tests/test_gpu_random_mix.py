"""Every method and tier on one seeded mix of small problems (p = 2..6, in
general position and not: Gaussian, uniform cube, lattice, duplicated rows,
ray-duplicated and near-degenerate sets), each against the oracle:

* RCom: the bucketed and bitonic filtered tiers, the exact precision, and all
  problems in one batched call, equal the oracle;
* ADIA: never below the oracle, equal to it where it is exact;
* the vertex check: equal to the oracle or declined with TD_DEV_NOT_GENERAL
  (or TD_DEV_NO_VALID_SUBSET when fewer than p - 1 points differ from z)."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _problems():
    rng = np.random.default_rng(2026)
    out = []
    for t in range(30):
        p = int(rng.integers(2, 7))
        nmax = {2: 90, 3: 80, 4: 50, 5: 30, 6: 22}[p]
        n = int(rng.integers(p + 3, nmax + 1))
        kind = t % 6
        if kind == 0:
            X = rng.standard_normal((n, p))
        elif kind == 1:
            X = rng.uniform(-1.0, 1.0, size=(n, p))
        elif kind == 2:
            X, _ = workloads.lattice_small(rng, p, n, R=2)
        elif kind == 3:
            if p == 6:
                n = min(n, 12)    # duplicated rows make many degenerate subsets for the oracle
            X = rng.standard_normal((max(p + 1, n // 2), p))
            X = np.vstack([X, X[: n - X.shape[0]]])          # duplicated rows
        elif kind == 4:
            X, _ = workloads.ray_duplicated(rng, p, max(p + 1, n // 2))
        else:
            X, _ = workloads.near_degenerate(rng, p, n)
        Z = np.vstack([0.3 * rng.standard_normal((2, p)), X[rng.integers(0, X.shape[0], size=2)],
                       rng.integers(-1, 2, size=(1, p)).astype(np.float64)])
        out.append((np.ascontiguousarray(X, dtype=np.float64), np.ascontiguousarray(Z, dtype=np.float64)))
    return out


PROBLEMS = _problems()


def test_rcom_tiers_and_batched(td, dev):
    exps = [oracle.depth_counts(X, Z) for X, Z in PROBLEMS]
    for i, ((X, Z), exp) in enumerate(zip(PROBLEMS, exps)):
        for opts in (dict(), dict(sweep="bitonic"), dict(precision="exact"), dict(prune=False)):
            got = td.depth(to_dev(X, dev), to_dev(Z, dev), **opts).cpu().numpy()
            assert np.array_equal(got, exp), (i, X.shape, opts, got, exp)
    outs = td.depth_batched([(to_dev(X, dev), to_dev(Z, dev)) for X, Z in PROBLEMS])
    for i, (o, exp) in enumerate(zip(outs, exps)):
        assert np.array_equal(o.cpu().numpy(), exp), (i, o, exp)


def test_adia_and_vertex(td, dev):
    for i, (X, Z) in enumerate(PROBLEMS):
        exp = oracle.depth_counts(X, Z)
        a = td.depth(to_dev(X, dev), to_dev(Z, dev), method="adia").cpu().numpy()
        assert np.all(a >= exp), (i, a, exp)
        av, _ = oracle.depth_adia(X, Z)
        assert np.array_equal(a, av), (i, a, av)
        v = td.depth(to_dev(X, dev), to_dev(Z, dev), method="vertex").cpu().numpy()
        st = td.get_stats()
        assert np.all((v == exp) | (v == -1)), (i, v, exp)
        if np.any(v == -1):
            assert {"not_general", "no_valid_subset"} & set(st["device_status_bits"]), st
