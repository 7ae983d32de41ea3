"""The vertex-form arithmetic of the device check (td_vertex.hpp), run on the
CPU through tests/vertex_check.hip (no GPU needed):

* exact mode: cofactors within the stated bound of 128-bit integer
  cofactors, every certified side equal to the exact sign, points on the
  hyperplane undecided;
* count mode: the vertex count (Proposition 1 with r = p - 1, every
  (p-1)-subset) equals the oracle's depth on data in general position, and
  on lattice data either equals it or declines (-1), never another value.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("vertex") / "vertex_check")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950",
                           os.path.join(HERE, "vertex_check.hip"), "-o", out])
    return out


def counts(exe, X, Z, tmp_path):
    f = tmp_path / "prob.txt"
    n, p = X.shape
    with open(f, "w") as fh:
        fh.write("%d %d %d\n" % (n, p, Z.shape[0]))
        for row in np.vstack([X, Z]):
            fh.write(" ".join(repr(float(v)) for v in row) + "\n")
    r = subprocess.run([exe, "count", str(f)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    return np.array([int(v) for v in r.stdout.split()])


def test_exact_arithmetic(exe):
    r = subprocess.run([exe, "self"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout
    assert r.stdout.startswith("ok ")
    assert int(r.stdout.split()[1]) > 30000


@pytest.mark.parametrize("p,n", [(2, 30), (3, 25), (4, 18), (5, 14), (6, 12)])
def test_general_position_equals_oracle(exe, tmp_path, p, n):
    rng = np.random.default_rng(100 + p)
    X = rng.standard_normal((n, p))
    Z = np.vstack([0.3 * rng.standard_normal((3, p)), X[:2]])
    got = counts(exe, X, Z, tmp_path)
    exp = oracle.depth_counts(X, Z)
    assert np.array_equal(got, exp), (got, exp)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_lattice_declines_or_agrees(exe, tmp_path, p):
    rng = np.random.default_rng(200 + p)
    X, Z = workloads.lattice_small(rng, p, 14)
    got = counts(exe, X, Z, tmp_path)
    exp = oracle.depth_counts(X, Z)
    assert np.all((got == exp) | (got == -1)), (got, exp)
    assert np.any(got == -1)   # lattice points lie on common hyperplanes
