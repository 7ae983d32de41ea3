"""Host checks of the seeded stand-ins for the every-observation workload: the
same draw for the same seed, the slicing the paper uses for smaller p and n,
the stated rounding, and argument errors."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("kind,rows,step", [("scores", 64, 1e-2), ("returns", 500, 1e-6)])
def test_observations(kind, rows, step):
    X4, Z4 = workloads.observations(kind, 4, rows)
    again, _ = workloads.observations(kind, 4, rows)
    assert X4.shape == (rows, 4) and X4.dtype == np.float64 and X4.flags.c_contiguous
    assert np.array_equal(X4, again)
    assert np.array_equal(Z4, X4) and Z4 is not X4
    # p = 3 takes the first three columns, a smaller n the first rows
    X3, _ = workloads.observations(kind, 3, rows)
    assert np.array_equal(X3, X4[:, :3])
    Xs, _ = workloads.observations(kind, 4, rows // 2)
    assert np.array_equal(Xs, X4[:rows // 2])
    # rounded to the stated step
    k = X4 / step
    assert np.max(np.abs(k - np.round(k))) < 1e-6
    assert len(np.unique(X4, axis=0)) > rows * 0.9


def test_observations_arguments():
    with pytest.raises(ValueError):
        workloads.observations("scores", 4, 65)
    with pytest.raises(ValueError):
        workloads.observations("returns", 5, 100)
    with pytest.raises(KeyError):
        workloads.observations("other", 3, 10)
