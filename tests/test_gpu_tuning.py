"""The autotuner's cache outside the process (td_tuning_save / td_tuning_load):
a saved file loads back into an emptied cache and saves again unchanged,
calls keep exact counts with the loaded shapes, and malformed or foreign
files are refused without touching the cache."""
import numpy as np
import pytest

import oracle
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _rows(path):
    lines = path.read_text().splitlines()
    return lines[:2], sorted(lines[2:])


def test_tuning_round_trip(td, dev, tmp_path):
    td.autotune(5, 300)
    td.autotune(3, 100)
    a = tmp_path / "a.txt"
    td.tuning_save(str(a))
    head, rows = _rows(a)
    assert head[0] == "td-tuning 1" and head[1].startswith("num_cu ")
    assert len(rows) >= 2
    td.release()                      # the cache goes with the device contexts
    e = tmp_path / "empty.txt"
    td.tuning_save(str(e))
    assert _rows(e)[1] == []
    td.tuning_load(str(a))
    b = tmp_path / "b.txt"
    td.tuning_save(str(b))
    assert _rows(b) == (head, rows)
    rng = np.random.default_rng(77)
    X = rng.standard_normal((300, 5))
    Z = 0.3 * rng.standard_normal((3, 5))
    got = td.depth(to_dev(X, dev), to_dev(Z, dev)).cpu().numpy()
    assert np.array_equal(got, oracle.depth_counts(X, Z))


def test_tuning_load_refuses_bad_files(td, dev, tmp_path):
    td.autotune(4, 120)
    a = tmp_path / "a.txt"
    td.tuning_save(str(a))
    head, rows = _rows(a)
    ncu = int(head[1].split()[1])
    cases = {
        "missing": None,
        "header": "tuning 1\nnum_cu %d\n" % ncu,
        "chunk": "td-tuning 1\nnum_cu %d\n3 4 8 100 64\n" % ncu,       # not a multiple of 64
        "width": "td-tuning 1\nnum_cu %d\n3 4 9 256 64\n" % ncu,       # no such kernel
        "short": "td-tuning 1\nnum_cu %d\n3 4 8 256\n" % ncu,
    }
    for name, text in cases.items():
        f = tmp_path / (name + ".txt")
        if text is not None:
            f.write_text(text)
        with pytest.raises(td.TDError) as e:
            td.tuning_load(str(f))
        assert e.value.code == 1, name
    other = tmp_path / "other.txt"
    other.write_text("td-tuning 1\nnum_cu %d\n3 4 8 256 64\n" % (ncu + 1))
    with pytest.raises(td.TDError) as e:
        td.tuning_load(str(other))
    assert e.value.code == 2
    # nothing of the refused files reached the cache
    b = tmp_path / "b.txt"
    td.tuning_save(str(b))
    assert _rows(b) == (head, rows)
