"""The C ABI library loads and exports every entry point of include/td.h, and
rejects invalid arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "td.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(td_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1409_3901_amd as td
    return td.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert "td_depth" in names and "td_depth_batched" in names
    import paper_1409_3901_amd as td
    assert sorted(td.SYMBOLS) == names
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures have the size and field offsets of the
    C structures (tests/abi_layout.c compiled against include/td.h)."""
    import subprocess
    import paper_1409_3901_amd as td
    exe = str(tmp_path / "abi_layout")
    subprocess.check_call(["gcc", "-std=c99", "-O0", os.path.join(ROOT, "tests", "abi_layout.c"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    c = dict(line.split() for line in out if line.strip())
    for cname, py in (("td_options", td.Options), ("td_stats", td.Stats), ("td_problem", td.Problem)):
        assert int(c[cname]) == ctypes.sizeof(py), cname
        names = [f for f, _ in py._fields_]
        cfields = [k.split(".", 1)[1] for k in c if k.startswith(cname + ".")]
        assert cfields == names, (cname, cfields, names)
        for f in names:
            assert int(c["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


def test_status_strings_and_version(lib):
    for code in range(8):
        assert lib.td_status_string(code)
    assert lib.td_version() >= 1


def test_invalid_arguments_rejected_without_device(lib):
    import paper_1409_3901_amd as td
    o = td.Options()
    assert lib.td_default_options(ctypes.byref(o)) == 0
    assert o.precision == 1 and o.filter_scale == 1.0 and o.prune == 1 and o.sweep == 0
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    # null pointers
    assert lib.td_depth(nul, 10, 3, fake, 2, fake, nul) == 1
    # p out of range, n out of range, m < 0
    assert lib.td_depth(fake, 10, 0, fake, 2, fake, nul) == 1
    assert lib.td_depth(fake, 10, 9, fake, 2, fake, nul) == 1
    assert lib.td_depth(fake, 0, 3, fake, 2, fake, nul) == 1
    assert lib.td_depth(fake, 1025, 3, fake, 2, fake, nul) == 1
    assert lib.td_depth(fake, 10, 3, fake, -1, fake, nul) == 1
    # m = 0 is a no-op
    assert lib.td_depth(fake, 10, 3, fake, 0, fake, nul) == 0
    # the tuning file calls reject a null path, and a missing or malformed
    # file, before touching a device
    assert lib.td_tuning_save(None) == 1
    assert lib.td_tuning_load(None) == 1
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        assert lib.td_tuning_load(os.path.join(d, "missing.txt").encode()) == 1
        for text in ("tuning 1\nnum_cu 256\n", "td-tuning 1\nnum_cu 256\n3 4 8 100 64\n",
                     "td-tuning 1\nnum_cu 256\n3 4 9 256 64\n", "td-tuning 2\nnum_cu 256\n"):
            f = os.path.join(d, "bad.txt")
            with open(f, "w") as fh:
                fh.write(text)
            assert lib.td_tuning_load(f.encode()) == 1, text
    # bad options
    bad = td.Options()
    lib.td_default_options(ctypes.byref(bad))
    bad.chunk = 100
    assert lib.td_depth_ex(fake, 10, 3, fake, 2, fake, ctypes.byref(bad), nul) == 1
    bad.chunk = 0
    bad.filter_scale = float("nan")
    assert lib.td_depth_ex(fake, 10, 3, fake, 2, fake, ctypes.byref(bad), nul) == 1
    bad.filter_scale = 1.0
    bad.precision = 7
    assert lib.td_depth_ex(fake, 10, 3, fake, 2, fake, ctypes.byref(bad), nul) == 1
    bad.precision = 1
    bad.sweep = 2
    assert lib.td_depth_ex(fake, 10, 3, fake, 2, fake, ctypes.byref(bad), nul) == 1
    bad.sweep = 0
    bad.prune = 2
    assert lib.td_depth_ex(fake, 10, 3, fake, 2, fake, ctypes.byref(bad), nul) == 1
    # batched: null array / negative count
    assert lib.td_depth_batched(None, 1, None, nul) == 1
    assert lib.td_depth_batched(None, 0, None, nul) == 0
