"""The C-ABI library loads and exports every entry point include/md.h declares,
and host-side argument validation rejects bad calls before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1305_4196_amd import binding
    path = binding.LIB_PATH
    if not os.path.exists(path):
        from paper_1305_4196_amd import build
        build.build()
    return binding.load()


def test_header_declares_the_five_hot_path_calls():
    names = declared()
    for n in ("md_build_cells", "md_build_neighbor_list", "md_compute_forces", "md_verlet_step",
              "md_force_vjp"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1305_4196_amd import binding
    names = declared()
    assert set(names) == set(binding.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_create_rejects_bad_arguments_on_host(lib):
    h = C.c_void_p()
    off = np.array([0, 10], dtype=np.int64)
    P = C.POINTER(C.c_int64)
    assert lib.md_create(C.byref(h), 0, 1, off.ctypes.data_as(P)) == -1
    assert lib.md_create(C.byref(h), 10, 0, off.ctypes.data_as(P)) == -1
    bad = np.array([0, 4, 4, 10], dtype=np.int64)       # empty replica
    assert lib.md_create(C.byref(h), 10, 3, bad.ctypes.data_as(P)) == -1
    bad = np.array([0, 9], dtype=np.int64)              # does not end at n
    assert lib.md_create(C.byref(h), 10, 1, bad.ctypes.data_as(P)) == -1
    assert lib.md_create(C.byref(h), (1 << 26) + 1, 1,
                         np.array([0, (1 << 26) + 1], dtype=np.int64).ctypes.data_as(P)) == -1
    assert lib.md_create(None, 10, 1, off.ctypes.data_as(P)) == -1


def test_null_context_is_rejected(lib):
    assert lib.md_build_cells(None, None, None, 2.5, 0.3, None) == -1
    assert lib.md_build_neighbor_list(None, 0, None) == -1
    assert lib.md_set_tuning(None, 0, 8) == -1
    assert lib.md_get_waves(None, None, 0, None) == -1
    assert lib.md_get_task_graph(None, None, None, 0) == -1
    assert lib.md_last_error(None) == b"null context"


def test_package_import_loads_nothing():
    import importlib
    import sys
    for m in [m for m in sys.modules if m.startswith("paper_1305_4196_amd")]:
        del sys.modules[m]
    pkg = importlib.import_module("paper_1305_4196_amd")
    assert pkg.__name__ == "paper_1305_4196_amd"
    assert "paper_1305_4196_amd.binding" not in sys.modules
