"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects malformed input before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(daic_\w+)\s*\(", src, re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_1710_05785_amd import daic

    return daic.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("daic_graph_create", "daic_problem_create", "daic_problem_set_init", "daic_run",
                 "daic_problem_get", "daic_last_error", "daic_trace_record", "daic_sched_train",
                 "daic_sched_save", "daic_sched_load", "daic_sched_step", "daic_trace_create",
                 "daic_trace_samples", "daic_problem_set_const", "daic_problem_check_init",
                 "daic_problem_save", "daic_problem_load", "daic_batch_get_state", "daic_batch_save",
                 "daic_batch_load"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_graph_create_rejects_bad_csr(L):
    from paper_1710_05785_amd import daic

    # row_ptr[n] != m
    with pytest.raises(daic.DaicError, match="row_ptr"):
        daic.Graph(np.array([0, 1, 3], dtype=np.uint64), np.array([1, 0], dtype=np.uint32))
    # not monotone
    with pytest.raises(daic.DaicError, match="monotone"):
        daic.Graph(np.array([0, 2, 1, 2], dtype=np.uint64), np.array([1, 0], dtype=np.uint32))
    # column out of range
    with pytest.raises(daic.DaicError, match="out of range"):
        daic.Graph(np.array([0, 1, 2], dtype=np.uint64), np.array([1, 2], dtype=np.uint32))


def test_problem_create_rejects_null_graph(L):
    from paper_1710_05785_amd import daic

    h = ctypes.c_void_p()
    rc = L.daic_problem_create(None, daic.SUM, daic.G_DEG_SCALE, 0.8, None, daic.F64,
                               ctypes.byref(h))
    assert rc == -1
    assert b"graph" in L.daic_last_error()


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_1710_05785_amd import daic

    monkeypatch.setattr(daic, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(daic, "_lib", None)
    with pytest.raises(daic.DaicError, match="no CPU fallback"):
        daic.lib()
