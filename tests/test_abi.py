"""The C-ABI library loads and exports every entry point declared in include/sssp.h (no GPU needed),
and host-side argument validation rejects malformed input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "sssp.h")).read()
    return sorted(set(re.findall(r"\b(sssp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1903_12085_amd import binding
    lib = binding.load()
    names = declared_symbols()
    assert "sssp_solve" in names and "sssp_solve_batch" in names and "sssp_delta_step" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(binding.SYMBOLS) <= set(names)


def _create(n, m, rp, col, w):
    from paper_1903_12085_amd import binding
    lib = binding.load()
    h = ctypes.c_void_p()
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    rc = lib.sssp_graph_create(n, m, P(rp), P(col), P(w), 0, None, ctypes.byref(h))
    return rc, lib.sssp_last_error().decode()


@pytest.mark.parametrize("case", ["n0", "rp0", "rpn", "nonmono", "colrange", "toolarge"])
def test_graph_create_rejects_malformed_csr(case):
    rp = np.array([0, 2, 3, 3], np.uint64)
    col = np.array([1, 2, 0], np.uint32)
    w = np.array([1, 2, 3], np.uint32)
    n, m = 3, 3
    if case == "n0":
        n = 0
    elif case == "rp0":
        rp = np.array([1, 2, 3, 3], np.uint64)
    elif case == "rpn":
        m = 2
    elif case == "nonmono":
        rp = np.array([0, 2, 1, 3], np.uint64)
    elif case == "colrange":
        col = np.array([1, 3, 0], np.uint32)
    elif case == "toolarge":
        n = 1 << 26
    rc, msg = _create(n, m, rp, col, w)
    assert rc == (-4 if case == "toolarge" else -1), (case, rc, msg)
    assert msg


def test_null_arguments_rejected():
    from paper_1903_12085_amd import binding
    lib = binding.load()
    assert lib.sssp_graph_create(3, 0, None, None, None, 0, None, None) == -1
    assert lib.sssp_solve(None, 0, 2, None, None) == -1
    assert lib.sssp_solve_batch(None, None, 0, 2, None, None) == -1
    assert lib.sssp_graph_destroy(None) == 0
