"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments on the host side before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsbfs.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dsbfs_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    from paper_1803_03922_amd import dsbfs
    lib = ctypes.CDLL(dsbfs.LIB_PATH)
    names = _declared()
    assert len(names) == 24
    for name in names:
        assert hasattr(lib, name), name
    # and the binding wraps every one of them under the same name
    for name in names:
        assert name in dsbfs.EXPORTED, name


def test_status_strings():
    from paper_1803_03922_amd import dsbfs
    assert dsbfs.dsbfs_status_str(0) == b"ok"
    assert dsbfs.dsbfs_status_str(dsbfs.ERR_BUDGET) == b"HBM budget exhausted"
    assert dsbfs.dsbfs_status_str(-99) == b"unknown status"


def test_default_factors():
    """Defaults are the factors tuned for this layout, in dd, dn, nd order;
    the header also carries the paper's (Section VI-B) as named constants."""
    from paper_1803_03922_amd import dsbfs
    o = dsbfs.dsbfs_run_opts()
    assert dsbfs.dsbfs_run_opts_default(ctypes.byref(o)) == 0
    assert list(o.factor0) == [0.02, 0.001, 1e-6]
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "dsbfs.h")).read()
    paper = {k: float(v) for k, v in re.findall(r"#define DSBFS_PAPER_FACTOR0_(\w+) (\S+)", hdr)}
    assert paper == {"DD": 0.5, "DN": 0.05, "ND": 1e-7}
    assert list(o.factor1) == [0.0, 0.0, 0.0]
    assert o.mode == 1 and o.want_parent == 1 and o.forced == 0
    # nn stays forward unless the DO-on-nn variant is asked for
    assert o.nn_do == 0 and o.factor0_nn == 1e-3 and o.factor1_nn == 0.0


def test_host_side_argument_errors():
    from paper_1803_03922_amd import dsbfs
    h = ctypes.c_void_p()
    st = dsbfs.dsbfs_graph_create(None, None, 0, 0, None, None, None, ctypes.byref(h))
    assert st == dsbfs.ERR_INVALID_ARG
    assert b"num_vertices" in dsbfs.dsbfs_last_error()
    st = dsbfs.dsbfs_graph_create(None, None, 5, 10, None, None, None, ctypes.byref(h))
    assert st == dsbfs.ERR_INVALID_ARG
    bo = dsbfs.dsbfs_build_opts(-1, 0, 1, 0)
    st = dsbfs.dsbfs_graph_create(None, None, 0, 10, ctypes.byref(bo), None, None, ctypes.byref(h))
    assert st == dsbfs.ERR_INVALID_ARG and b"threshold" in dsbfs.dsbfs_last_error()
    bo = dsbfs.dsbfs_build_opts(32, 0, 1, 2)
    st = dsbfs.dsbfs_graph_create(None, None, 0, 10, ctypes.byref(bo), None, None, ctypes.byref(h))
    assert st == dsbfs.ERR_INVALID_ARG and b"skip_nn_copy" in dsbfs.dsbfs_last_error()
    assert dsbfs.dsbfs_graph_create(None, None, 0, 1, None, None, None, None) == dsbfs.ERR_INVALID_ARG
    assert dsbfs.dsbfs_bfs(None, None, 0, None, None, None, None, None) == dsbfs.ERR_INVALID_ARG
    assert dsbfs.dsbfs_bfs_noalloc(None, 0, None, None, None, None, None) == dsbfs.ERR_INVALID_ARG
    assert dsbfs.dsbfs_graph_destroy(None) == 0
    assert dsbfs.dsbfs_workspace_destroy(None) == 0
    assert dsbfs.dsbfs_server_destroy(None) == 0
    assert dsbfs.dsbfs_server_create(None, None, None) == dsbfs.ERR_INVALID_ARG
    assert dsbfs.dsbfs_server_stats_get(None, None) == dsbfs.ERR_INVALID_ARG
    assert dsbfs.dsbfs_graph_create_rmat(None, None, None, None, None) == dsbfs.ERR_INVALID_ARG
    assert dsbfs.dsbfs_pagerank(None, 0.85, 1, 0.0, None, None, None, None) == dsbfs.ERR_INVALID_ARG
    sp = dsbfs.rmat_spec(40)
    assert dsbfs.dsbfs_rmat_generate(ctypes.byref(sp), None, None, None) == dsbfs.ERR_INVALID_ARG
    sp = dsbfs.rmat_spec(10, a=0.7, b=0.3, c=0.3)
    assert dsbfs.dsbfs_rmat_generate(ctypes.byref(sp), None, None, None) == dsbfs.ERR_INVALID_ARG


def test_now_is_monotonic():
    from paper_1803_03922_amd import dsbfs
    a = dsbfs.now_ns()
    b = dsbfs.now_ns()
    assert 0 < a <= b
