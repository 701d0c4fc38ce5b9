"""CPU oracle for degree-separated direction-optimized BFS (ctypes binding).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library or its
binding. The arithmetic lives in ``oracle.c``; this file only marshals numpy
arrays. See oracle.c for the paper passage each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
F64P = ctypes.POINTER(ctypes.c_double)


class SplitStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("n", "m", "d", "e_nn", "e_nd", "e_dn", "e_dd", "n_ndsrc", "n_ddsrc",
                 "n_dnsrc", "max_deg")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Level(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int64 * 3), ("s", ctypes.c_int64 * 3), ("U", ctypes.c_int64 * 3),
                ("FV", ctypes.c_int64 * 3), ("BV", ctypes.c_double * 3),
                ("dir", ctypes.c_int32 * 3), ("FV_nn", ctypes.c_int64), ("q_nn", ctypes.c_int64),
                ("frontier_normal", ctypes.c_int64), ("frontier_delegate", ctypes.c_int64)]

    def as_dict(self):
        return {"q": list(self.q), "s": list(self.s), "U": list(self.U), "FV": list(self.FV),
                "BV": list(self.BV), "dir": list(self.dir), "FV_nn": int(self.FV_nn),
                "q_nn": int(self.q_nn), "frontier_normal": int(self.frontier_normal),
                "frontier_delegate": int(self.frontier_delegate)}


class Level4(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int64 * 4), ("s", ctypes.c_int64 * 4), ("U", ctypes.c_int64 * 4),
                ("FV", ctypes.c_int64 * 4), ("BV", ctypes.c_double * 4),
                ("dir", ctypes.c_int32 * 4), ("frontier_normal", ctypes.c_int64),
                ("frontier_delegate", ctypes.c_int64)]

    def as_dict(self):
        return {"q": list(self.q), "s": list(self.s), "U": list(self.U), "FV": list(self.FV),
                "BV": list(self.BV), "dir": list(self.dir),
                "frontier_normal": int(self.frontier_normal),
                "frontier_delegate": int(self.frontier_delegate)}


class WorkLevel(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int64 * 3), ("s", ctypes.c_int64 * 3), ("U", ctypes.c_int64 * 3),
                ("FV", ctypes.c_int64 * 3), ("BV", ctypes.c_double * 3),
                ("dir", ctypes.c_int32 * 3), ("runs", ctypes.c_int32 * 5)] + \
               [(k, ctypes.c_int64) for k in
                ("f_norm", "f_deleg", "e_nn", "e_nd", "e_dd", "e_dn", "c_dn", "e_bu_dn", "c_dd",
                 "e_bu_dd", "c_nd", "e_bu_nd", "c_deleg", "s_dn", "s_dd", "s_nd", "cl_nn", "cl_nd",
                 "cl_dd", "cl_dn", "cl_bu_dn", "cl_bu_deleg")]

    def as_dict(self):
        out = {}
        for k, t in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if hasattr(v, "__len__") else int(v)
        return out


class MsLevel(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int64), ("e", ctypes.c_int64), ("v", ctypes.c_int64),
                ("bottom_up", ctypes.c_int32), ("pad", ctypes.c_int32)]


# Visits of or_work_bytes, in its order.
WORK_VISITS = ("init", "normal_frontier", "delegate_previsit", "nd_forward", "deleg_forward",
               "dn_backward", "deleg_backward")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP for the CSR build only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-o", tmp, os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        vp = ctypes.c_void_p
        L.or_graph_build.restype = ctypes.c_int
        L.or_graph_build.argtypes = [I32P, I32P, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.POINTER(vp)]
        L.or_graph_free.argtypes = [vp]
        L.or_graph_n.restype = ctypes.c_int32
        L.or_graph_n.argtypes = [vp]
        L.or_graph_m.restype = ctypes.c_int64
        L.or_graph_m.argtypes = [vp]
        L.or_graph_off.restype = I64P
        L.or_graph_off.argtypes = [vp]
        L.or_graph_col.restype = I32P
        L.or_graph_col.argtypes = [vp]
        L.or_bfs.restype = ctypes.c_int
        L.or_bfs.argtypes = [vp, ctypes.c_int32, I32P, I32P]
        L.or_apsp.restype = ctypes.c_int
        L.or_apsp.argtypes = [ctypes.c_int32, I32P, I32P, ctypes.c_int64, I32P]
        L.or_components.restype = ctypes.c_int
        L.or_components.argtypes = [ctypes.c_int32, I32P, I32P, ctypes.c_int64, I32P]
        L.or_check_bfs.restype = ctypes.c_int
        L.or_check_bfs.argtypes = [vp, ctypes.c_int32, I32P, I32P, I32P, I64P]
        L.or_split_stats.restype = ctypes.c_int
        L.or_split_stats.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(SplitStats)]
        L.or_delegate_ids.restype = ctypes.c_int
        L.or_delegate_ids.argtypes = [vp, ctypes.c_int64, I32P]
        L.or_split_rows.restype = ctypes.c_int
        L.or_split_rows.argtypes = [vp, ctypes.c_int64, I32P] + [I64P, I32P] * 4
        L.or_bv_term.restype = ctypes.c_double
        L.or_bv_term.argtypes = [ctypes.c_double, ctypes.c_int64]
        L.or_bv_approx.restype = ctypes.c_double
        L.or_bv_approx.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.or_do_replay.restype = ctypes.c_int
        L.or_do_replay.argtypes = [vp, ctypes.c_int64, I32P, F64P, F64P, ctypes.c_int,
                                   ctypes.POINTER(Level), ctypes.c_int]
        L.or_do_replay4.restype = ctypes.c_int
        L.or_do_replay4.argtypes = [vp, ctypes.c_int64, I32P, F64P, F64P, ctypes.c_int,
                                    ctypes.POINTER(Level4), ctypes.c_int]
        L.or_pagerank.restype = ctypes.c_int
        L.or_pagerank.argtypes = [vp, ctypes.c_double, ctypes.c_int32, F64P]
        L.or_work_prepare.restype = ctypes.c_int
        L.or_work_prepare.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(vp)]
        L.or_work_free.argtypes = [vp]
        L.or_do_work.restype = ctypes.c_int
        L.or_do_work.argtypes = [vp, I32P, F64P, F64P, ctypes.POINTER(WorkLevel), ctypes.c_int]
        L.or_work_bytes.restype = ctypes.c_int
        L.or_work_bytes.argtypes = [ctypes.POINTER(WorkLevel), ctypes.c_int, ctypes.c_int64,
                                    ctypes.c_int, F64P, I64P]
        L.or_ms_work.restype = ctypes.c_int
        L.or_ms_work.argtypes = [vp, I32P, ctypes.c_int32, ctypes.c_int32, I32P,
                                 ctypes.POINTER(MsLevel), ctypes.c_int, F64P]
        _lib = L
    return _lib


def _i32(a):
    return a.ctypes.data_as(I32P)


def _i64(a):
    return a.ctypes.data_as(I64P)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Graph:
    """The simple symmetric graph of an edge list, as the oracle's own CSR."""

    def __init__(self, src, dst, n: int):
        L = _load()
        self._src, self._dst = _c32(src), _c32(dst)
        h = ctypes.c_void_p()
        rc = L.or_graph_build(_i32(self._src), _i32(self._dst), len(self._src), n,
                              ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"or_graph_build failed ({rc})")
        self._h = h
        self.n = n
        self.m = int(L.or_graph_m(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_graph_free(h)
            self._h = None

    @property
    def off(self) -> np.ndarray:
        return np.ctypeslib.as_array(_load().or_graph_off(self._h), shape=(self.n + 1,)).copy()

    @property
    def col(self) -> np.ndarray:
        if self.m == 0:
            return np.zeros(0, dtype=np.int32)
        return np.ctypeslib.as_array(_load().or_graph_col(self._h), shape=(self.m,)).copy()

    def degrees(self) -> np.ndarray:
        return np.diff(self.off).astype(np.int64)

    def bfs(self, s: int, want_parent: bool = True):
        depth = np.empty(self.n, dtype=np.int32)
        parent = np.empty(self.n, dtype=np.int32) if want_parent else None
        rc = _load().or_bfs(self._h, s, _i32(depth), _i32(parent) if want_parent else None)
        if rc != 0:
            raise ValueError(f"or_bfs failed ({rc})")
        return depth, parent

    def components(self) -> np.ndarray:
        label = np.empty(self.n, dtype=np.int32)
        rc = _load().or_components(self.n, _i32(self._src), _i32(self._dst), len(self._src),
                                   _i32(label))
        if rc != 0:
            raise ValueError(f"or_components failed ({rc})")
        return label

    def check(self, s: int, depth, parent=None, label=None):
        """(code, bad_vertex); code 0 means every invariant holds."""
        depth = _c32(depth)
        parent = None if parent is None else _c32(parent)
        label = None if label is None else _c32(label)
        bad = ctypes.c_int64(-1)
        rc = _load().or_check_bfs(self._h, s, _i32(depth),
                                  _i32(parent) if parent is not None else None,
                                  _i32(label) if label is not None else None, ctypes.byref(bad))
        return int(rc), int(bad.value)

    def split_stats(self, TH: int) -> dict:
        st = SplitStats()
        rc = _load().or_split_stats(self._h, TH, ctypes.byref(st))
        if rc != 0:
            raise ValueError("or_split_stats failed")
        return st.as_dict()

    def delegate_ids(self, TH: int) -> np.ndarray:
        did = np.empty(self.n, dtype=np.int32)
        _load().or_delegate_ids(self._h, TH, _i32(did))
        return did

    def split_rows(self, TH: int) -> dict:
        st = self.split_stats(TH)
        did = self.delegate_ids(TH)
        n, d = self.n, st["d"]
        arrs = {
            "nn_off": np.zeros(n + 1, np.int64), "nn_col": np.zeros(max(st["e_nn"], 1), np.int32),
            "nd_off": np.zeros(n + 1, np.int64), "nd_col": np.zeros(max(st["e_nd"], 1), np.int32),
            "dn_off": np.zeros(d + 1, np.int64), "dn_col": np.zeros(max(st["e_dn"], 1), np.int32),
            "dd_off": np.zeros(d + 1, np.int64), "dd_col": np.zeros(max(st["e_dd"], 1), np.int32),
        }
        args = []
        for k in ("nn", "nd", "dn", "dd"):
            args += [_i64(arrs[k + "_off"]), _i32(arrs[k + "_col"])]
        rc = _load().or_split_rows(self._h, TH, _i32(did), *args)
        if rc != 0:
            raise ValueError("or_split_rows failed")
        for k in ("nn", "nd", "dn", "dd"):
            arrs[k + "_col"] = arrs[k + "_col"][:st["e_" + k]]
        arrs["did"] = did
        return arrs

    def pagerank(self, alpha: float, iterations: int) -> np.ndarray:
        """FP64 power iteration from the uniform vector (or_pagerank)."""
        r = np.empty(self.n, dtype=np.float64)
        rc = _load().or_pagerank(self._h, alpha, iterations, r.ctypes.data_as(F64P))
        if rc != 0:
            raise ValueError(f"or_pagerank failed ({rc})")
        return r

    def ms_work(self, sources, permille: int, want_depth: bool = False,
                max_levels: int = 4096):
        """Work model of one bit-parallel multi-source batch (or_ms_work):
        (levels as dicts, algorithmic bytes, depth rows [k][n] or None)."""
        srcs = _c32(sources)
        k = len(srcs)
        depth = np.empty((k, self.n), dtype=np.int32) if want_depth else None
        out = (MsLevel * max_levels)()
        b = ctypes.c_double(0.0)
        nl = _load().or_ms_work(self._h, _i32(srcs), k, permille,
                                _i32(depth) if want_depth else None, out, max_levels,
                                ctypes.byref(b))
        if nl < 0:
            raise ValueError(f"or_ms_work failed ({nl})")
        levels = [{"active": int(out[i].active), "e": int(out[i].e), "v": int(out[i].v),
                   "bottom_up": int(out[i].bottom_up)} for i in range(min(nl, max_levels))]
        return levels, float(b.value), depth

    def do_replay(self, TH: int, depth, factor0=(0.5, 0.05, 1e-7), factor1=(0.0, 0.0, 0.0),
                  bv_exact: bool = False, max_levels: int = 4096):
        depth = _c32(depth)
        out = (Level * max_levels)()
        f0 = (ctypes.c_double * 3)(*factor0)
        f1 = (ctypes.c_double * 3)(*factor1)
        nl = _load().or_do_replay(self._h, TH, _i32(depth), f0, f1, int(bv_exact), out,
                                  max_levels)
        if nl < 0:
            raise ValueError("or_do_replay failed")
        return [out[i].as_dict() for i in range(min(nl, max_levels))]


class WorkModel:
    """The work model of searches on one graph at one threshold (or_do_work):
    per level, the schedule and the work of every visit, and the algorithmic
    bytes per visit (or_work_bytes)."""

    def __init__(self, graph: Graph, TH: int):
        h = ctypes.c_void_p()
        rc = _load().or_work_prepare(graph._h, TH, ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"or_work_prepare failed ({rc})")
        self._h = h
        self._graph = graph   # the prepared rows point into the graph
        self.n = graph.n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_work_free(h)
            self._h = None

    def levels(self, depth, factor0, factor1, max_levels: int = 4096):
        depth = _c32(depth)
        out = (WorkLevel * max_levels)()
        f0 = (ctypes.c_double * 3)(*factor0)
        f1 = (ctypes.c_double * 3)(*factor1)
        nl = _load().or_do_work(self._h, _i32(depth), f0, f1, out, max_levels)
        if nl < 0:
            raise ValueError("or_do_work failed")
        return out, min(nl, max_levels)

    def run(self, depth, factor0, factor1, want_parent: bool = True):
        """(levels as dicts, {visit: bytes}, {visit: levels with work})."""
        out, nl = self.levels(depth, factor0, factor1)
        b = (ctypes.c_double * 7)()
        la = (ctypes.c_int64 * 7)()
        rc = _load().or_work_bytes(out, nl, self.n, 8 if want_parent else 4, b, la)
        if rc != 0:
            raise ValueError("or_work_bytes failed")
        return ([out[i].as_dict() for i in range(nl)], dict(zip(WORK_VISITS, list(b))),
                dict(zip(WORK_VISITS, list(la))))


def _replay4(graph, TH, depth, factor0, factor1, bv_exact=False, max_levels=4096):
    depth = _c32(depth)
    out = (Level4 * max_levels)()
    f0 = (ctypes.c_double * 4)(*factor0)
    f1 = (ctypes.c_double * 4)(*factor1)
    nl = _load().or_do_replay4(graph._h, TH, _i32(depth), f0, f1, int(bv_exact), out, max_levels)
    if nl < 0:
        raise ValueError("or_do_replay4 failed")
    return [out[i].as_dict() for i in range(min(nl, max_levels))]


Graph.do_replay4 = lambda self, TH, depth, factor0, factor1, bv_exact=False: \
    _replay4(self, TH, depth, factor0, factor1, bv_exact)
Graph.do_replay4.__doc__ = """Schedule with nn under the direction decision too (or_do_replay4):
per level, q, s, U, FV, BV and dir for (dd, dn, nd, nn)."""


def apsp(n: int, src, dst) -> np.ndarray:
    """Floyd-Warshall hop distances (n <= 1024), -1 where unreachable."""
    src, dst = _c32(src), _c32(dst)
    dist = np.empty(n * n, dtype=np.int32)
    rc = _load().or_apsp(n, _i32(src), _i32(dst), len(src), _i32(dist))
    if rc != 0:
        raise ValueError("or_apsp failed")
    return dist.reshape(n, n)


def bv_term(a: float, od: int) -> float:
    return float(_load().or_bv_term(a, od))


def bv_approx(U: int, q: int, s: int) -> float:
    return float(_load().or_bv_approx(U, q, s))
