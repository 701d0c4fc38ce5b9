"""ctypes binding of libdsbfs.so (C-ABI in include/dsbfs.h).

Argument marshalling only: every step of the search runs in the HIP library.
PyTorch supplies device memory (through the caching allocator, handed to the
library as a dsbfs_allocator) and streams. If the library is missing this
module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# PyTorch first: its HIP runtime (libamdhip64.so.7, bundled with torch) is
# then already in the process when libdsbfs.so is loaded, and the library's
# dependency on that soname binds to it. Loaded the other way round, the
# process would hold two HIP runtimes, and device memory and streams from
# torch would not be valid in the library's.
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsbfs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1803_03922_amd.build_lib`")

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
ERR_INVALID_ARG = -1
ERR_RANGE = -2
ERR_OUT_OF_MEMORY = -3
ERR_BUDGET = -4
ERR_HIP = -5
ERR_NOT_READY = -6
ERR_DEVICE = -7

vp = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)

ALLOC_FN = ctypes.CFUNCTYPE(vp, vp, ctypes.c_size_t, vp)
FREE_FN = ctypes.CFUNCTYPE(None, vp, vp, vp)


class dsbfs_allocator(ctypes.Structure):
    _fields_ = [("ctx", vp), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class dsbfs_build_opts(ctypes.Structure):
    _fields_ = [("threshold", i32), ("edges_on_device", i32), ("keep_plain_csr", i32),
                ("skip_nn_copy", i32)]


class dsbfs_graph_stats(ctypes.Structure):
    _fields_ = [(k, i64) for k in ("n", "m_dir", "d", "e_nn", "e_nd", "e_dn", "e_dd", "n_ndsrc",
                                   "n_ddsrc", "n_dnsrc", "max_degree", "bytes_layout",
                                   "bytes_plain")] + [("threshold", i32), ("reserved", i32),
                                                      ("n_nnsrc", i64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class dsbfs_rmat_spec(ctypes.Structure):
    _fields_ = [("scale", i32), ("permute", i32), ("num_edges", i64), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("perm_seed", ctypes.c_uint64)]


class dsbfs_run_opts(ctypes.Structure):
    _fields_ = [("mode", i32), ("want_parent", i32), ("factor0", ctypes.c_double * 3),
                ("factor1", ctypes.c_double * 3), ("forced", i32), ("profile", i32),
                ("forced_seed", ctypes.c_uint64), ("nn_do", i32), ("reserved", i32),
                ("factor0_nn", ctypes.c_double), ("factor1_nn", ctypes.c_double)]


class dsbfs_level_stats(ctypes.Structure):
    _fields_ = [("q", i64 * 3), ("s", i64 * 3), ("U", i64 * 3), ("FV", i64 * 3),
                ("BV", ctypes.c_double * 3), ("dir", i32 * 3), ("reserved", i32),
                ("FV_nn", i64), ("q_nn", i64), ("frontier_normal", i64),
                ("frontier_delegate", i64), ("kernel_ms", ctypes.c_double * 11),
                ("U_nn", i64), ("s_nn", i64), ("BV_nn", ctypes.c_double), ("dir_nn", i32),
                ("reserved2", i32)]

    def as_dict(self):
        return {"q": list(self.q), "s": list(self.s), "U": list(self.U), "FV": list(self.FV),
                "BV": list(self.BV), "dir": list(self.dir), "FV_nn": int(self.FV_nn),
                "q_nn": int(self.q_nn), "frontier_normal": int(self.frontier_normal),
                "frontier_delegate": int(self.frontier_delegate), "U_nn": int(self.U_nn),
                "s_nn": int(self.s_nn), "BV_nn": float(self.BV_nn), "dir_nn": int(self.dir_nn)}


KERNEL_NAMES = ("init", "prev_normal", "prev_deleg", "td_normal", "td_deleg", "bu_normal",
                "bu_deleg", "close", "plain", "td_nn", "bu_nn")


class dsbfs_kernel_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", i64), ("bytes", i64), ("edges", i64)]


class dsbfs_run_stats(ctypes.Structure):
    _fields_ = [("num_levels", i32), ("capacity", i32),
                ("levels", ctypes.POINTER(dsbfs_level_stats)), ("reached", i64),
                ("edges_cc", i64), ("kernels", dsbfs_kernel_profile * len(KERNEL_NAMES))]


class dsbfs_ms_opts(ctypes.Structure):
    _fields_ = [("block", i32), ("blocks_per_cu", i32), ("bu_permille", i32), ("use_graph", i32),
                ("lanes_per_batch", i32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class dsbfs_query_stats(ctypes.Structure):
    _fields_ = [("arrival_ns", i64), ("admit_ns", i64), ("start_ns", i64), ("done_ns", i64),
                ("graph_id", i32), ("source", i32), ("levels", i32), ("batched", i32),
                ("waited_budget", i32), ("loaded_graph", i32)]


class dsbfs_server_stats(ctypes.Structure):
    _fields_ = [(k, i64) for k in ("budget_bytes", "used_bytes", "graphs", "resident_graphs",
                                   "loads", "evictions", "budget_waits", "queries_done")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class dsbfs_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_lanes", i32), ("batched", i32),
                ("ms", dsbfs_ms_opts), ("join_levels", i32), ("reserved", i32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


dsbfs_run_opts_default = _sig("dsbfs_run_opts_default", i32, [ctypes.POINTER(dsbfs_run_opts)])
dsbfs_graph_create = _sig("dsbfs_graph_create", i32,
                          [I32P, I32P, i64, i32, ctypes.POINTER(dsbfs_build_opts),
                           ctypes.POINTER(dsbfs_allocator), vp, ctypes.POINTER(vp)])
dsbfs_graph_stats_get = _sig("dsbfs_graph_stats_get", i32, [vp, ctypes.POINTER(dsbfs_graph_stats)])
dsbfs_graph_export = _sig("dsbfs_graph_export", i32, [vp, i32, vp, i64, I64P])
dsbfs_graph_destroy = _sig("dsbfs_graph_destroy", i32, [vp])
dsbfs_workspace_create = _sig("dsbfs_workspace_create", i32, [vp, i32, ctypes.POINTER(vp)])
dsbfs_workspace_destroy = _sig("dsbfs_workspace_destroy", i32, [vp])
dsbfs_bfs = _sig("dsbfs_bfs", i32, [vp, vp, i32, ctypes.POINTER(dsbfs_run_opts), vp, vp,
                                    ctypes.POINTER(dsbfs_run_stats), vp])
dsbfs_rmat_generate = _sig("dsbfs_rmat_generate", i32, [ctypes.POINTER(dsbfs_rmat_spec), vp, vp,
                                                        vp])
dsbfs_graph_create_rmat = _sig("dsbfs_graph_create_rmat", i32,
                               [ctypes.POINTER(dsbfs_rmat_spec), ctypes.POINTER(dsbfs_build_opts),
                                ctypes.POINTER(dsbfs_allocator), vp, ctypes.POINTER(vp)])
dsbfs_pagerank = _sig("dsbfs_pagerank", i32, [vp, ctypes.c_double, i32, ctypes.c_double, vp,
                                              ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                              vp])
dsbfs_bfs_noalloc = _sig("dsbfs_bfs_noalloc", i32, [vp, i32, ctypes.POINTER(dsbfs_run_opts), vp,
                                                    vp, ctypes.POINTER(dsbfs_run_stats), vp])
dsbfs_msbfs = _sig("dsbfs_msbfs", i32, [vp, vp, I32P, i32, ctypes.POINTER(dsbfs_ms_opts), vp, vp])
dsbfs_msbfs_tune = _sig("dsbfs_msbfs_tune", i32, [vp, vp, I32P, i32, ctypes.c_char_p,
                                                  ctypes.POINTER(dsbfs_ms_opts), vp])
dsbfs_server_create = _sig("dsbfs_server_create", i32,
                           [ctypes.POINTER(dsbfs_server_opts), ctypes.POINTER(dsbfs_allocator),
                            ctypes.POINTER(vp)])
dsbfs_server_add_graph = _sig("dsbfs_server_add_graph", i32, [vp, vp, I32P])
dsbfs_server_submit = _sig("dsbfs_server_submit", i32, [vp, i32, i32, i64, I64P])
dsbfs_server_wait = _sig("dsbfs_server_wait", i32, [vp, i64, i64, ctypes.POINTER(vp),
                                                    ctypes.POINTER(dsbfs_query_stats)])
dsbfs_server_release = _sig("dsbfs_server_release", i32, [vp, i64])
dsbfs_server_stats_get = _sig("dsbfs_server_stats_get", i32, [vp, ctypes.POINTER(dsbfs_server_stats)])
dsbfs_server_destroy = _sig("dsbfs_server_destroy", i32, [vp])
dsbfs_now_ns = _sig("dsbfs_now_ns", i64, [])
dsbfs_status_str = _sig("dsbfs_status_str", ctypes.c_char_p, [i32])
dsbfs_last_error = _sig("dsbfs_last_error", ctypes.c_char_p, [])

EXPORTED = [n for n in dir() if n.startswith("dsbfs_") and callable(globals()[n])
            and hasattr(globals()[n], "argtypes")]


class DsbfsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = dsbfs_last_error().decode(errors="replace")
        super().__init__(f"{where}: {dsbfs_status_str(status).decode()} ({status}): {msg}")


def check(st: int, where: str):
    if st != OK:
        raise DsbfsError(st, where)


# ---------------------------------------------------------------------------
# Teardown order: every live library object (servers, workspaces, graphs) is
# destroyed explicitly before the interpreter shuts down, while the HIP
# runtime and PyTorch's allocator (which the library frees into) still work.
# Finalizers that run during interpreter shutdown call nothing in the library.
# ---------------------------------------------------------------------------
import atexit  # noqa: E402
import sys  # noqa: E402
import weakref  # noqa: E402

_live = weakref.WeakValueDictionary()   # creation number -> object
_serial = [0]


def _track(obj):
    _serial[0] += 1
    _live[_serial[0]] = obj


def shutdown():
    """Destroys every live server, workspace and graph, newest first (servers
    own their graphs, and a workspace is destroyed before its graph). Called
    at interpreter exit, before PyTorch and the HIP runtime are torn down; a
    program may call it earlier itself."""
    objs = [o for _, o in sorted(_live.items(), reverse=True)]
    for kind in (Server, Workspace, Graph):
        for o in objs:
            if isinstance(o, kind):
                try:
                    o.destroy()
                except Exception:
                    pass


atexit.register(shutdown)


# ---------------------------------------------------------------------------
# torch plumbing: device memory and streams
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


class TorchAllocator:
    """dsbfs_allocator backed by PyTorch's caching allocator on the current device."""

    def __init__(self):
        torch = _torch()
        self.device = torch.cuda.current_device()

        def _alloc(ctx, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                          stream or 0)
            except Exception:
                return None

        def _free(ctx, ptr, stream):
            if ptr:
                torch.cuda.caching_allocator_delete(ptr)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = dsbfs_allocator(None, self._a, self._f)


_default_alloc = None


def default_allocator() -> TorchAllocator:
    global _default_alloc
    if _default_alloc is None:
        _default_alloc = TorchAllocator()
    return _default_alloc


def current_stream() -> int:
    return _torch().cuda.current_stream().cuda_stream


def _i32ptr(a: np.ndarray):
    return a.ctypes.data_as(I32P)


def _dev_ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


# The paper's direction-switch factors for (dd, dn, nd) (Section VI-B), the
# header's DSBFS_PAPER_FACTOR0_* constants. The library's defaults differ:
# run_opts() without factor0 takes them from dsbfs_run_opts_default.
PAPER_FACTOR0 = (0.5, 0.05, 1e-7)


def run_opts(mode: int = 1, want_parent: bool = True, factor0=None, factor1=None,
             forced: int = 0, forced_seed: int = 0, profile: bool = False, nn_do: bool = False,
             factor_nn=None) -> dsbfs_run_opts:
    o = dsbfs_run_opts()
    check(dsbfs_run_opts_default(ctypes.byref(o)), "dsbfs_run_opts_default")
    o.mode = mode
    o.want_parent = int(bool(want_parent))
    if factor0 is not None:
        o.factor0 = (ctypes.c_double * 3)(*factor0)
    if factor1 is not None:
        o.factor1 = (ctypes.c_double * 3)(*factor1)
    o.forced = forced
    o.forced_seed = forced_seed
    o.profile = int(bool(profile))
    o.nn_do = int(bool(nn_do))
    if factor_nn is not None:
        o.factor0_nn, o.factor1_nn = float(factor_nn[0]), float(factor_nn[1])
    return o


def rmat_spec(scale: int, edge_factor: int = 16, seed: int | None = None, permute: bool = True,
              a: float = 0.57, b: float = 0.19, c: float = 0.19,
              perm_seed: int | None = None) -> dsbfs_rmat_spec:
    """RMAT spec with the workload's conventions: graph seed
    0x1803039220000000 + scale, relabelling seed graph seed ^ 1."""
    gs = (0x1803039220000000 + scale) if seed is None else seed
    ps = (gs ^ 1) if perm_seed is None else perm_seed
    return dsbfs_rmat_spec(scale, int(permute), edge_factor << scale, a, b, c, gs, ps)


def rmat_generate(spec: dsbfs_rmat_spec, stream: int | None = None):
    """The RMAT edge list of spec on the device: (src, dst) int32 torch tensors."""
    torch = _torch()
    stream = current_stream() if stream is None else stream
    src = torch.empty(max(spec.num_edges, 1), dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    check(dsbfs_rmat_generate(ctypes.byref(spec), _dev_ptr(src), _dev_ptr(dst), stream),
          "dsbfs_rmat_generate")
    return src[:spec.num_edges], dst[:spec.num_edges]


class Graph:
    """A graph resident on the current GPU (dsbfs_graph)."""

    def __init__(self, src, dst, n: int, threshold: int = 32, keep_plain_csr: bool = True,
                 allocator: TorchAllocator | None = None, stream: int | None = None,
                 rmat: dsbfs_rmat_spec | None = None, nn_copy: bool = True):
        """From an edge list (host numpy or device torch arrays), or, with
        rmat given (src, dst, n ignored), generated on the device. nn_copy =
        False skips the compact nn copy (skip_nn_copy)."""
        self.alloc = allocator or default_allocator()
        self.stream = current_stream() if stream is None else stream
        opts = dsbfs_build_opts(threshold, 0, int(keep_plain_csr), int(not nn_copy))
        h = vp()
        if rmat is not None:
            check(dsbfs_graph_create_rmat(ctypes.byref(rmat), ctypes.byref(opts),
                                          ctypes.byref(self.alloc.struct), self.stream,
                                          ctypes.byref(h)), "dsbfs_graph_create_rmat")
            self._finish(h, 1 << rmat.scale)
            return
        on_dev = not isinstance(src, np.ndarray)
        if on_dev:
            opts.edges_on_device = 1
            ps = ctypes.cast(ctypes.c_void_p(_dev_ptr(src)), I32P)
            pd = ctypes.cast(ctypes.c_void_p(_dev_ptr(dst)), I32P)
            g = int(src.numel())
        else:
            self._src = np.ascontiguousarray(src, dtype=np.int32)
            self._dst = np.ascontiguousarray(dst, dtype=np.int32)
            ps, pd, g = _i32ptr(self._src), _i32ptr(self._dst), len(self._src)
        check(dsbfs_graph_create(ps, pd, g, n, ctypes.byref(opts), ctypes.byref(self.alloc.struct),
                                 self.stream, ctypes.byref(h)), "dsbfs_graph_create")
        self._src = self._dst = None
        self._finish(h, n)

    def _finish(self, h, n):
        self.h = h
        self.n = n
        st = dsbfs_graph_stats()
        check(dsbfs_graph_stats_get(self.h, ctypes.byref(st)), "dsbfs_graph_stats_get")
        self.stats = st.as_dict()
        _track(self)

    def export(self, which: int, dtype) -> np.ndarray:
        nbytes = ctypes.c_int64(0)
        check(dsbfs_graph_export(self.h, which, None, 0, ctypes.byref(nbytes)), "export")
        out = np.empty(max(nbytes.value // np.dtype(dtype).itemsize, 0), dtype=dtype)
        if nbytes.value:
            check(dsbfs_graph_export(self.h, which, out.ctypes.data_as(vp), nbytes.value,
                                     ctypes.byref(nbytes)), "export")
        return out

    def destroy(self):
        if self.h:
            check(dsbfs_graph_destroy(self.h), "dsbfs_graph_destroy")
            self.h = None

    def release_ownership(self):
        """Forget the handle (after moving it to a server)."""
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.destroy()
        except Exception:
            pass


class Workspace:
    def __init__(self, graph: Graph, max_lanes: int = 0):
        h = vp()
        check(dsbfs_workspace_create(graph.h, max_lanes, ctypes.byref(h)), "dsbfs_workspace_create")
        self.h = h
        self.graph = graph
        _track(self)

    def destroy(self):
        if self.h:
            check(dsbfs_workspace_destroy(self.h), "dsbfs_workspace_destroy")
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.destroy()
        except Exception:
            pass


def bfs(graph: Graph, ws: Workspace, source: int, depth, parent=None, opts=None,
        want_stats: bool = False, capacity: int = 256, stream: int | None = None):
    """Runs dsbfs_bfs into device int32 tensors depth/parent; returns stats or None."""
    stream = current_stream() if stream is None else stream
    if opts is None:
        opts = run_opts(want_parent=parent is not None)
    st = None
    levels = None
    if want_stats:
        levels = (dsbfs_level_stats * capacity)()
        st = dsbfs_run_stats()
        st.capacity = capacity
        st.levels = ctypes.cast(levels, ctypes.POINTER(dsbfs_level_stats))
    check(dsbfs_bfs(graph.h, ws.h, source, ctypes.byref(opts), _dev_ptr(depth), _dev_ptr(parent),
                    ctypes.byref(st) if st is not None else None, stream), "dsbfs_bfs")
    if not want_stats:
        return None
    nl = st.num_levels
    kern = {name: {"ms": float(st.kernels[i].ms), "launches": int(st.kernels[i].launches),
                   "bytes": int(st.kernels[i].bytes), "edges": int(st.kernels[i].edges)}
            for i, name in enumerate(KERNEL_NAMES)}
    return {"num_levels": nl, "reached": int(st.reached), "edges_cc": int(st.edges_cc),
            "levels": [levels[i].as_dict() for i in range(min(nl, capacity))],
            "level_kernel_ms": [{name: float(levels[i].kernel_ms[j])
                                 for j, name in enumerate(KERNEL_NAMES)}
                                for i in range(min(nl, capacity))],
            "kernels": kern}


def bfs_noalloc(graph: Graph, source: int, depth, parent=None, opts=None,
                stream: int | None = None):
    """Runs dsbfs_bfs_noalloc (no workspace, no allocation) into device int32
    tensors depth/parent."""
    stream = current_stream() if stream is None else stream
    if opts is None:
        opts = run_opts(want_parent=parent is not None)
    check(dsbfs_bfs_noalloc(graph.h, source, ctypes.byref(opts), _dev_ptr(depth),
                            _dev_ptr(parent), None, stream), "dsbfs_bfs_noalloc")


def pagerank(graph: Graph, rank, alpha: float = 0.85, iterations: int = 20,
             tolerance: float = 0.0, stream: int | None = None):
    """dsbfs_pagerank into a device float64 tensor rank[n]; returns
    (steps run, last L1 change)."""
    stream = current_stream() if stream is None else stream
    it = i32(0)
    dl = ctypes.c_double(0.0)
    check(dsbfs_pagerank(graph.h, alpha, iterations, tolerance, _dev_ptr(rank), ctypes.byref(it),
                         ctypes.byref(dl), stream), "dsbfs_pagerank")
    return it.value, dl.value


def msbfs(graph: Graph, ws: Workspace, sources, depth, opts: dsbfs_ms_opts | None = None,
          stream: int | None = None):
    stream = current_stream() if stream is None else stream
    srcs = np.ascontiguousarray(sources, dtype=np.int32)
    check(dsbfs_msbfs(graph.h, ws.h, _i32ptr(srcs), len(srcs),
                      ctypes.byref(opts) if opts is not None else None, _dev_ptr(depth), stream),
          "dsbfs_msbfs")


def msbfs_tune(graph: Graph, ws: Workspace, sources, cache_path: str | None = None,
               stream: int | None = None) -> dsbfs_ms_opts:
    stream = current_stream() if stream is None else stream
    srcs = np.ascontiguousarray(sources, dtype=np.int32)
    best = dsbfs_ms_opts()
    check(dsbfs_msbfs_tune(graph.h, ws.h, _i32ptr(srcs), len(srcs),
                           cache_path.encode() if cache_path else None, ctypes.byref(best),
                           stream), "dsbfs_msbfs_tune")
    return best


def now_ns() -> int:
    return int(dsbfs_now_ns())


class _DevRow:
    """A device int32 vector at a raw address, exposed to torch through the
    CUDA array interface (no copy). torch accepts only writable views; the
    row stays the library's and callers treat it as read-only."""

    def __init__(self, ptr: int, n: int):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<i4", "data": (ptr, False),
                                         "version": 2, "strides": None}


def device_row(ptr: int, n: int):
    """torch view of a device int32[n] row owned by the library."""
    return _torch().as_tensor(_DevRow(ptr, n), device="cuda")


class Server:
    """Continuous-batching query server (dsbfs_server)."""

    PLAIN, BATCHED, ADAPTIVE = 0, 1, 2

    def __init__(self, budget_bytes: int, max_lanes: int = 64, batched: bool | int = True,
                 ms: dsbfs_ms_opts | None = None, join_levels: int = 0,
                 allocator: TorchAllocator | None = None):
        """batched: False/0 plain, True/1 continuous batching, 2 adaptive.
        allocator: result rows from it (e.g. default_allocator(), PyTorch's
        caching allocator; its callbacks then run on the scheduler thread),
        else from hipMalloc."""
        o = dsbfs_server_opts()
        o.hbm_budget_bytes = int(budget_bytes)
        o.max_lanes = max_lanes
        o.batched = int(batched)
        o.ms = ms if ms is not None else dsbfs_ms_opts(256, 4, 2, 0)
        o.join_levels = join_levels
        self.alloc = allocator
        h = vp()
        check(dsbfs_server_create(ctypes.byref(o),
                                  ctypes.byref(allocator.struct) if allocator else None,
                                  ctypes.byref(h)), "dsbfs_server_create")
        self.h = h
        self.n_of = {}
        _track(self)

    def add_graph(self, graph: Graph) -> int:
        gid = ctypes.c_int32(0)
        check(dsbfs_server_add_graph(self.h, graph.h, ctypes.byref(gid)), "dsbfs_server_add_graph")
        self.n_of[gid.value] = graph.n
        graph.release_ownership()
        return gid.value

    def submit(self, gid: int, source: int, arrival_ns: int = 0) -> int:
        t = ctypes.c_int64(0)
        check(dsbfs_server_submit(self.h, gid, source, arrival_ns, ctypes.byref(t)),
              "dsbfs_server_submit")
        return t.value

    def wait(self, ticket: int, timeout_ns: int = -1):
        """(device pointer of the depth row, stats dict); raises on NOT_READY."""
        p = vp()
        st = dsbfs_query_stats()
        check(dsbfs_server_wait(self.h, ticket, timeout_ns, ctypes.byref(p), ctypes.byref(st)),
              "dsbfs_server_wait")
        return p.value, {k: int(getattr(st, k)) for k, _ in st._fields_}

    def release(self, ticket: int):
        check(dsbfs_server_release(self.h, ticket), "dsbfs_server_release")

    def stats(self) -> dict:
        st = dsbfs_server_stats()
        check(dsbfs_server_stats_get(self.h, ctypes.byref(st)), "dsbfs_server_stats_get")
        return st.as_dict()

    def destroy(self):
        if self.h:
            check(dsbfs_server_destroy(self.h), "dsbfs_server_destroy")
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.destroy()
        except Exception:
            pass
