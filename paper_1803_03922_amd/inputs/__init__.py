"""Seeded synthetic workloads (RMAT, Erdos-Renyi, vertex relabelling, sources).

Thin ctypes binding over ``gen.c``. This module holds no BFS arithmetic and is
shared by the GPU path's tests/benchmarks and the CPU oracle's tests: it is
the only code that both sides use.

Workload recipe (paper Section VI-A, "Reporting"): RMAT scale N with 2^N
vertices, edge factor 16, A,B,C,D = 0.57/0.19/0.19/0.05, IDs relabelled by a
deterministic bijective hash after generation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdsbfs_inputs.so")
_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19
EDGE_FACTOR = 16


def graph_seed(scale: int) -> int:
    """Seed of the RMAT graph at a given scale."""
    return 0x1803039220000000 + scale


def build(force: bool = True) -> str:
    """Compile gen.c into libdsbfs_inputs.so next to it (host code, gcc)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp,
                               os.path.join(_HERE, "gen.c")])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.inp_splitmix64_mix.restype = ctypes.c_uint64
        lib.inp_splitmix64_mix.argtypes = [ctypes.c_uint64]
        lib.inp_splitmix64_at.restype = ctypes.c_uint64
        lib.inp_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.inp_rmat.restype = ctypes.c_int
        lib.inp_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, i32p, i32p, ctypes.c_int]
        lib.inp_permute.restype = ctypes.c_int
        lib.inp_permute.argtypes = [ctypes.c_int, ctypes.c_uint64, i32p, i32p, ctypes.c_int64,
                                    ctypes.c_int]
        lib.inp_perm_value.restype = ctypes.c_uint64
        lib.inp_perm_value.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        lib.inp_er.restype = ctypes.c_int
        lib.inp_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p,
                               ctypes.c_int]
        lib.inp_pick_sources.restype = ctypes.c_int64
        lib.inp_pick_sources.argtypes = [i32p, i32p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_uint64, i32p]
        lib.inp_pick_sources_deg.restype = ctypes.c_int64
        lib.inp_pick_sources_deg.argtypes = [i32p, ctypes.c_int32, ctypes.c_int64,
                                             ctypes.c_uint64, i32p]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def splitmix64_at(seed: int, k: int) -> int:
    return int(_load().inp_splitmix64_at(seed & (2**64 - 1), k))


def splitmix64_mix(z: int) -> int:
    return int(_load().inp_splitmix64_mix(z & (2**64 - 1)))


def perm_value(bits: int, seed: int, x: int) -> int:
    return int(_load().inp_perm_value(bits, seed & (2**64 - 1), x))


def rmat_edges(scale: int, edge_factor: int = EDGE_FACTOR, seed: int | None = None,
               permute: bool = True, a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C,
               nthreads: int = 0):
    """RMAT edge list (src, dst) as int32 numpy arrays, n = 2^scale.

    The graph seed defaults to graph_seed(scale); the relabelling seed is
    graph seed ^ 1.
    """
    lib = _load()
    if seed is None:
        seed = graph_seed(scale)
    g = edge_factor << scale
    src = np.empty(g, dtype=np.int32)
    dst = np.empty(g, dtype=np.int32)
    rc = lib.inp_rmat(scale, g, a, b, c, seed, _p(src), _p(dst), nthreads)
    if rc != 0:
        raise ValueError("inp_rmat: bad arguments")
    if permute:
        rc = lib.inp_permute(scale, seed ^ 1, _p(src), _p(dst), g, nthreads)
        if rc != 0:
            raise ValueError("inp_permute: bad arguments")
    return src, dst


def er_edges(n: int, num_pairs: int, seed: int = 0x22, nthreads: int = 0):
    """Uniform (u, v) pairs with replacement over [0, n) as int32 arrays."""
    lib = _load()
    src = np.empty(num_pairs, dtype=np.int32)
    dst = np.empty(num_pairs, dtype=np.int32)
    rc = lib.inp_er(n, num_pairs, seed, _p(src), _p(dst), nthreads)
    if rc != 0:
        raise ValueError("inp_er: bad arguments")
    return src, dst


def pick_sources(src: np.ndarray, dst: np.ndarray, n: int, k: int, seed: int) -> np.ndarray:
    """k distinct seeded sources, each with at least one non-loop incident pair."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    out = np.empty(max(k, 1), dtype=np.int32)
    got = lib.inp_pick_sources(_p(src), _p(dst), len(src), n, k, seed, _p(out))
    if got < 0:
        raise ValueError("inp_pick_sources: bad arguments")
    return out[:got].copy()


def pick_sources_deg(deg: np.ndarray, k: int, seed: int) -> np.ndarray:
    """pick_sources from a degree array (same sources: eligible iff degree > 0)."""
    lib = _load()
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    out = np.empty(max(k, 1), dtype=np.int32)
    got = lib.inp_pick_sources_deg(_p(deg), len(deg), k, seed, _p(out))
    if got < 0:
        raise ValueError("inp_pick_sources_deg: bad arguments")
    return out[:got].copy()
