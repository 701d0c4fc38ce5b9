#!/usr/bin/env python3
"""Writes the oracle's depth digests used by the full-size GPU parity tests.

For each workload below, every listed source is searched by the CPU oracle
(serial FIFO BFS over its own CSR, oracle/oracle.c) and one line is stored:
the source, the size of its component, the component's undirected simple
edges (the GTEPS numerator), its eccentricity (largest depth) and the SHA-256
of the depth row as n int32 values, little-endian. A GPU test hashes its own
row the same way; equal digests mean bit-identical rows, and on a mismatch
the test recomputes that one oracle row to name the first differing vertex.

This script calls only the oracle and the seeded input generators (which hold
no BFS arithmetic); nothing here comes from the GPU library.

    python tests/golden/make_digests.py [--which rmat22,rmat26,rmat24,served] [--threads 8]

Workloads (graph seed 0x1803039220000000 + scale, relabelled, symmetrized,
self-loops and duplicates dropped):
  rmat22  RMAT scale 22, 64 sources picked with seed 1002
  rmat26  RMAT scale 26, 64 sources picked with seed 1003
  rmat24  RMAT scale 24, 1024 sources picked with seed 1004
  rmat28  RMAT scale 28, 8 sources picked with seed 1005 (needs about 120 GB
          of host memory; written on a host with that much)
  served  RMAT 18, 20, 22, 24 and Erdos-Renyi n = 2^22 with 8n pairs
          (seed 0x22), 64 sources each picked with seed 6000 + graph index
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1803_03922_amd import inputs  # noqa: E402

OUT = [HERE]   # directory the digest files are written to (--out)

SERVED = (("rmat", 18), ("rmat", 20), ("rmat", 22), ("rmat", 24), ("er", 22))


def digest(depth: np.ndarray) -> str:
    """SHA-256 of a depth row as int32 little-endian bytes."""
    return hashlib.sha256(np.ascontiguousarray(depth, dtype="<i4").data).hexdigest()


def edges_of(kind: str, scale: int):
    n = 1 << scale
    if kind == "rmat":
        src, dst = inputs.rmat_edges(scale)
    else:
        src, dst = inputs.er_edges(n, 8 * n, seed=0x22)
    return n, src, dst


def rows(O, deg, sources, threads):
    """(source, reached, edges_cc, ecc, sha256) per source, oracle searches in parallel."""
    def one(s):
        depth, _ = O.bfs(int(s), want_parent=False)
        reached = depth >= 0
        return (int(s), int(reached.sum()), int(deg[reached].sum() // 2), int(depth.max()),
                digest(depth))

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, [int(s) for s in sources]))


def write(path, header, lines):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        f.write("# columns: index source reached edges_cc max_depth sha256(depth as int32 LE)\n")
        for i, r in enumerate(lines):
            f.write(f"{i} {r[0]} {r[1]} {r[2]} {r[3]} {r[4]}\n")
    os.replace(tmp, path)
    print(f"wrote {path} ({len(lines)} rows)", flush=True)


def make_rmat(scale, k, seed, threads, name):
    t0 = time.time()
    n, src, dst = edges_of("rmat", scale)
    sources = inputs.pick_sources(src, dst, n, k, seed=seed)
    O = oracle.Graph(src, dst, n)
    del src, dst
    deg = O.degrees()
    print(f"{name}: oracle CSR of scale {scale} in {time.time() - t0:.1f}s", flush=True)
    out = rows(O, deg, sources, threads)
    write(os.path.join(OUT[0], f"depth_digests_{name}.txt"),
          [f"Oracle depth rows: RMAT scale {scale}, edge factor 16, A,B,C,D = .57/.19/.19/.05,",
           f"graph seed 0x1803039220000000 + {scale}, relabelled, symmetrized, deduplicated;",
           f"n = {n}, m_dir = {O.m}; {len(sources)} sources from pick_sources(k={k}, "
           f"seed={seed}).",
           f"Written by: python tests/golden/make_digests.py --which {name}"], out)
    print(f"{name}: {len(out)} rows in {time.time() - t0:.1f}s", flush=True)


def make_served(threads):
    t0 = time.time()
    out = []
    for gi, (kind, scale) in enumerate(SERVED):
        n, src, dst = edges_of(kind, scale)
        sources = inputs.pick_sources(src, dst, n, 64, seed=6000 + gi)
        O = oracle.Graph(src, dst, n)
        del src, dst
        deg = O.degrees()
        for r in rows(O, deg, sources, threads):
            out.append((gi,) + r)
        print(f"served graph {gi} ({kind} {scale}, m_dir {O.m}) done at {time.time() - t0:.1f}s",
              flush=True)
    path = os.path.join(OUT[0], "depth_digests_served.txt")
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("# Oracle depth rows of the served mix: graph 0..3 = RMAT scale 18, 20, 22, 24\n"
                "# (edge factor 16, graph seed 0x1803039220000000 + scale, relabelled), graph 4 =\n"
                "# Erdos-Renyi n = 2^22 with 8n uniform pairs (seed 0x22); all symmetrized and\n"
                "# deduplicated. 64 sources per graph from pick_sources(k=64, seed=6000 + graph).\n"
                "# Written by: python tests/golden/make_digests.py --which served\n"
                "# columns: graph source reached edges_cc max_depth sha256(depth as int32 LE)\n")
        for r in out:
            f.write(" ".join(str(x) for x in r) + "\n")
    os.replace(tmp, path)
    print(f"wrote {path} ({len(out)} rows)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--which", default="rmat22,served,rmat26,rmat24")
    ap.add_argument("--out", default=HERE, help="directory of the digest files")
    ap.add_argument("--threads", type=int, default=8)
    a = ap.parse_args()
    OUT[0] = a.out
    os.makedirs(OUT[0], exist_ok=True)
    oracle.build(force=False)
    inputs.build(force=False)
    for w in a.which.split(","):
        if w == "rmat22":
            make_rmat(22, 64, 1002, a.threads, "rmat22")
        elif w == "rmat26":
            make_rmat(26, 64, 1003, a.threads, "rmat26")
        elif w == "rmat24":
            make_rmat(24, 1024, 1004, a.threads, "rmat24")
        elif w == "rmat28":
            make_rmat(28, 8, 1005, a.threads, "rmat28")
        elif w == "served":
            make_served(a.threads)
        elif w:
            raise SystemExit(f"unknown workload {w}")


if __name__ == "__main__":
    main()
