#!/usr/bin/env python3
"""Benchmark of degree-separated direction-optimized BFS on one MI355X.

Default workload: RMAT scale 26 (67.1M vertices, 1.07B generated edges,
A,B,C,D = .57/.19/.19/.05, IDs relabelled, symmetrized, de-duplicated),
threshold TH = 32, 64 seeded sources with degree >= 1. One step = one
single-source search from the next source (init + every level: previsit,
direction decision, visits, close) with the graph resident in HBM.

value = harmonic mean over the timed steps of GTEPS(s) = m_cc(s) / t(s), with
m_cc(s) the undirected simple edges of the source's component and t(s) the
HIP-event time of the call on its stream.

Also reported: the roofline of the dominant kernel (algorithmic bytes from
the kernels' own work counts / their HIP-event time), the CPU oracle timed on
one host core on a bounded sample of the same workload, and (with --batched /
--served) the multi-source and served forms.

    python bench.py [--steps K] [--warmup W] [--scale S] [--threshold TH]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def harmonic(xs):
    xs = [x for x in xs if x > 0]
    return len(xs) / sum(1.0 / x for x in xs) if xs else 0.0


def geometric(xs):
    xs = [x for x in xs if x > 0]
    return math.exp(sum(math.log(x) for x in xs) / len(xs)) if xs else 0.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--threshold", type=int, default=32)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--mode", choices=("do", "plain"), default="do")
    ap.add_argument("--cpu-sources", type=int, default=1,
                    help="sources of the CPU oracle sample (0 = skip)")
    ap.add_argument("--no-parent", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is design only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1803_03922_amd import dsbfs, inputs

    torch.cuda.set_device(0)
    dev = torch.cuda.get_device_properties(0)
    log(f"device {dev.name} CUs={dev.multi_processor_count}")

    t0 = time.time()
    src, dst = inputs.rmat_edges(args.scale)
    n = 1 << args.scale
    log(f"generated RMAT scale {args.scale}: {len(src)} pairs in {time.time() - t0:.1f}s")
    sources = inputs.pick_sources(src, dst, n, args.sources, seed=1003)

    t0 = time.time()
    g = dsbfs.Graph(src, dst, n, threshold=args.threshold, keep_plain_csr=(args.mode == "plain"))
    torch.cuda.synchronize()
    build_s = time.time() - t0
    st = g.stats
    log(f"built graph in {build_s:.1f}s: m_dir={st['m_dir']} d={st['d']} "
        f"nn/nd/dn/dd={st['e_nn']}/{st['e_nd']}/{st['e_dn']}/{st['e_dd']}")
    ws = dsbfs.Workspace(g)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = None if args.no_parent else torch.empty(n, dtype=torch.int32, device="cuda")
    opts = dsbfs.run_opts(mode=1 if args.mode == "do" else 0, want_parent=parent is not None,
                          profile=True)
    stream = torch.cuda.current_stream()

    def step(s):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = dsbfs.bfs(g, ws, int(s), depth, parent, opts=opts, want_stats=True, capacity=64)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), r

    for i in range(args.warmup):
        step(sources[i % len(sources)])
    torch.cuda.synchronize()

    times, rates, levels = [], [], []
    kern = {}
    t_wall = time.time()
    for i in range(args.steps):
        s = sources[i % len(sources)]
        ms, r = step(s)
        times.append(ms)
        rates.append(r["edges_cc"] / (ms * 1e-3) / 1e9)
        levels.append(r["num_levels"])
        for name, k in r["kernels"].items():
            a = kern.setdefault(name, {"ms": 0.0, "launches": 0, "bytes": 0, "edges": 0})
            for f in a:
                a[f] += k[f]
        if i % 16 == 15:
            log(f"step {i + 1}/{args.steps}: {ms:.3f} ms, {rates[-1]:.1f} GTEPS")
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    value = harmonic(rates)
    ms_per_step = sum(times) / len(times)
    nominal = [(16 << args.scale) / (t * 1e-3) / 1e9 for t in times]

    dom = max(kern.items(), key=lambda kv: kv[1]["ms"])
    dname, dk = dom
    achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9 if dk["ms"] > 0 else 0.0
    total_kernel_ms = sum(k["ms"] for k in kern.values())
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": dname, "launches_per_step": dk["launches"] / args.steps,
                "bytes_per_launch": dk["bytes"] / max(dk["launches"], 1),
                "avg_launch_ms": dk["ms"] / max(dk["launches"], 1)}
    all_bytes = sum(k["bytes"] for k in kern.values())
    path_gbs = all_bytes / (sum(times) * 1e-3) / 1e9

    cpu = None
    if args.cpu_sources > 0:
        import oracle
        oracle.build(force=False)
        t0 = time.time()
        O = oracle.Graph(src, dst, n)
        log(f"oracle CSR built in {time.time() - t0:.1f}s (untimed)")
        deg = O.degrees()
        crates = []
        for s in sources[:args.cpu_sources].tolist():
            c0 = time.perf_counter()
            dref, _ = O.bfs(int(s), want_parent=False)
            c1 = time.perf_counter()
            m_cc = int(deg[dref >= 0].sum() // 2)
            crates.append(m_cc / (c1 - c0) / 1e9)
            log(f"oracle BFS s={s}: {c1 - c0:.2f}s, {crates[-1]:.3f} GTEPS")
            if s == sources[0]:
                dsbfs.bfs(g, ws, int(s), depth, parent, opts=dsbfs.run_opts(want_parent=False))
                torch.cuda.synchronize()
                assert np.array_equal(depth.cpu().numpy(), dref), "GPU depth != oracle depth"
        cpu = {"value": round(harmonic(crates), 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"{len(crates)} of the {len(sources)} sources, serial FIFO BFS on one "
                         f"host thread, CSR build untimed"}
        del O

    line = {
        "metric": "GTEPS (harmonic mean, 1 GPU) + p50/p99 query latency, batched vs plain BFS",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"single-source {'DOBFS' if args.mode == 'do' else 'top-down BFS'}"
                               f", RMAT scale {args.scale} edge factor 16, TH {args.threshold}",
                   "scale": args.scale, "threshold": args.threshold, "sources": len(sources),
                   "parents": parent is not None, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "gteps_geometric": round(geometric(rates), 3),
            "gteps_nominal_geometric": round(geometric(nominal), 3),
            "levels_mean": sum(levels) / len(levels),
            "path_algorithmic_gbs": round(path_gbs, 2),
            "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in kern.items()},
            "kernel_gbs": {k: round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
                           for k, v in kern.items() if v["ms"] > 0},
            "kernel_share": round(total_kernel_ms / sum(times), 3),
            "graph": st, "build_s": round(build_s, 2), "timed_wall_s": round(wall, 2),
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
