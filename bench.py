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


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 summary in
    profiles/ (FETCH_SIZE + WRITE_SIZE runs, calibrated on a copy kernel), if
    one exists for this workload and for the current kernel source; else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1803_03922_amd", "csrc", "bfs.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic: "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if (kv.get("kernel") == kernel and kv.get("workload") == workload.replace(" ", "_")
                    and kv.get("source_sha256") == h):
                return float(kv["bytes_per_launch"])
    return None


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
    ap.add_argument("--batched", type=int, default=1,
                    help="1: also measure multi-source BFS (RMAT scale --ms-scale, 1024 sources)")
    ap.add_argument("--ms-scale", type=int, default=24)
    ap.add_argument("--ms-sources", type=int, default=1024)
    ap.add_argument("--served", type=int, default=1,
                    help="1: also measure the query server (5 graphs, 3 Poisson rates)")
    ap.add_argument("--serve-queries", type=int, default=4096)
    ap.add_argument("--serve-scales", default="18,20,22,24")
    ap.add_argument("--factor-sweep", default="",
                    help="comma-separated factor0 values tried for each of dd, dn, nd in turn "
                         "(the other two at their defaults), e.g. 1e-8,1e-6,1e-4,1e-2,0.05,0.5,2,10")
    ap.add_argument("--factor-steps", type=int, default=16)
    ap.add_argument("--factor-grid", default="",
                    help="joint sweep: 'dd values;dn values;nd values', each comma-separated; "
                         "every combination is timed over --factor-steps sources")
    ap.add_argument("--th-sweep", default="16,32,64,128",
                    help="thresholds re-run on the same graph and sources ('' = none)")
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
    mode = 1 if args.mode == "do" else 0
    opts = dsbfs.run_opts(mode=mode, want_parent=parent is not None)
    popts = dsbfs.run_opts(mode=mode, want_parent=parent is not None, profile=True)
    stream = torch.cuda.current_stream()

    def timed(gr, wsp, s, o, want_stats=False):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = dsbfs.bfs(gr, wsp, int(s), depth, parent, opts=o, want_stats=want_stats,
                      capacity=64)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), r

    # The GTEPS numerator of a source (edges of its component) comes from an
    # untimed search with statistics; the timed searches run without them.
    edges_cc, nlev = {}, {}
    for s in sources.tolist():
        _, r = timed(g, ws, s, opts, want_stats=True)
        edges_cc[s], nlev[s] = r["edges_cc"], r["num_levels"]
    for i in range(args.warmup):
        timed(g, ws, sources[i % len(sources)], opts)
    torch.cuda.synchronize()

    times, rates, levels = [], [], []
    t_wall = time.time()
    for i in range(args.steps):
        s = int(sources[i % len(sources)])
        ms, _ = timed(g, ws, s, opts)
        times.append(ms)
        rates.append(edges_cc[s] / (ms * 1e-3) / 1e9)
        levels.append(nlev[s])
        if i % 16 == 15:
            log(f"step {i + 1}/{args.steps}: {ms:.3f} ms, {rates[-1]:.1f} GTEPS")
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    value = harmonic(rates)
    ms_per_step = sum(times) / len(times)
    nominal = [(16 << args.scale) / (t * 1e-3) / 1e9 for t in times]

    # Kernel breakdown: the same searches again with every kernel timed by HIP
    # events on the search's stream (direct launches instead of graphs).
    kern, ptimes = {}, []
    for i in range(args.steps):
        ms, r = timed(g, ws, sources[i % len(sources)], popts, want_stats=True)
        ptimes.append(ms)
        for name, k in r["kernels"].items():
            a = kern.setdefault(name, {"ms": 0.0, "launches": 0, "bytes": 0, "edges": 0})
            for f in a:
                a[f] += k[f]
    torch.cuda.synchronize()

    dom = max(kern.items(), key=lambda kv: kv[1]["ms"])
    dname, dk = dom
    achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9 if dk["ms"] > 0 else 0.0
    total_kernel_ms = sum(k["ms"] for k in kern.values())
    kname = {"prev_normal": "k_normal_level", "td_normal": "k_td_nd", "bu_normal": "k_bu_normal",
             "bu_deleg": "k_bu_deleg", "td_deleg": "k_td_deleg", "prev_deleg": "k_prev_deleg",
             "close": "k_close", "init": "k_init", "plain": "k_plain_expand"}[dname]
    wl = f"RMAT{args.scale} TH{args.threshold} {args.mode} {args.sources}src parents={int(parent is not None)}"
    tr = measured_traffic(kname, wl)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": None if tr is None else round(tr / 1e6, 2),
                "traffic_unit": "MB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                "kernel": dname, "launches_per_step": dk["launches"] / args.steps,
                "bytes_per_launch": dk["bytes"] / max(dk["launches"], 1),
                "avg_launch_ms": dk["ms"] / max(dk["launches"], 1)}
    all_bytes = sum(k["bytes"] for k in kern.values())
    path_gbs = all_bytes / (sum(times) * 1e-3) / 1e9

    def time_factors(f0):
        o3 = dsbfs.run_opts(want_parent=parent is not None, factor0=f0)
        tt, rr = [], []
        for i in range(args.factor_steps):
            s = int(sources[i % len(sources)])
            ms, _ = timed(g, ws, s, o3)
            tt.append(ms)
            rr.append(edges_cc[s] / (ms * 1e-3) / 1e9)
        return round(harmonic(rr), 3), round(sum(tt) / len(tt), 4)

    fsweep = []
    fvals = [float(x) for x in args.factor_sweep.split(",") if x.strip()]
    base = list(dsbfs.run_opts().factor0)
    for ki, kname_f in enumerate(("dd", "dn", "nd")):
        for v in fvals:
            f0 = list(base)
            f0[ki] = v
            gt, mss = time_factors(f0)
            fsweep.append({"kernel": kname_f, "factor0": v, "gteps": gt, "ms_per_step": mss})
            log(f"factor0[{kname_f}] = {v:g}: {gt} GTEPS")
    if args.factor_grid:
        import itertools
        axes = [[float(x) for x in part.split(",") if x.strip()]
                for part in args.factor_grid.split(";")]
        for f0 in itertools.product(*axes):
            gt, mss = time_factors(list(f0))
            fsweep.append({"factor0": list(f0), "gteps": gt, "ms_per_step": mss})
            log(f"factor0 = {list(f0)}: {gt} GTEPS, {mss} ms")

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

    del ws, g
    torch.cuda.empty_cache()
    sweep = []
    for th in [int(x) for x in args.th_sweep.split(",") if x.strip()]:
        gs = dsbfs.Graph(src, dst, n, threshold=th, keep_plain_csr=False)
        wss = dsbfs.Workspace(gs)
        o2 = dsbfs.run_opts(want_parent=parent is not None)
        tt, rr, byts = [], [], 0
        for s in sources.tolist()[:min(args.steps, len(sources))]:
            _, r = timed(gs, wss, s, o2, want_stats=True)   # untimed: numerator and bytes
            ms, _ = timed(gs, wss, s, o2)
            tt.append(ms)
            rr.append(r["edges_cc"] / (ms * 1e-3) / 1e9)
            byts += sum(k["bytes"] for k in r["kernels"].values())
        gst = gs.stats
        sweep.append({"threshold": th, "gteps": round(harmonic(rr), 3),
                      "ms_per_step": round(sum(tt) / len(tt), 4),
                      "algorithmic_gbs": round(byts / (sum(tt) * 1e-3) / 1e9, 2),
                      "d": gst["d"], "e_nn": gst["e_nn"], "e_nd": gst["e_nd"],
                      "e_dn": gst["e_dn"], "e_dd": gst["e_dd"],
                      "bytes_layout": gst["bytes_layout"]})
        log(f"TH {th}: {sweep[-1]['gteps']} GTEPS, d={gst['d']}")
        wss.destroy()
        gs.destroy()
    want_parent = parent is not None
    del depth, parent, src, dst
    torch.cuda.empty_cache()
    batched = bench_batched(args, torch, dsbfs, inputs) if args.batched else None
    torch.cuda.empty_cache()
    served = bench_served(args, torch, dsbfs, inputs) if args.served else None

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
                   "parents": want_parent, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "th_sweep": sweep,
        "factor_sweep": fsweep,
        "batched": batched,
        "served": served,
        "detail": {
            "gteps_geometric": round(geometric(rates), 3),
            "gteps_nominal_geometric": round(geometric(nominal), 3),
            "levels_mean": sum(levels) / len(levels),
            "path_algorithmic_gbs": round(path_gbs, 2),
            "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in kern.items()},
            "kernel_gbs": {k: round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
                           for k, v in kern.items() if v["ms"] > 0},
            "kernel_share_profiled": round(total_kernel_ms / sum(ptimes), 3),
            "ms_per_step_profiled": round(sum(ptimes) / len(ptimes), 4),
            "graph": st, "build_s": round(build_s, 2), "timed_wall_s": round(wall, 2),
        },
    }
    print(json.dumps(line), flush=True)


def bench_batched(args, torch, dsbfs, inputs):
    """Multi-source BFS: all sources (up to 256 lanes per batch) in one persistent,
    graph-captured launch, tuned by the autotuner, against single-source
    DOBFS from the same sources on the same graph (depth only on both sides)."""
    scale = args.ms_scale
    n = 1 << scale
    src, dst = inputs.rmat_edges(scale)
    g = dsbfs.Graph(src, dst, n, threshold=args.threshold, keep_plain_csr=True)
    sources = inputs.pick_sources(src, dst, n, args.ms_sources, seed=1004)
    del src, dst
    ws = dsbfs.Workspace(g, max_lanes=64)
    t0 = time.time()
    opts = dsbfs.msbfs_tune(g, ws, sources)   # times candidates on one batch
    log(f"msbfs tuned in {time.time() - t0:.1f}s: {opts.as_dict()}")
    depth = torch.empty((len(sources), n), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    dsbfs.msbfs(g, ws, sources, depth, opts)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    dsbfs.msbfs(g, ws, sources, depth, opts)
    e1.record(stream)
    e1.synchronize()
    t_batch = e0.elapsed_time(e1)
    log(f"msbfs: {len(sources)} sources in {t_batch:.1f} ms")
    del depth
    torch.cuda.empty_cache()
    d1 = torch.empty(n, dtype=torch.int32, device="cuda")
    o1 = dsbfs.run_opts(want_parent=False)
    # edges of each source's component from an untimed search with
    # statistics; the timed single searches run without them (captured level
    # graphs), as in the single-source bench
    ecc = {}
    for s in set(sources.tolist()):
        ecc[s] = dsbfs.bfs(g, ws, s, d1, None, opts=o1, want_stats=True)["edges_cc"]
    tot_ms, tot_e = 0.0, 0
    for s in sources.tolist():
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dsbfs.bfs(g, ws, s, d1, None, opts=o1)
        b.record(stream)
        b.synchronize()
        tot_ms += a.elapsed_time(b)
        tot_e += ecc[s]
    log(f"single-source DOBFS: {tot_ms:.1f} ms total")
    k = len(sources)
    lanes = opts.lanes_per_batch or (64 if k <= 64 else 128 if k <= 128 else 256)
    out = {"workload": f"RMAT scale {scale}, {k} sources = "
                       f"{(k + lanes - 1) // lanes} batches of {lanes} lanes, one persistent "
                       f"{'graph-captured ' if opts.use_graph else ''}launch",
           "value": round(tot_e / (t_batch * 1e-3) / 1e9, 2), "unit": "GTEPS (aggregate)",
           "launch_ms": round(t_batch, 2),
           "plain_gteps": round(tot_e / (tot_ms * 1e-3) / 1e9, 2),
           "plain_ms_total": round(tot_ms, 2),
           "speedup": round(tot_ms / t_batch, 2), "tuned": opts.as_dict()}
    ws.destroy()
    g.destroy()
    return out


def _poisson_run(dsbfs, server, gids, pools, ncc, rate, nq, seed):
    """Submits nq queries with Poisson arrivals at `rate` per second (graph
    uniform, source uniform in its pool), collects and releases every result;
    returns per-query latency (ms) and aggregate GTEPS."""
    import threading
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nq)
    which = rng.integers(0, len(gids), size=nq)
    picks = [int(pools[k][rng.integers(0, len(pools[k]))]) for k in which.tolist()]
    tickets = [None] * nq
    ready = threading.Semaphore(0)
    stats = [None] * nq

    def collect():
        for i in range(nq):
            ready.acquire()
            _, st = server.wait(tickets[i])
            server.release(tickets[i])
            stats[i] = st

    th = threading.Thread(target=collect)
    th.start()
    t0 = dsbfs.now_ns() + 2_000_000
    at = t0
    for i in range(nq):
        at += int(gaps[i] * 1e9)
        while True:
            now = dsbfs.now_ns()
            if now >= at:
                break
            if at - now > 300_000:
                time.sleep((at - now - 200_000) / 1e9)
        tickets[i] = server.submit(gids[which[i]], picks[i], at)
        ready.release()
    th.join()
    lat = np.array([(st["done_ns"] - st["arrival_ns"]) / 1e6 for st in stats])
    t_first = min(st["arrival_ns"] for st in stats)
    t_last = max(st["done_ns"] for st in stats)
    edges = sum(ncc[k] for k in which.tolist())
    lanes = sum(st["batched"] for st in stats) / nq
    return lat, edges / ((t_last - t_first) * 1e-9) / 1e9, lanes


def bench_served(args, torch, dsbfs, inputs):
    """Query stream over 5 resident graphs (RMAT 18/20/22/24 + ER 2^22 with
    8n pairs), Poisson arrivals at 0.5, 1 and 2 times the plain server's
    service rate, served plainly (one query at a time), with continuous
    batching, and adaptively (single-source searches while the queue is short,
    batches once it is long); p50/p99 latency and aggregate GTEPS per rate."""
    specs = [("rmat", int(x)) for x in args.serve_scales.split(",")] + [("er", 22)]
    built = []
    for kind, sc in specs:
        n = 1 << sc
        if kind == "rmat":
            src, dst = inputs.rmat_edges(sc)
        else:
            src, dst = inputs.er_edges(n, 8 * n, seed=0x22)
        built.append((kind, sc, n, src, dst))
    # Sources: uniform over the component of the highest-degree vertex (the
    # giant component), whose edge count is the GTEPS numerator of a query.
    pools, ncc = [], []
    for kind, sc, n, src, dst in built:
        g = dsbfs.Graph(src, dst, n, threshold=args.threshold, keep_plain_csr=False)
        ws = dsbfs.Workspace(g)
        deg = g.export(0, np.int32)
        d = torch.empty(n, dtype=torch.int32, device="cuda")
        r = dsbfs.bfs(g, ws, int(np.argmax(deg)), d, None, opts=dsbfs.run_opts(want_parent=False),
                      want_stats=True)
        reached = np.nonzero(d.cpu().numpy() >= 0)[0].astype(np.int32)
        pools.append(reached)
        ncc.append(r["edges_cc"])
        ws.destroy()
        g.destroy()
    nmax = max(b[2] for b in built)
    out = {"workload": "resident RMAT " + "/".join(str(b[1]) for b in built if b[0] == "rmat") +
                       " + ER 2^22 (8n pairs); Poisson single-source queries, graph uniform, "
                       "sources uniform over each graph's giant component",
           "queries_per_rate": args.serve_queries, "rates": []}
    servers = {}
    modes = {"plain": 0, "batched": 1, "adaptive": 2}
    for mode in modes:
        graphs = [dsbfs.Graph(src, dst, n, threshold=args.threshold, keep_plain_csr=True)
                  for _, _, n, src, dst in built]
        resident = sum(2 * (G.stats["bytes_layout"] + G.stats["bytes_plain"]) + 64 * G.n
                       for G in graphs)
        budget = resident + 4 * 64 * 4 * nmax
        S = dsbfs.Server(budget, max_lanes=64, batched=modes[mode])
        gids = [S.add_graph(G) for G in graphs]
        servers[mode] = (S, gids)
        out["hbm_budget_bytes"] = budget
    # plain service rate on this mix
    S, gids = servers["plain"]
    _poisson_run(dsbfs, S, gids, pools, ncc, 1e6, 256, 4999)
    t0 = dsbfs.now_ns()
    _poisson_run(dsbfs, S, gids, pools, ncc, 1e9, 512, 4998)
    mu = 512 / ((dsbfs.now_ns() - t0) * 1e-9)
    out["mu_plain_qps"] = round(mu, 1)
    log(f"plain service rate {mu:.0f} queries/s")
    for idx, f in enumerate((0.5, 1.0, 2.0)):
        row = {"rate_factor": f, "rate_qps": round(f * mu, 1)}
        for mode in modes:
            S, gids = servers[mode]
            lat, gteps, lanes = _poisson_run(dsbfs, S, gids, pools, ncc, f * mu,
                                             args.serve_queries, 5000 + idx)
            row[mode] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "gteps": round(gteps, 2), "share_as_lanes": round(lanes, 3)}
            log(f"rate {f} x mu, {mode}: p50 {row[mode]['p50_ms']} ms, "
                f"p99 {row[mode]['p99_ms']} ms, {row[mode]['gteps']} GTEPS")
        out["rates"].append(row)
    for S, _ in servers.values():
        S.destroy()
    return out


if __name__ == "__main__":
    main()
