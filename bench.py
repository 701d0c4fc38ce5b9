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

Also reported: the roofline of the dominant kernel (the oracle work model's
bytes for the profiled searches / the kernel's HIP-event time, with the
kernels' own byte counts beside it, and the measured HBM traffic per launch
from the committed rocprofv3 summary while the kernel's source is unchanged),
the CPU oracle timed on one host core on a bounded sample of the same
workload, the threshold and factor sweeps, the depth-only form, RMAT 16 and
22, and, unless switched off (0), the multi-source (--batched), served
(--served), PageRank (--pagerank-steps) and device-generated RMAT 28
(--big-scale) legs.

    python bench.py [--steps K] [--warmup W] [--scale S] [--threshold TH]
"""
from __future__ import annotations

import argparse
import ctypes
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


def measured_traffic(kernel, workload, source="bfs.hip"):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 summary in
    profiles/ (FETCH_SIZE + WRITE_SIZE runs, calibrated on a copy kernel), if
    one exists for this workload and for the current text of the kernel's
    source file (csrc/<source>); else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1803_03922_amd", "csrc", source)
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


def host_info():
    """nproc and CPU model of this host (for the CPU baseline)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model,
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def copy_peak(torch, nbytes=4 << 30, reps=10):
    """HBM bandwidth of a device-to-device copy (read + write bytes / time),
    the achievable peak to set the kernels' figures against."""
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


# library kernel names (dsbfs KERNEL_NAMES) of the work model's visits
VISIT_KERNEL = {"init": "init", "normal_frontier": "prev_normal", "delegate_previsit": "prev_deleg",
                "nd_forward": "td_normal", "deleg_forward": "td_deleg",
                "dn_backward": "bu_normal", "deleg_backward": "bu_deleg"}
KERNEL_SYMBOL = {"prev_normal": "k_normal_level", "td_normal": "k_td_nd",
                 "bu_normal": "k_bu_normal", "bu_deleg": "k_bu_deleg", "td_deleg": "k_td_deleg",
                 "prev_deleg": "k_prev_deleg", "close": "k_close", "init": "k_init",
                 "plain": "k_plain_expand"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps; one step = one search from each of the --sources sources")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--threshold", type=int, default=32)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--mode", choices=("do", "plain"), default="do")
    ap.add_argument("--model-sources", type=int, default=16,
                    help="sources of the profiled pass and of the work model (roofline)")
    ap.add_argument("--cpu-sources", type=int, default=2,
                    help="sources the CPU oracle times one by one on one core (0 = skip the "
                         "CPU leg: no cpu_baseline and no work-model roofline)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="threads for the oracle's other searches (untimed)")
    ap.add_argument("--no-parent", action="store_true")
    ap.add_argument("--configs", type=int, default=1,
                    help="1: also plain BFS at RMAT 16 and DOBFS at RMAT 22 (64 sources each)")
    ap.add_argument("--batched", type=int, default=1,
                    help="1: also measure multi-source BFS (RMAT scale --ms-scale, 1024 sources)")
    ap.add_argument("--ms-scale", type=int, default=24)
    ap.add_argument("--ms-sources", type=int, default=1024)
    ap.add_argument("--ms-single", type=int, default=1,
                    help="1 = time single-source DOBFS from the same sources beside the "
                         "multi-source launch; 0 = skip it (profiling runs)")
    ap.add_argument("--served", type=int, default=1,
                    help="1: also measure the query server (5 graphs, 3 Poisson rates)")
    ap.add_argument("--serve-queries", type=int, default=4096)
    ap.add_argument("--serve-scales", default="18,20,22,24")
    ap.add_argument("--factor-sweep", default="1e-8,1e-6,1e-4,1e-2,0.05,0.5,2,10",
                    help="comma-separated factor0 values tried for each of dd, dn, nd in turn "
                         "(the other two at their defaults); '' = none")
    ap.add_argument("--depth-only", type=int, default=1,
                    help="1 = also time the sources without the parent output; 0 = skip")
    ap.add_argument("--factor-steps", type=int, default=16,
                    help="sources timed per factor setting; 0 = no factor legs")
    ap.add_argument("--factor-grid", default="",
                    help="joint sweep: 'dd values;dn values;nd values', each comma-separated; "
                         "every combination is timed over --factor-steps sources")
    ap.add_argument("--pagerank-steps", type=int, default=20,
                    help="PageRank steps timed on the main graph (0 = skip)")
    ap.add_argument("--big-scale", type=int, default=28,
                    help="also generate, build and search RMAT at this scale on the device (0 = skip)")
    ap.add_argument("--big-sources", type=int, default=16)
    ap.add_argument("--th-sweep", default="16,32,64,128,256,512",
                    help="thresholds re-run on the same graph and sources ('' = none)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(more than one GPU is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1803_03922_amd import dsbfs, inputs

    torch.cuda.set_device(0)
    dev = torch.cuda.get_device_properties(0)
    log(f"device {dev.name} CUs={dev.multi_processor_count}")
    copy_gbs = copy_peak(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")

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

    def timed(gr, wsp, s, o, want_stats=False, out=None):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        d_, p_ = out if out is not None else (depth, parent)
        e0.record(stream)
        r = dsbfs.bfs(gr, wsp, int(s), d_, p_ if o.want_parent else None, opts=o,
                      want_stats=want_stats, capacity=64)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), r

    # The GTEPS numerator of a source (edges of its component) comes from an
    # untimed search with statistics; the timed searches run without them.
    edges_cc, nlev, sched = {}, {}, {}
    for s in sources.tolist():
        _, r = timed(g, ws, s, opts, want_stats=True)
        edges_cc[s], nlev[s] = r["edges_cc"], r["num_levels"]
        sched[s] = [lv["dir"] for lv in r["levels"]]
    for _ in range(args.warmup):
        for s in sources.tolist():
            timed(g, ws, s, opts)
    torch.cuda.synchronize()

    # timed region: K steps, each one search from every source
    times, rates, levels = [], [], []
    torch.cuda.synchronize()
    t_wall = time.time()
    for step in range(args.steps):
        for s in sources.tolist():
            ms, _ = timed(g, ws, s, opts)
            times.append(ms)
            rates.append(edges_cc[s] / (ms * 1e-3) / 1e9)
            levels.append(nlev[s])
        log(f"step {step + 1}/{args.steps}: {sum(times[-len(sources):]):.1f} ms, "
            f"harmonic {harmonic(rates[-len(sources):]):.1f} GTEPS")
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    value = harmonic(rates)
    ms_per_search = sum(times) / len(times)
    per_source_ms = {}
    for i, s in enumerate(sources.tolist() * args.steps):
        per_source_ms.setdefault(s, []).append(times[i])
    nominal = [(16 << args.scale) / (t * 1e-3) / 1e9 for t in times]
    tiny = [int(s) for s in sources.tolist() if edges_cc[s] * 1000 < max(edges_cc.values())]

    # Kernel breakdown: the model sources again with every kernel timed by HIP
    # events on the search's stream (direct launches instead of graphs).
    msrc = sources.tolist()[:args.model_sources]
    kern, ptimes, gpu_levels = {}, [], {}
    for s in msrc:
        ms, r = timed(g, ws, s, popts, want_stats=True)
        ptimes.append(ms)
        gpu_levels[s] = r["levels"]
        for name, k in r["kernels"].items():
            a = kern.setdefault(name, {"ms": 0.0, "launches": 0, "bytes": 0, "edges": 0})
            for f in a:
                a[f] += k[f]
    torch.cuda.synchronize()
    dname, dk = max(kern.items(), key=lambda kv: kv[1]["ms"])
    self_gbs = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9 if dk["ms"] > 0 else 0.0
    unprof_ms = sum(sum(per_source_ms[s]) / len(per_source_ms[s]) for s in msrc)

    def time_factors(f0, nn=None):
        o3 = dsbfs.run_opts(want_parent=parent is not None, factor0=f0, nn_do=nn is not None,
                            factor_nn=nn)
        # untimed: a change of nn_do captures new level graphs on the host
        timed(g, ws, int(sources[0]), o3)
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
    paper = None
    if mode == 1 and args.factor_steps > 0:
        gt, mss = time_factors(list(dsbfs.PAPER_FACTOR0))
        gtd, mssd = time_factors(base)
        paper = {"factor0": list(dsbfs.PAPER_FACTOR0), "gteps": gt, "ms_per_search": mss,
                 "default_factor0": base, "default_gteps": gtd, "default_ms_per_search": mssd,
                 "sources": args.factor_steps}
        log(f"paper factors {dsbfs.PAPER_FACTOR0}: {gt} GTEPS; default {base}: {gtd} GTEPS")
    # the same searches without the parent output (depths only, as the paper's
    # search produces), one pass over all sources
    depth_only = None
    if parent is not None and args.depth_only:
        o_np = dsbfs.run_opts(mode=mode, want_parent=False)
        timed(g, ws, int(sources[0]), o_np)   # untimed: captures the depth-only level graphs
        tt, rr = [], []
        for s in sources.tolist():
            ms, _ = timed(g, ws, s, o_np)
            tt.append(ms)
            rr.append(edges_cc[s] / (ms * 1e-3) / 1e9)
        depth_only = {"gteps": round(harmonic(rr), 3), "ms_per_search": round(sum(tt) / len(tt), 4),
                      "sources": len(tt)}
        log(f"depths only: {depth_only['gteps']} GTEPS")
    # the DO-on-nn variant (nn under the direction decision too), per nn factor
    nn_sweep = []
    for fnn in ((1e-6, 0.0), (1e-4, 0.0), (1e-3, 0.0), (1e-2, 0.0), (1.0, 0.0)) \
            if mode == 1 and args.factor_steps > 0 else ():
        gt, mss = time_factors(base, nn=fnn)
        nn_sweep.append({"factor0_nn": fnn[0], "factor1_nn": fnn[1], "gteps": gt,
                         "ms_per_search": mss})
        log(f"nn_do factor0_nn = {fnn[0]:g}: {gt} GTEPS")
    for ki, kname_f in enumerate(("dd", "dn", "nd")):
        for v in fvals if mode == 1 and args.factor_steps > 0 else []:
            f0 = list(base)
            f0[ki] = v
            gt, mss = time_factors(f0)
            fsweep.append({"kernel": kname_f, "factor0": v, "gteps": gt, "ms_per_search": mss})
            log(f"factor0[{kname_f}] = {v:g}: {gt} GTEPS")
    if args.factor_grid:
        import itertools
        axes = [[float(x) for x in part.split(",") if x.strip()]
                for part in args.factor_grid.split(";")]
        for f0 in itertools.product(*axes):
            gt, mss = time_factors(list(f0))
            fsweep.append({"factor0": list(f0), "gteps": gt, "ms_per_search": mss})
            log(f"factor0 = {list(f0)}: {gt} GTEPS, {mss} ms")

    # CPU leg: the oracle (test infrastructure) times its serial search on one
    # core, and its work model gives the algorithmic bytes of the same
    # searches the profiled pass timed.
    cpu, model = None, None
    if args.cpu_sources > 0:
        cpu, model = cpu_leg(args, src, dst, n, sources, msrc, opts, gpu_levels, dsbfs, g, ws,
                             depth, parent, torch)

    roofline = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernel": dname,
                "launches_per_source": dk["launches"] / len(msrc),
                "avg_launch_ms": dk["ms"] / max(dk["launches"], 1),
                "self_counted": {"bytes_per_launch": dk["bytes"] / max(dk["launches"], 1),
                                 "achieved": round(self_gbs, 2)},
                "copy_peak_gbs": round(copy_gbs, 1)}
    if model is not None:
        mb = model["kernel_bytes"].get(dname, 0.0)
        ach = mb / (dk["ms"] * 1e-3) / 1e9 if dk["ms"] > 0 else 0.0
        roofline.update({"achieved": round(ach, 2), "frac": round(ach / HBM_PEAK_GBS, 5),
                         "frac_of_copy": round(ach / copy_gbs, 5),
                         "algorithmic_bytes_per_launch": mb / max(dk["launches"], 1),
                         "bytes_source": "oracle work model over the profiled searches"})
    else:
        roofline.update({"achieved": round(self_gbs, 2), "frac": round(self_gbs / HBM_PEAK_GBS, 5),
                         "bytes_source": "kernels' own work counts (no CPU leg)"})
    # traffic per launch over the same searches as avg_launch_ms: the model
    # sources (the picker draws in sequence, so the first k of any larger pick)
    wl = f"RMAT{args.scale} TH{args.threshold} {args.mode} {len(msrc)}src parents={int(parent is not None)}"
    tr = measured_traffic(KERNEL_SYMBOL[dname], wl)
    roofline["traffic"] = None if tr is None else round(tr, 0)
    roofline["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"

    pr = bench_pagerank(args, torch, dsbfs, g, n) if args.pagerank_steps and mode == 1 else None
    del ws, g
    torch.cuda.empty_cache()
    sweep = []
    for th in [int(x) for x in args.th_sweep.split(",") if x.strip()] if mode == 1 else []:
        gs = dsbfs.Graph(src, dst, n, threshold=th, keep_plain_csr=False)
        wss = dsbfs.Workspace(gs)
        o2 = dsbfs.run_opts(want_parent=parent is not None)
        tt, rr, byts = [], [], 0
        for s in sources.tolist():
            _, r = timed(gs, wss, s, o2, want_stats=True)   # untimed: numerator and bytes
            ms, _ = timed(gs, wss, s, o2)
            tt.append(ms)
            rr.append(r["edges_cc"] / (ms * 1e-3) / 1e9)
            byts += sum(k["bytes"] for k in r["kernels"].values())
        gst = gs.stats
        sweep.append({"threshold": th, "gteps": round(harmonic(rr), 3),
                      "ms_per_search": round(sum(tt) / len(tt), 4),
                      "self_counted_gbs": round(byts / (sum(tt) * 1e-3) / 1e9, 2),
                      "d": gst["d"], "d_frac": round(gst["d"] / n, 5),
                      "e_nn": gst["e_nn"], "e_nd": gst["e_nd"],
                      "e_dn": gst["e_dn"], "e_dd": gst["e_dd"],
                      "bytes_layout": gst["bytes_layout"]})
        log(f"TH {th}: {sweep[-1]['gteps']} GTEPS, d={gst['d']}")
        wss.destroy()
        gs.destroy()
    want_parent = parent is not None
    del depth, parent, src, dst
    torch.cuda.empty_cache()
    configs = bench_configs(args, torch, dsbfs, inputs) if args.configs else None
    torch.cuda.empty_cache()
    batched = bench_batched(args, torch, dsbfs, inputs) if args.batched else None
    torch.cuda.empty_cache()
    served = bench_served(args, torch, dsbfs, inputs) if args.served else None
    torch.cuda.empty_cache()
    big = bench_big(args, torch, dsbfs, inputs) if args.big_scale else None

    line = {
        "metric": "GTEPS (harmonic mean, 1 GPU) + p50/p99 query latency, batched vs plain BFS",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sum(times) / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"single-source {'DOBFS' if args.mode == 'do' else 'top-down BFS'}"
                               f", RMAT scale {args.scale} edge factor 16, TH {args.threshold}; "
                               f"one step = one search from each of {len(sources)} sources",
                   "scale": args.scale, "threshold": args.threshold, "sources": len(sources),
                   "sources_timed": len(sources), "searches_timed": len(times),
                   "parents": want_parent, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "work_model": model,
        "th_sweep": sweep,
        "depth_only": depth_only,
        "factors": {"paper_vs_default": paper, "sweep": fsweep, "nn_do": nn_sweep},
        "configs": configs,
        "batched": batched,
        "served": served,
        "device_generated": big,
        "pagerank": pr,
        "detail": {
            "ms_per_search": round(ms_per_search, 4),
            "gteps_geometric": round(geometric(rates), 3),
            "gteps_nominal_geometric": round(geometric(nominal), 3),
            "sources_in_tiny_components": tiny,
            "levels_mean": sum(levels) / len(levels),
            "kernel_ms_per_search": {k: round(v["ms"] / len(msrc), 4) for k, v in kern.items()},
            "kernel_launches_per_search": {k: v["launches"] / len(msrc) for k, v in kern.items()},
            "kernel_self_counted_gbs": {k: round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
                                        for k, v in kern.items() if v["ms"] > 0},
            "kernel_share_profiled": round(sum(k["ms"] for k in kern.values()) / sum(ptimes), 3),
            "ms_per_search_profiled": round(sum(ptimes) / len(ptimes), 4),
            "ms_per_search_unprofiled_same_sources": round(unprof_ms / len(msrc), 4),
            "graph": st, "build_s": round(build_s, 2), "timed_wall_s": round(wall, 2),
            "host": host_info(),
        },
    }
    print(json.dumps(line), flush=True)


def cpu_leg(args, src, dst, n, sources, msrc, opts, gpu_levels, dsbfs, g, ws, depth, parent,
            torch):
    """The oracle's serial search timed on one core (cpu_baseline), and its work
    model of the profiled searches (algorithmic bytes per kernel)."""
    import concurrent.futures as cf

    import oracle
    oracle.build(force=False)
    t0 = time.time()
    O = oracle.Graph(src, dst, n)
    log(f"oracle CSR built in {time.time() - t0:.1f}s (untimed)")
    deg = O.degrees()
    rows, crates, csecs = {}, [], []
    timed_src = sources.tolist()[:args.cpu_sources]
    for s in timed_src:
        c0 = time.perf_counter()
        dref, _ = O.bfs(int(s), want_parent=False)
        c1 = time.perf_counter()
        m_cc = int(deg[dref >= 0].sum() // 2)
        crates.append(m_cc / (c1 - c0) / 1e9)
        csecs.append(c1 - c0)
        if s in msrc:
            rows[s] = dref
        log(f"oracle BFS s={s}: {c1 - c0:.2f}s, {crates[-1]:.3f} GTEPS")
    # one GPU row against the oracle's (the GPU tests check every source)
    s0 = timed_src[0]
    dsbfs.bfs(g, ws, int(s0), depth, None, opts=dsbfs.run_opts(want_parent=False))
    torch.cuda.synchronize()
    d0 = rows.get(s0)
    if d0 is None:
        d0, _ = O.bfs(int(s0), want_parent=False)
    assert np.array_equal(depth.cpu().numpy(), d0), "GPU depth != oracle depth"
    host = host_info()
    cpu = {"value": round(harmonic(crates), 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
           "sample": f"{len(crates)} of the {len(sources)} sources, one after another, serial "
                     f"FIFO BFS on one host thread ({sum(csecs):.1f} s), CSR build untimed",
           "nproc": host["nproc"], "cpu_model": host["cpu_model"]}

    rest = [s for s in msrc if s not in rows]
    with cf.ThreadPoolExecutor(max_workers=args.cpu_threads) as ex:
        for s, r in zip(rest, ex.map(lambda s: O.bfs(int(s), want_parent=False)[0], rest)):
            rows[s] = r
    t0 = time.time()
    W = oracle.WorkModel(O, args.threshold)
    log(f"work model rows prepared in {time.time() - t0:.1f}s")
    f0, f1 = list(opts.factor0), list(opts.factor1)
    want_parent = parent is not None

    def one(s):
        return s, W.run(rows[s], f0, f1, want_parent=want_parent)

    kb, lv_count, sched_ok = {}, {}, True
    with cf.ThreadPoolExecutor(max_workers=args.cpu_threads) as ex:
        for s, (lv, B, La) in ex.map(one, msrc):
            for visit, b in B.items():
                k = VISIT_KERNEL[visit]
                kb[k] = kb.get(k, 0.0) + b
                lv_count[k] = lv_count.get(k, 0) + La[visit]
            gl = gpu_levels[s]
            if len(gl) != len(lv) or any(a["dir"] != b["dir"] for a, b in zip(gl, lv)):
                sched_ok = False
    del O, W
    total = sum(kb.values())
    model = {"sources": len(msrc), "kernel_bytes": kb, "kernel_levels_with_work": lv_count,
             "bytes_per_search": total / len(msrc),
             "schedule_equals_gpu": sched_ok,
             "path_gbs": None}
    log(f"work model: {total / len(msrc) / 1e9:.3f} GB per search; schedule "
        f"{'equals' if sched_ok else 'DIFFERS FROM'} the GPU's")
    return cpu, model


def bench_configs(args, torch, dsbfs, inputs):
    """The small configurations: plain top-down BFS on RMAT 16 (plain CSR) and
    degree-separated DOBFS on RMAT 22 (TH 32), 64 sources each, with the
    oracle's serial search timed beside them on the same sources."""
    import oracle
    oracle.build(force=False)
    out = []
    for scale, mode, seed, th in ((16, 0, 1001, 32), (22, 1, 1002, 32)):
        n = 1 << scale
        src, dst = inputs.rmat_edges(scale)
        sources = inputs.pick_sources(src, dst, n, 64, seed=seed)
        g = dsbfs.Graph(src, dst, n, threshold=th, keep_plain_csr=mode == 0)
        ws = dsbfs.Workspace(g)
        d = torch.empty(n, dtype=torch.int32, device="cuda")
        p = torch.empty(n, dtype=torch.int32, device="cuda")
        o = dsbfs.run_opts(mode=mode, want_parent=True)
        stream = torch.cuda.current_stream()
        ecc = {s: dsbfs.bfs(g, ws, s, d, p, opts=o, want_stats=True)["edges_cc"]
               for s in sources.tolist()}
        for s in sources.tolist():   # warm-up
            dsbfs.bfs(g, ws, s, d, p, opts=o)
        tt, rr = [], []
        for s in sources.tolist():
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dsbfs.bfs(g, ws, s, d, p, opts=o)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            tt.append(ms)
            rr.append(ecc[s] / (ms * 1e-3) / 1e9)
        O = oracle.Graph(src, dst, n)
        deg = O.degrees()
        crates = []
        for s in sources.tolist()[:4]:
            c0 = time.perf_counter()
            dref, _ = O.bfs(int(s), want_parent=False)
            c1 = time.perf_counter()
            crates.append(int(deg[dref >= 0].sum() // 2) / (c1 - c0) / 1e9)
        big = max(ecc.values())
        tiny = [int(s) for s in sources.tolist() if ecc[s] * 1000 < big]
        rows = [r for s, r in zip(sources.tolist(), rr) if ecc[s] * 1000 >= big]
        out.append({"workload": f"RMAT scale {scale}, {'plain top-down BFS' if mode == 0 else f'DOBFS TH {th}'}"
                                f", parents, 64 sources",
                    "gteps_harmonic": round(harmonic(rr), 3),
                    "gteps_geometric": round(geometric(rr), 3),
                    "gteps_harmonic_giant_component": round(harmonic(rows), 3),
                    "sources_in_tiny_components": tiny,
                    "ms_per_search": round(sum(tt) / len(tt), 4),
                    "oracle_gteps": round(harmonic(crates), 4),
                    "oracle_sample": "4 sources, serial FIFO BFS on one host thread"})
        log(f"RMAT {scale} mode {mode}: {out[-1]['gteps_harmonic']} GTEPS harmonic "
            f"({out[-1]['gteps_harmonic_giant_component']} without {len(tiny)} tiny-component "
            f"sources), oracle {out[-1]['oracle_gteps']}")
        del O
        ws.destroy()
        g.destroy()
    return out


def bench_pagerank(args, torch, dsbfs, g, n):
    """PageRank (alpha 0.85) on the degree-separated layout of the main graph:
    --pagerank-steps FP64 power-iteration steps in one call, HIP-event timed;
    algorithmic bytes per step 12 m + 40 n + 28 d (column and gathered
    contribution per directed edge; rank, degree, delegate ID, contribution,
    offsets and new rank per vertex; delegate state, offsets and vertex per
    delegate)."""
    st = g.stats
    rank = torch.empty(n, dtype=torch.float64, device="cuda")
    dsbfs.pagerank(g, rank, iterations=2)   # warm-up
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    steps, delta = dsbfs.pagerank(g, rank, iterations=args.pagerank_steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    b = 12 * st["m_dir"] + 40 * st["n"] + 28 * st["d"]
    ach = b / (ms * 1e-3) / 1e9
    out = {"workload": f"PageRank alpha 0.85, FP64, RMAT scale {args.scale} TH {args.threshold}, "
                       f"{steps} steps in one call",
           "ms_per_step": round(ms, 4), "gedges_per_s": round(st["m_dir"] / (ms * 1e-3) / 1e9, 2),
           "last_l1_change": delta,
           "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
                        "algorithmic_bytes_per_step": b}}
    log(f"pagerank: {ms:.2f} ms per step, {ach:.0f} GB/s algorithmic")
    del rank
    return out


def bench_big(args, torch, dsbfs, inputs):
    """RMAT at --big-scale generated and built on the device (the edge list
    never exists on the host or in HBM), then single-source DOBFS with
    parents from --big-sources seeded sources (picked from the degree array,
    the same sources as from the edge list)."""
    scale = args.big_scale
    n = 1 << scale
    stream = torch.cuda.current_stream()
    t0 = time.time()
    g = dsbfs.Graph(None, None, 0, threshold=args.threshold, keep_plain_csr=False,
                    rmat=dsbfs.rmat_spec(scale))
    torch.cuda.synchronize()
    build_s = time.time() - t0
    st = g.stats
    log(f"RMAT {scale} generated and built on the device in {build_s:.1f}s: m_dir={st['m_dir']}")
    sources = inputs.pick_sources_deg(g.export(0, np.int32), args.big_sources, 1005)
    ws = dsbfs.Workspace(g)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    o = dsbfs.run_opts(want_parent=True)
    ecc = {s: dsbfs.bfs(g, ws, int(s), depth, parent, opts=o, want_stats=True)["edges_cc"]
           for s in sources.tolist()}
    tt, rr = [], []
    for s in sources.tolist():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dsbfs.bfs(g, ws, int(s), depth, parent, opts=o)
        e1.record(stream)
        e1.synchronize()
        tt.append(e0.elapsed_time(e1))
        rr.append(ecc[s] / (tt[-1] * 1e-3) / 1e9)
    out = {"workload": f"RMAT scale {scale} edge factor 16, TH {args.threshold}, generated and "
                       f"built on the device; single-source DOBFS with parents, "
                       f"{len(sources)} sources",
           "build_s": round(build_s, 2), "gteps_harmonic": round(harmonic(rr), 3),
           "gteps_geometric": round(geometric(rr), 3),
           "ms_per_search": round(sum(tt) / len(tt), 4), "m_dir": st["m_dir"], "d": st["d"],
           "bytes_layout": st["bytes_layout"],
           "device_bytes_in_use": torch.cuda.memory_allocated()}
    log(f"RMAT {scale}: {out['gteps_harmonic']} GTEPS harmonic, {out['ms_per_search']} ms")
    ws.destroy()
    g.destroy()
    return out


def bench_batched(args, torch, dsbfs, inputs):
    """Multi-source BFS: all sources in one persistent, graph-captured launch,
    at the tuner's lane width and at 64 lanes per batch (16 batches of 64),
    against single-source DOBFS from the same sources on the same graph (depth
    only on both sides). The roofline of each launch comes from the oracle's
    multi-source work model (CPU leg)."""
    scale = args.ms_scale
    n = 1 << scale
    src, dst = inputs.rmat_edges(scale)
    g = dsbfs.Graph(src, dst, n, threshold=args.threshold, keep_plain_csr=True)
    sources = inputs.pick_sources(src, dst, n, args.ms_sources, seed=1004)
    ws = dsbfs.Workspace(g, max_lanes=64)
    t0 = time.time()
    tuned = dsbfs.msbfs_tune(g, ws, sources)   # times candidates on one batch
    log(f"msbfs tuned in {time.time() - t0:.1f}s: {tuned.as_dict()}")
    k = len(sources)
    depth = torch.empty((k, n), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    shapes = {}
    narrow = dsbfs.dsbfs_ms_opts(tuned.block, tuned.blocks_per_cu, tuned.bu_permille,
                                 tuned.use_graph, 64)
    for name, o in (("tuned", tuned), ("64_lanes", narrow)):
        dsbfs.msbfs(g, ws, sources, depth, o)   # warm-up (and graph capture)
        torch.cuda.synchronize()
        ts = []
        for _ in range(2):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dsbfs.msbfs(g, ws, sources, depth, o)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        lanes = o.lanes_per_batch or (64 if k <= 64 else 128 if k <= 128 else 256)
        shapes[name] = {"lanes_per_batch": lanes, "batches": (k + lanes - 1) // lanes,
                        "launch_ms": round(min(ts), 3), "launch_ms_runs": [round(t, 3) for t in ts],
                        "opts": o.as_dict()}
        log(f"msbfs {name}: {k} sources, {lanes} lanes per batch, {min(ts):.1f} ms")
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
    tot_ms, tot_e = 0.0, sum(ecc[s] for s in sources.tolist())
    for s in sources.tolist() if args.ms_single else ():
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dsbfs.bfs(g, ws, s, d1, None, opts=o1)
        b.record(stream)
        b.synchronize()
        tot_ms += a.elapsed_time(b)
    log(f"single-source DOBFS: {tot_ms:.1f} ms total")
    ws.destroy()
    g.destroy()
    for name, sh in shapes.items():
        sh["gteps"] = round(tot_e / (sh["launch_ms"] * 1e-3) / 1e9, 2)
        sh["speedup_vs_single_source"] = round(tot_ms / sh["launch_ms"], 2) if tot_ms else None
        o = sh["opts"]
        wl = (f"RMAT{scale} {k}src lanes={sh['lanes_per_batch']} block={o['block']} "
              f"bpc={o['blocks_per_cu']} bu={o['bu_permille']}")
        sh["traffic"] = measured_traffic("k_msbfs", wl, "msbfs.hip")
    if args.cpu_sources > 0:
        cpu_leg_batched(src, dst, n, sources, shapes)
    for sh in shapes.values():
        if "roofline" in sh:
            sh["roofline"]["traffic"] = sh.pop("traffic")
            sh["roofline"]["traffic_unit"] = ("bytes per launch (rocprofv3 FETCH_SIZE + "
                                              "WRITE_SIZE, calibrated)")
    t = shapes["tuned"]
    out = {"workload": f"RMAT scale {scale}, {k} sources in one persistent graph-captured launch",
           "value": t["gteps"], "unit": "GTEPS (aggregate)", "launch_ms": t["launch_ms"],
           "plain_gteps": round(tot_e / (tot_ms * 1e-3) / 1e9, 2) if tot_ms else None,
           "plain_ms_total": round(tot_ms, 2), "speedup": t["speedup_vs_single_source"],
           "shapes": shapes}
    return out


def cpu_leg_batched(src, dst, n, sources, shapes):
    """CPU leg of the multi-source bench: the oracle's work model of every
    batch of each launch shape (algorithmic bytes), for the launch's roofline."""
    import concurrent.futures as cf

    import oracle
    oracle.build(force=False)
    t0 = time.time()
    O = oracle.Graph(src, dst, n)
    for name, sh in shapes.items():
        lanes, permille = sh["lanes_per_batch"], sh["opts"]["bu_permille"]
        batches = [sources[i:i + lanes] for i in range(0, len(sources), lanes)]
        # or_ms_work parallelizes each batch itself
        with cf.ThreadPoolExecutor(max_workers=1) as ex:
            res = list(ex.map(lambda b: O.ms_work(b, permille), batches))
        total = sum(b for _, b, _ in res)
        ach = total / (sh["launch_ms"] * 1e-3) / 1e9
        sh["roofline"] = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
                          "algorithmic_bytes": total,
                          "levels_per_batch": [len(lv) for lv, _, _ in res],
                          "bytes_source": "oracle multi-source work model"}
        log(f"msbfs {name}: work model {total / 1e9:.2f} GB, {ach:.0f} GB/s algorithmic "
            f"({time.time() - t0:.1f}s)")
    del O


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
        # Results are released as they complete, not in submission order:
        # under a budget that binds, a finished result held while waiting for
        # an earlier query that needs its memory would wait for ever.
        p = ctypes.c_void_p()
        qs = dsbfs.dsbfs_query_stats()
        nxt, left, outstanding = 0, nq, []
        while left:
            while ready.acquire(blocking=False):
                outstanding.append(nxt)
                nxt += 1
            if not outstanding:
                ready.acquire()
                outstanding.append(nxt)
                nxt += 1
            keep = []
            for i in outstanding:
                st = dsbfs.dsbfs_server_wait(server.h, tickets[i], 0, ctypes.byref(p),
                                             ctypes.byref(qs))
                if st == dsbfs.OK:
                    stats[i] = {k: int(getattr(qs, k)) for k, _ in qs._fields_}
                    server.release(tickets[i])
                    left -= 1
                elif st == dsbfs.ERR_NOT_READY:
                    keep.append(i)
                else:
                    dsbfs.check(st, "dsbfs_server_wait")
            if len(keep) == len(outstanding):
                time.sleep(50e-6)
            outstanding = keep

    # short thread switches: the polling collector and the submitter share the GIL
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
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
    sys.setswitchinterval(switch)
    lat = np.array([(st["done_ns"] - st["arrival_ns"]) / 1e6 for st in stats])
    t_first = min(st["arrival_ns"] for st in stats)
    t_last = max(st["done_ns"] for st in stats)
    edges = sum(ncc[k] for k in which.tolist())
    lanes = sum(st["batched"] for st in stats) / nq
    waited = sum(st["waited_budget"] for st in stats) / nq
    return lat, edges / ((t_last - t_first) * 1e-9) / 1e9, lanes, waited


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
    out["hbm_budget_bytes"] = {}
    for mode in modes:
        # the exact resident footprint of the mix in this mode, from a server
        # with room for everything; the budget then leaves room for four
        # 64-lane blocks of result rows at the largest graph, more than the
        # five graphs' cohorts hold at once (the rate runs are not limited by
        # memory; the tight-budget run below is)
        probe = dsbfs.Server(1 << 50, max_lanes=64, batched=modes[mode])
        for _, _, n, src, dst in built:
            probe.add_graph(dsbfs.Graph(src, dst, n, threshold=args.threshold,
                                        keep_plain_csr=True))
        resident = probe.stats()["used_bytes"]
        probe.destroy()
        budget = resident + 4 * 64 * 4 * nmax
        S = dsbfs.Server(budget, max_lanes=64, batched=modes[mode])
        gids = [S.add_graph(dsbfs.Graph(src, dst, n, threshold=args.threshold,
                                        keep_plain_csr=True))
                for _, _, n, src, dst in built]
        assert S.stats()["resident_graphs"] == len(built)
        servers[mode] = (S, gids)
        out["hbm_budget_bytes"][mode] = {"budget": budget, "resident_graphs_bytes": resident}
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
            st0 = S.stats()
            lat, gteps, lanes, waited = _poisson_run(dsbfs, S, gids, pools, ncc, f * mu,
                                                     args.serve_queries, 5000 + idx)
            st1 = S.stats()
            row[mode] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "gteps": round(gteps, 2), "share_as_lanes": round(lanes, 3),
                         "budget_waits": st1["budget_waits"] - st0["budget_waits"],
                         "share_waited_budget": round(waited, 4),
                         "graph_loads": st1["loads"] - st0["loads"],
                         "graph_evictions": st1["evictions"] - st0["evictions"]}
            log(f"rate {f} x mu, {mode}: p50 {row[mode]['p50_ms']} ms, "
                f"p99 {row[mode]['p99_ms']} ms, {row[mode]['gteps']} GTEPS, "
                f"{row[mode]['budget_waits']} waited for budget")
        out["rates"].append(row)
    for S, _ in servers.values():
        S.destroy()
    # Admission under budgets that bind: batched serving at 2 x mu_plain with
    # room for 16 and for 8 result rows of the largest graph (1.07 / 0.54 GB
    # at RMAT 24), against about 35 rows of 21 MB on average in flight at
    # that rate: queries wait for memory at admission (oldest first).
    resident = out["hbm_budget_bytes"]["batched"]["resident_graphs_bytes"]
    out["tight_budget"] = []
    for rows in (16, 8):
        budget = resident + rows * 4 * nmax
        S = dsbfs.Server(budget, max_lanes=64, batched=1)
        gids = [S.add_graph(dsbfs.Graph(src, dst, n, threshold=args.threshold,
                                        keep_plain_csr=True))
                for _, _, n, src, dst in built]
        st0 = S.stats()
        lat, gteps, lanes, waited = _poisson_run(dsbfs, S, gids, pools, ncc, 2.0 * mu,
                                                 args.serve_queries, 5002)
        st1 = S.stats()
        tb = {"mode": "batched", "rate_factor": 2.0, "rows_of_largest": rows, "budget": budget,
              "room_for_rows_bytes": budget - resident,
              "p50_ms": round(float(np.percentile(lat, 50)), 3),
              "p99_ms": round(float(np.percentile(lat, 99)), 3),
              "gteps": round(gteps, 2),
              "budget_waits": st1["budget_waits"] - st0["budget_waits"],
              "share_waited_budget": round(waited, 4)}
        out["tight_budget"].append(tb)
        log(f"budget with room for {rows} rows ({(budget - resident) / 1e9:.2f} GB), 2 x mu, "
            f"batched: p50 {tb['p50_ms']} ms, p99 {tb['p99_ms']} ms, "
            f"{tb['budget_waits']} waited for budget")
        S.destroy()
    return out


if __name__ == "__main__":
    main()
