#!/usr/bin/env python3
"""Benchmark: Brandes BC throughput (GTEPS) on one MI355X.

One step = one full BC run (every source of the workload: forward sigma pass,
reverse dependency pass, BC accumulation) over the resident graph, with the
graph and the output already in device memory when the timed region starts.

    GTEPS = k * nnz / t / 1e9     (k sources, nnz = CSR arcs = 2m)

Prints one JSON line (see the fields below).  `roofline` reports the dominant
kernel's algorithmic bytes per launch over its HIP-event-timed average launch
duration; `cpu_baseline` times the CPU oracle on a bounded sample of the same
workload on this host's cores.
"""
from __future__ import annotations

import argparse
import functools
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BC GTEPS (sources×2m/s) and HBM roofline %; batched vs per-source; p50/p99"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work (element-granular: each array element a
# kernel must touch, counted once per use), per execution path.  Units are the
# kernels' own work counters: owners, arcs, hits, and (batched path) vertices
# examined.
#   plain forward level kernel, per owner vertex: queue entry 4 + row_ptr
#     pair 8 + sigma write 8; per arc read: neighbour id 4 + level-code word 4;
#     per parent arc: parent sigma 8.
#   plain reverse level kernel, per owner vertex: queue entry 4 + row_ptr pair
#     8 + sigma 8 + c write 8 + BC read-modify-write 16; per arc: 4 + 4; per
#     child arc: child c 8.
#   batched forward kernel (64 sources per probe), per vertex examined:
#     visited mask 8 + row_ptr pair 8 + next-level mask write 8; per (vertex,
#     source) discovered: sigma write 8; per arc probed: neighbour id 4 +
#     frontier mask 8; per (arc, source) parent pair: parent sigma 8.
#   batched reverse kernel, per vertex examined: level mask 8 (the scan of F_L
#     that finds the level's vertices) + row_ptr pair 8; per (vertex, source)
#     at the level: sigma read 8 + c write 8 (delta, c and BC are completed in
#     the kernel); per arc probed: 4 + 8; per (arc, source) child pair: child
#     c 8.
BYTES = {
    ("plain", "forward"): {"owners": 20, "arcs": 8, "hits": 8},
    ("plain", "reverse"): {"owners": 44, "arcs": 8, "hits": 8},
    ("batched", "forward"): {"owners": 8, "arcs": 12, "hits": 8, "vertices": 24},
    ("batched", "reverse"): {"owners": 16, "arcs": 12, "hits": 8, "vertices": 16},
}
# sssp pass kernel: per pass, the stamp of every vertex 4; per vertex whose
# arcs are relaxed: row_ptr pair 8 + its distance 4; per arc relaxed:
# neighbour id 4 + weight 4 + neighbour distance 4; per improvement: atomic
# min 4 + stamp write 4.
SSSP_BYTES = {"vertex": 4, "owners": 12, "arcs": 12, "hits": 8}
# pagerank sum kernel, per iteration: per vertex row_ptr_in pair 8 + out-
# offsets pair 8 (out-degree) + rank read 8 + rank write 8 + share write 8;
# per arc: in-neighbour id 4 + its share 8.
PR_BYTES = {"vertex": 40, "arc": 12}
KERNELS = {
    ("plain", "forward"): "k_level_forward", ("plain", "reverse"): "k_level_reverse",
    ("batched", "forward"): "k_batch_forward", ("batched", "reverse"): "k_batch_reverse",
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2401_02472_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str, src_hash: str, width: int = 0):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel sources and, given a batch width, at that width
    (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*(\w+)", text)
    m_val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != src_hash:
        return None
    m_w = re.search(r"--batch-width (\d+)", text)
    if width and m_w and int(m_w.group(1)) != width:
        return None
    return float(m_val.group(1))


def traffic_point(traffic, avg_ms: float) -> dict:
    """The counter side of the roofline: fabric bytes per launch (from the
    committed counter summary) over the live average launch time, and its
    fraction of peak.  The L2's misses include MALL hits, so this bounds the
    HBM rate from above; well above `achieved` it measures over-fetch."""
    if traffic is None or avg_ms <= 0:
        return {"traffic_gbps": None, "traffic_frac": None}
    gbps = traffic / (avg_ms / 1e3) / 1e9
    return {"traffic_gbps": round(gbps, 1), "traffic_frac": round(gbps / HBM_PEAK_GBS, 4)}


def cpu_baseline(g, sources, target_s: float):
    import numpy as np

    import oracle

    threads = min(os.cpu_count() or 1, 16, oracle.max_threads())
    probe = sources[:1]
    directed = bool(g.params.get("directed"))
    run, kind = functools.partial(oracle.bc, directed=directed), "oracle"
    if directed:
        kind = "oracle (directed)"
    t = time.perf_counter()
    _, st = run(g.row_ptr, g.col_idx, probe, threads=1)
    if st == oracle.RANGE:  # counts beyond double: the long-double oracle
        run, kind = oracle.bc_ext, "oracle (extended range, long double)"
        t = time.perf_counter()
        run(g.row_ptr, g.col_idx, probe, threads=1)
    t1 = max(time.perf_counter() - t, 1e-6)
    m = int(max(threads, min(len(sources), round(target_s * threads / t1))))
    m = min(m, len(sources))
    sample = np.ascontiguousarray(sources[:m])
    t = time.perf_counter()
    run(g.row_ptr, g.col_idx, sample, threads=threads)
    dt = time.perf_counter() - t
    return {"value": round(m * g.nnz / dt / 1e9, 4), "unit": "GTEPS", "cores": threads,
            "kind": kind,
            "sample": f"first {m} of the {len(sources)} workload sources, {dt:.2f} s "
                      f"on {threads} threads",
            "one_thread_value": round(g.nnz / t1 / 1e9, 4),
            "one_thread_sample": f"first source on 1 thread, {t1:.2f} s"}


def profile_stride(g, s: int) -> int:
    """Level stride of the batched path's measurement: 1 up to 16 levels, else
    about 8 measured levels per pass (BFS depth from s by scipy)."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path

    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    dist = shortest_path(a, method="D", directed=bool(g.params.get("directed")), unweighted=True,
                         indices=[s])[0]
    d = int(dist[np.isfinite(dist)].max())
    return 1 if d <= 16 else max(1, d // 8)


def reached_arcs(g, sources):
    """Sum over the sources of the arcs leaving the vertices each one reaches
    (the degree sum of its connected component); None for a directed graph
    (reachability differs per source)."""
    if g.params.get("directed"):
        return None
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    _, label = connected_components(a, directed=False)
    comp_arcs = np.bincount(label, weights=g.degrees().astype(np.float64))
    return int(comp_arcs[label[np.asarray(sources, np.int64)]].sum())


def graphs_bench(args) -> int:
    """graphs-mix: 16 small R-MAT graphs (scales 10-12, edge factor 16, 64
    sources each) in one bc_run_graphs call per step (BC_LOOP_AUTO picks the
    graphs whose batches share one device-resident launch), against one
    bc_run_async call per graph (BC_MODE_AUTO) on the same sources.  GTEPS =
    sum of k * nnz over the graphs / step time."""
    import numpy as np
    import torch

    import graphgen as gg
    import paper_2401_02472_amd as bcm

    torch.cuda.set_device(0)
    bcm.load_library()
    graphs = [gg.rmat(sc, 16, seed=10 * sc + j) for sc in (10, 11, 12) for j in range(6)][:16]
    srcs = [gg.sample_sources(g, 64, seed=3) for g in graphs]
    Gs = [bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) for g in graphs]
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in graphs]
    work = sum(s.size * g.nnz for s, g in zip(srcs, graphs))
    auto = bcm.make_options(bcm.BC_MODE_AUTO)

    def one_call():
        return bcm.bc_run_graphs(Gs, srcs, outs, level_loop=bcm.BC_LOOP_AUTO)

    def per_graph():
        for G, src, o in zip(Gs, srcs, outs):
            G.run_async(src, o, auto)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t) * 1e3)
        return (time.perf_counter() - t0) * 1e3 / args.steps, ms

    loops = one_call()
    ms_step, step_ms = timed(one_call)
    ms_each, _ = timed(per_graph)
    q = np.percentile(step_ms, [50, 99])
    cpu = None
    if args.cpu_seconds > 0:  # the oracle over the graphs, one after another
        import oracle
        threads = min(os.cpu_count() or 1, 16, oracle.max_threads())
        t = time.perf_counter()
        done = 0
        for g, src in zip(graphs, srcs):
            oracle.bc(g.row_ptr, g.col_idx, src, threads=threads)
            done += src.size * g.nnz
            if time.perf_counter() - t > args.cpu_seconds:
                break
        dt = time.perf_counter() - t
        cpu = {"value": round(done / dt / 1e9, 4), "unit": "GTEPS", "cores": threads,
               "kind": "oracle", "sample": f"the graphs in order until {args.cpu_seconds} s, "
                                           f"{dt:.2f} s on {threads} threads"}
    rec = {
        "metric": METRIC, "value": round(work / (ms_step / 1e3) / 1e9, 3), "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "graphs-mix", "graphs": len(graphs), "scales": [10, 11, 12],
                   "edgefactor": 16, "sources_per_graph": 64, "level_loop": "auto",
                   "joined": int(sum(1 for x in loops if x == bcm.BC_LOOP_DEVICE))},
        "p50_ms": round(float(q[0]), 3), "p99_ms": round(float(q[1]), 3),
        "per_graph_calls": {"ms_per_step": round(ms_each, 3),
                            "gteps": round(work / (ms_each / 1e3) / 1e9, 3)},
        "roofline": None, "cpu_baseline": cpu,
    }
    for G in Gs:
        G.close()
    print(json.dumps(rec), flush=True)
    return 0


def serving_bench(args) -> int:
    """Serving mix: Poisson stream of BC requests over 16 resident R-MAT graphs
    (scales 14-20 with two seeds each, plus 21 and 22; edge factor 16); each
    request asks for k in {1, 8, 64} random sources of a uniformly chosen graph.
    Saturation throughput is measured with a burst first; Poisson streams then
    run at 0.5, 0.8 and 0.95 of it (the headline line is --serving-load), and
    once more under a small workspace budget that makes admission queue.
    Reports GTEPS (sum of k * nnz over the requests / wall time) and p50 / p99
    latency from arrival to the result on the host."""
    import numpy as np
    import torch

    import graphgen as gg
    import paper_2401_02472_amd as bcm
    from paper_2401_02472_amd.serving import BCServer

    torch.cuda.set_device(0)
    bcm.load_library()
    specs = [(sc, sd) for sc in range(14, 21) for sd in (1, 2)] + [(21, 1), (22, 1)]
    graphs, Gs = {}, {}
    for sc, sd in specs:
        gid = f"rmat-s{sc}-seed{sd}"
        print(f"# generating {gid}", file=sys.stderr, flush=True)
        g = gg.rmat(sc, 16, seed=sd)
        graphs[gid] = g
        Gs[gid] = bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC)
    gids = list(graphs)
    rng = np.random.default_rng(args.serving_seed)

    def make_request(i):
        gid = gids[int(rng.integers(len(gids)))]
        k = int(rng.choice([1, 8, 64]))
        return gid, gg.sample_sources(graphs[gid], k, seed=1000 + i)

    def poisson_run(srv, lam, reqs):
        """Submit `reqs` as a Poisson stream of rate lam; (wall s, latency stats)."""
        srv.completed.clear()
        t0 = time.perf_counter()
        arrival = t0
        futs = []
        for gid, src in reqs:
            arrival += float(rng.exponential(1.0 / lam))
            delay = arrival - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            futs.append(srv.submit(gid, src))
        for f in futs:
            f.result()
        return time.perf_counter() - t0, srv.latency_stats()

    budget = int(args.hbm_budget_gib) << 30
    srv = BCServer(Gs, budget=budget, slots=args.slots, max_lanes=256)
    # warm-up: every graph once (landmarks, level hints, workspaces), then
    # `serving_warmup` requests of the mix
    for gid in gids:
        srv.submit(gid, gg.sample_sources(graphs[gid], 64, seed=7)).result()
    for f in [srv.submit(gid, src) for gid, src in
              (make_request(50_000 + i) for i in range(args.serving_warmup))]:
        f.result()
    # saturation: a burst
    burst = [make_request(i) for i in range(args.serving_burst)]
    t = time.perf_counter()
    futs = [srv.submit(gid, src) for gid, src in burst]
    for f in futs:
        f.result()
    sat_dt = time.perf_counter() - t
    sat_rate = len(burst) / sat_dt
    sat_gteps = sum(src.size * graphs[gid].nnz for gid, src in burst) / sat_dt / 1e9
    print(f"# saturation {sat_rate:.1f} req/s, {sat_gteps:.1f} GTEPS", file=sys.stderr, flush=True)
    # Poisson streams at several fractions of saturation; the headline is
    # args.serving_load
    loads = sorted(set([0.5, 0.8, 0.95, args.serving_load]))
    per_load = {}
    stream_reqs = None
    for li, load in enumerate(loads):
        reqs = [make_request(100_000 * (li + 1) + i) for i in range(args.serving_requests)]
        wall_l, lat_l = poisson_run(srv, load * sat_rate, reqs)
        work_l = sum(src.size * graphs[gid].nnz for gid, src in reqs)
        per_load[str(load)] = {"gteps": round(work_l / wall_l / 1e9, 3),
                               "p50_ms": round(lat_l["p50_ms"], 3),
                               "p99_ms": round(lat_l["p99_ms"], 3),
                               "mean_ms": round(lat_l["mean_ms"], 3)}
        print(f"# load {load}: {per_load[str(load)]}", file=sys.stderr, flush=True)
        if load == args.serving_load:
            stream_reqs, wall, lat = reqs, wall_l, lat_l
    launches = srv.launches
    srv.close()
    # the same mix under a small workspace budget: admission queues launches
    # and frees idle graphs' pools.  Its own saturation (a burst under that
    # budget) sets the arrival rate: at the large budget's rate the small one
    # would be overloaded and the latencies would only measure the backlog.
    stress = None
    if args.serving_stress_gib > 0:
        srv2 = BCServer(Gs, budget=int(args.serving_stress_gib) << 30, slots=args.slots,
                        max_lanes=256)
        burst2 = [make_request(800_000 + i) for i in range(args.serving_burst)]
        t = time.perf_counter()
        for f in [srv2.submit(gid, src) for gid, src in burst2]:
            f.result()
        sat2_dt = time.perf_counter() - t
        sat2_rate = len(burst2) / sat2_dt
        sat2_gteps = sum(src.size * graphs[gid].nnz for gid, src in burst2) / sat2_dt / 1e9
        reqs = [make_request(900_000 + i) for i in range(args.serving_requests)]
        wall_s, lat_s = poisson_run(srv2, args.serving_load * sat2_rate, reqs)
        work_s = sum(src.size * graphs[gid].nnz for gid, src in reqs)
        stress = {"hbm_budget_gib": args.serving_stress_gib, "load": args.serving_load,
                  "saturation_gteps": round(sat2_gteps, 3),
                  "gteps": round(work_s / wall_s / 1e9, 3), "p50_ms": round(lat_s["p50_ms"], 3),
                  "p99_ms": round(lat_s["p99_ms"], 3), "max_reserved_gib":
                  round(srv2.max_reserved / 2**30, 2), "launches": srv2.launches,
                  "trims": srv2.trims}
        srv2.close()
    work = sum(src.size * graphs[gid].nnz for gid, src in stream_reqs)
    value = work / wall / 1e9
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        threads = min(os.cpu_count() or 1, 16, oracle.max_threads())
        sample = stream_reqs[:args.serving_cpu_sample]
        t = time.perf_counter()
        for gid, src in sample:
            oracle.bc(graphs[gid].row_ptr, graphs[gid].col_idx, src, threads=threads)
        dt = time.perf_counter() - t
        cpu = {"value": round(sum(s.size * graphs[g].nnz for g, s in sample) / dt / 1e9, 4),
               "unit": "GTEPS", "cores": threads, "kind": "oracle",
               "sample": f"first {len(sample)} requests of the stream, one after another, "
                         f"{dt:.2f} s on {threads} threads"}
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": len(stream_reqs), "warmup": len(gids) + args.serving_warmup,
        "ms_per_step": round(wall * 1e3 / len(stream_reqs), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "serving-mix", "graphs": len(gids), "edgefactor": 16,
                   "requests": len(stream_reqs), "k": [1, 8, 64], "arrivals": "poisson",
                   "load": args.serving_load, "slots": args.slots,
                   "hbm_budget_gib": args.hbm_budget_gib},
        "p50_ms": round(lat["p50_ms"], 3), "p99_ms": round(lat["p99_ms"], 3),
        "mean_latency_ms": round(lat["mean_ms"], 3),
        "saturation": {"requests_per_s": round(sat_rate, 2), "gteps": round(sat_gteps, 3)},
        "loads": per_load, "stress": stress,
        "launches": launches, "roofline": None, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    for G in Gs.values():
        G.close()
    return 0


def sssp_bench(args) -> int:
    """SSSP workload: the scale-22 R-MAT with weights in [1, 100] (seed 3); a step
    is one shortest-path run from each of --sssp-sources sampled sources.
    GTEPS = sources x arcs / time (the BC metric's convention)."""
    import numpy as np
    import torch

    import graphgen as gg
    import oracle
    import paper_2401_02472_amd as bcm

    torch.cuda.set_device(0)
    bcm.load_library()
    g, _ = gg.workload("rmat-s22-ef16")
    w = gg.edge_weights(g, seed=3)
    sources = gg.sample_sources(g, args.sssp_sources, seed=103)
    G = bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC)
    G.set_weights(w)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        for s in sources:
            G.sssp(int(s), out)
    torch.cuda.synchronize()
    G.profile_enable(1)
    G.profile_read(reset=True)
    step_ms = []
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        start.record(stream)
        for s in sources:
            G.sssp(int(s), out)
        stop.record(stream)
        stop.synchronize()
        step_ms.append(start.elapsed_time(stop))
    wall = time.perf_counter() - t0
    prof = G.profile_read(reset=True)
    G.profile_enable(False)
    ms_per_step = wall * 1e3 / args.steps
    value = len(sources) * g.nnz / (ms_per_step / 1e3) / 1e9
    pc = prof["sssp"]
    launches = max(pc["launches"], 1)
    alg = (SSSP_BYTES["vertex"] * g.n * pc["launches"] + SSSP_BYTES["owners"] * pc["owners"] +
           SSSP_BYTES["arcs"] * pc["arcs"] + SSSP_BYTES["hits"] * pc["hits"]) / launches
    avg_ms = pc["ms"] / launches
    achieved = alg / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    src_hash = kernel_source_hash()
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic("k_sssp_pass", "sssp-rmat-s22-ef16", src_hash),
            **traffic_point(read_traffic("k_sssp_pass", "sssp-rmat-s22-ef16", src_hash), avg_ms),
            "kernel": "k_sssp_pass", "alg_bytes_per_launch": int(alg),
            "avg_launch_ms": round(avg_ms, 5), "launches": pc["launches"],
            "passes_per_source": round(pc["launches"] / (args.steps * len(sources)), 2),
            "kernel_source_hash": src_hash}
    # the oracle (one thread: the fixed-point passes are sequential) on a prefix
    cpu = None
    if args.cpu_seconds > 0:
        t = time.perf_counter()
        m = 0
        for s in sources:
            oracle.sssp(g.row_ptr, g.col_idx, w, int(s))
            m += 1
            if time.perf_counter() - t > args.cpu_seconds:
                break
        dt = time.perf_counter() - t
        cpu = {"value": round(m * g.nnz / dt / 1e9, 4), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "sample": f"first {m} of the {len(sources)} sources, "
                                           f"{dt:.2f} s on one thread"}
    q = np.percentile(step_ms, [50, 99])
    rec = {
        "metric": "SSSP GTEPS (sources x arcs / s); HBM roofline", "value": round(value, 3),
        "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "sssp-rmat-s22-ef16", "n": g.n, "nnz": g.nnz,
                   "sources": len(sources), "weights": "uniform [1, 100] per edge, seed 3",
                   "graph": g.params},
        "p50_ms": round(float(q[0]), 3), "p99_ms": round(float(q[1]), 3),
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    G.close()
    return 0


def pagerank_bench(args) -> int:
    """PageRank workload: the scale-22 R-MAT; a step is one run of --pr-iterations
    iterations (damping 0.85, tol 0).  GTEPS = arcs x iterations / time."""
    import numpy as np
    import torch

    import graphgen as gg
    import oracle
    import paper_2401_02472_amd as bcm

    torch.cuda.set_device(0)
    bcm.load_library()
    g, _ = gg.workload("rmat-s22-ef16")
    iters = args.pr_iterations
    G = bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        G.pagerank(0.85, 0.0, iters, out)
    torch.cuda.synchronize()
    G.profile_enable(1)
    G.profile_read(reset=True)
    step_ms = []
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        start.record(stream)
        G.pagerank(0.85, 0.0, iters, out)
        stop.record(stream)
        stop.synchronize()
        step_ms.append(start.elapsed_time(stop))
    wall = time.perf_counter() - t0
    prof = G.profile_read(reset=True)
    G.profile_enable(False)
    ms_per_step = wall * 1e3 / args.steps
    value = iters * g.nnz / (ms_per_step / 1e3) / 1e9
    pc = prof["pagerank"]
    launches = max(pc["launches"], 1)
    alg = PR_BYTES["vertex"] * g.n + PR_BYTES["arc"] * g.nnz
    avg_ms = pc["ms"] / launches
    achieved = alg / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    src_hash = kernel_source_hash()
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic("k_pr_pull", "pagerank-rmat-s22-ef16", src_hash),
            **traffic_point(read_traffic("k_pr_pull", "pagerank-rmat-s22-ef16", src_hash), avg_ms),
            "kernel": "k_pr_pull", "alg_bytes_per_launch": int(alg),
            "avg_launch_ms": round(avg_ms, 5), "launches": pc["launches"],
            "kernel_source_hash": src_hash}
    cpu = None
    if args.cpu_seconds > 0:
        m = 3
        t = time.perf_counter()
        oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 0.0, m)
        dt = time.perf_counter() - t
        cpu = {"value": round(m * g.nnz / dt / 1e9, 4), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "sample": f"{m} iterations on one thread, {dt:.2f} s"}
    q = np.percentile(step_ms, [50, 99])
    rec = {
        "metric": "PageRank GTEPS (arcs x iterations / s); HBM roofline", "value": round(value, 3),
        "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "pagerank-rmat-s22-ef16", "n": g.n, "nnz": g.nnz,
                   "iterations": iters, "damping": 0.85, "graph": g.params},
        "p50_ms": round(float(q[0]), 3), "p99_ms": round(float(q[1]), 3),
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    G.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat-s22-ef16")
    ap.add_argument("--mode", default="auto", choices=["auto", "plain", "batched"])
    ap.add_argument("--batch-width", type=int, default=0)
    ap.add_argument("--sparse-div", type=int, default=0,
                    help="batched forward: sparse step below nnz/D frontier arcs (0 = the "
                         "graph's setting, -1 = never)")
    ap.add_argument("--sources", type=int, default=0, help="use only the first N sources")
    ap.add_argument("--group-cut", type=int, default=0,
                    help="batched work items: vertices above this degree become chunk items "
                         "(0 = the graph's setting)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="batched work items: arcs per chunk item (0 = the graph's setting)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target oracle CPU time for the cpu_baseline sample (0 = skip)")
    ap.add_argument("--compare-plain", type=int, default=32,
                    help="also time this many sources on the one-source-at-a-time path "
                         "(0 = skip) and report the ratio")
    ap.add_argument("--concurrency", type=int, default=0,
                    help="batches run at once (0 = the library's choice)")
    ap.add_argument("--level-loop", choices=("auto", "host", "device", "graph"), default="auto",
                    help="who drives the batched level loop (graph: the host loop with its "
                         "level chunks replayed as captured HIP graphs)")
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="skip the run with host transfers")
    ap.add_argument("--no-autotune", action="store_true",
                    help="auto mode: keep the library's default settings")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    ap.add_argument("--slots", type=int, default=4, help="serving: launches in flight")
    ap.add_argument("--hbm-budget-gib", type=int, default=64, help="serving: HBM budget")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-warmup", type=int, default=100)
    ap.add_argument("--serving-stress-gib", type=int, default=8,
                    help="serving: second run under this workspace budget (0 = skip)")
    ap.add_argument("--serving-burst", type=int, default=200)
    ap.add_argument("--serving-load", type=float, default=0.8)
    ap.add_argument("--serving-seed", type=int, default=105)
    ap.add_argument("--serving-cpu-sample", type=int, default=12)
    ap.add_argument("--sssp-sources", type=int, default=16,
                    help="sssp-rmat-s22-ef16: sources per step")
    ap.add_argument("--pr-iterations", type=int, default=20,
                    help="pagerank-rmat-s22-ef16: iterations per step")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path (sources would shard across GPUs, each holding the whole "
              "graph, with one all-reduce of BC at the end).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import graphgen as gg
    import paper_2401_02472_amd as bcm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.workload == "serving-mix":
        return serving_bench(args)
    if args.workload == "graphs-mix":
        return graphs_bench(args)
    if args.workload == "sssp-rmat-s22-ef16":
        return sssp_bench(args)
    if args.workload == "pagerank-rmat-s22-ef16":
        return pagerank_bench(args)
    torch.cuda.set_device(0)
    bcm.load_library()

    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    g, sources = gg.workload(args.workload)
    if args.sources:
        sources = sources[:args.sources]
    k = int(len(sources))
    mode = {"auto": bcm.BC_MODE_AUTO, "plain": bcm.BC_MODE_PLAIN,
            "batched": bcm.BC_MODE_BATCHED}[args.mode]
    loop = {"auto": bcm.BC_LOOP_AUTO, "host": bcm.BC_LOOP_HOST, "device": bcm.BC_LOOP_DEVICE,
            "graph": bcm.BC_LOOP_GRAPH}[args.level_loop]
    opt = bcm.make_options(mode, args.batch_width, sparse_div=args.sparse_div,
                           concurrency=args.concurrency, level_loop=loop)

    gflags = (bcm.BC_GRAPH_DIRECTED if g.params.get("directed")
              else bcm.BC_GRAPH_TRUST_SYMMETRIC)
    G = bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=gflags)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        print(f"# calibration copy of {args.calibrate_copy_mib} MiB done", file=sys.stderr,
              flush=True)

    tuning = None
    if mode == bcm.BC_MODE_AUTO and not args.no_autotune:
        # the library's own choice of batch width, sparse-step threshold and
        # plain / batched crossover, timed on the first 64 sources
        tuning = G.autotune(sources)
        print(f"# autotune: {tuning}", file=sys.stderr, flush=True)
    if args.group_cut or args.chunk:
        G.set_work_items(args.group_cut or 64, args.chunk or 512)
    # end to end in the paper's convention (before the warm-up, so that the
    # timed steps are the last runs in a profiler trace)
    end_to_end = None
    if not args.no_end_to_end:
        # host sources in, host BC out (one H2D of the sources, one D2H of BC),
        # and the one-time graph upload
        t = time.perf_counter()
        G2 = bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=gflags)
        create_ms = (time.perf_counter() - t) * 1e3
        G2.close()
        t = time.perf_counter()
        G.run(sources)
        run_host_ms = (time.perf_counter() - t) * 1e3
        end_to_end = {"run_host_ms": round(run_host_ms, 3), "create_graph_ms": round(create_ms, 3),
                      "gteps_with_transfers": round(k * g.nnz / (run_host_ms / 1e3) / 1e9, 3)}
    for _ in range(args.warmup):
        G.run_async(sources, out, opt)
    torch.cuda.synchronize()
    print(f"# warmup done: n={g.n} nnz={g.nnz} k={k}", file=sys.stderr, flush=True)

    min_batched = tuning["min_batched"] if tuning else 16
    path = "plain" if mode == bcm.BC_MODE_PLAIN or (mode == bcm.BC_MODE_AUTO and
                                                   k < min_batched) else "batched"
    # timed steps: the library's measurement hooks (events around launches,
    # work counters) are off
    G.profile_enable(False)
    step_ms = []
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        start.record(stream)
        G.run_async(sources, out, opt)
        stop.record(stream)
        stop.synchronize()
        step_ms.append(start.elapsed_time(stop))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = k * g.nnz / (ms_per_step / 1e3) / 1e9
    print(f"# timed {args.steps} steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    # measured steps (not part of `value`): events around the launches and the
    # kernels' work counters.  Event records are sampled so that they do not
    # slow short launches: the plain path measures every 16th source, the
    # batched host loop every stride-th level (all levels up to 16 deep; about
    # 8 per pass beyond).
    stride = 16 if path == "plain" else profile_stride(g, int(sources[0]))

    def measured(options, steps=2):
        G.profile_enable(stride)
        G.profile_read(reset=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            G.run_async(sources, out, options)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) * 1e3 / steps
        p = G.profile_read(reset=True)
        G.profile_enable(False)
        return p, dt, steps

    prof, meas_ms, meas_steps = measured(opt)
    levels_per_step = prof["levels"] / meas_steps

    src_hash = kernel_source_hash()
    # the batch width of the run (counter summaries taken at another width do
    # not describe its kernels)
    width = args.batch_width or (tuning["batch_width"] if tuning else 64)

    def roofline_of(prof, path, ms_step, steps):
        """Dominant kernel of a profile and its roofline point."""
        if prof["fused"]["launches"]:
            # device-resident level loop: one launch runs whole batches, forward
            # and reverse; its bytes are both passes' work counters
            pc = prof["fused"]
            alg_bytes = sum(BYTES[("batched", c)][u] * prof[c][u]
                            for c in ("forward", "reverse") for u in BYTES[("batched", c)])
            kernel_name = "k_batch_fused"
        else:
            cls = max(("forward", "reverse"), key=lambda c: prof[c]["ms"])
            pc = prof[cls]
            alg_bytes = sum(BYTES[(path, cls)][u] * pc[u] for u in BYTES[(path, cls)])
            kernel_name = KERNELS[(path, cls)]
        launches = max(pc["launches"], 1)
        avg_ms = pc["ms"] / launches
        per_launch = alg_bytes / launches
        achieved = per_launch / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
        # a kernel that runs alone takes at most the step's time: with the
        # launches of concurrent parts overlapping, it would not
        kernel_ms_step = pc["ms"] / steps
        assert kernel_ms_step <= ms_step * 1.001, (
            f"{kernel_name}: {kernel_ms_step:.3f} ms of launches per {ms_step:.3f} ms step")
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": read_traffic(kernel_name, args.workload, src_hash, width),
                **traffic_point(read_traffic(kernel_name, args.workload, src_hash, width), avg_ms),
                "kernel": kernel_name, "alg_bytes_per_launch": round(per_launch),
                "avg_launch_ms": round(avg_ms, 5), "launches": pc["launches"],
                "kernel_ms_per_step": round(kernel_ms_step, 3),
                "step_ms": round(ms_step, 3), "steps": steps,
                "kernel_source_hash": src_hash}

    if prof["fused"]["launches"]:
        path = "batched-device-loop"
    # The roofline point comes from steps run as one part: with concurrent
    # parts (batches on several streams) a launch's event duration also counts
    # the other parts' kernels running beside it, so it is not the kernel's own.
    one_part = path == "batched" and args.concurrency != 1
    if one_part:
        opt1 = bcm.make_options(mode, args.batch_width, sparse_div=args.sparse_div, concurrency=1,
                                level_loop=loop)
        roof_prof, roof_ms, roof_steps = measured(opt1)
    else:
        roof_prof, roof_ms, roof_steps = prof, meas_ms, meas_steps
    roofline = roofline_of(roof_prof, path, roof_ms, roof_steps)
    roofline["measured_as"] = "one part" if one_part else "the benchmarked configuration"

    plain_cmp = None
    if args.compare_plain and path.startswith("batched"):
        try:  # the one-source path computes in double, on undirected graphs
            G.single_source(int(sources[0]))
        except bcm.BCError as exc:
            if exc.status == bcm.BC_ERR_RANGE:
                plain_cmp = {"skipped": "path counts beyond double's range: the one-source-at-"
                                        "a-time path has no extended range"}
            elif exc.status == bcm.BC_ERR_UNSUPPORTED:
                plain_cmp = {"skipped": "directed graph: the one-source-at-a-time path is "
                                        "undirected only"}
            else:
                raise
    if args.compare_plain and path.startswith("batched") and plain_cmp is None:
        sub = np.asarray(sources[:args.compare_plain], np.int32)
        popt = bcm.make_options(bcm.BC_MODE_PLAIN)
        G.run_async(sub, out, popt)
        torch.cuda.synchronize()
        t = time.perf_counter()
        G.run_async(sub, out, popt)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t
        pg = len(sub) * g.nnz / pdt / 1e9
        plain_cmp = {"sources": int(len(sub)), "gteps": round(pg, 3),
                     "ms_per_source": round(pdt * 1e3 / len(sub), 4),
                     "batched_over_plain": round(value / pg, 3)}

    ra = reached_arcs(g, sources)

    cpu = None
    if args.cpu_seconds > 0:
        print("# timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(g, np.asarray(sources, np.int32), args.cpu_seconds)

    q = np.percentile(step_ms, [50, 99]) if step_ms else [0.0, 0.0]
    # per step, from the measured steps of the benchmarked configuration
    kernels = {c: {"launches": round(prof[c]["launches"] / meas_steps, 1),
                   "ms": round(prof[c]["ms"] / meas_steps, 3)}
               for c in ("forward", "compact", "reverse", "finish", "fused")}
    kernels["measured_step_ms"] = round(meas_ms, 3)
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "nnz": g.nnz, "sources": k,
                   "mode": args.mode, "path": path, "batch_width": args.batch_width or
                   ((tuning["batch_width"] if tuning else 64) if path.startswith("batched") else 1),
                   "sparse_div": args.sparse_div or (tuning["sparse_div"] if tuning else 64),
                   "group_cut": args.group_cut or (tuning["group_cut"] if tuning else 64),
                   "chunk": args.chunk or (tuning["chunk"] if tuning else 512),
                   "concurrency": args.concurrency, "level_loop": args.level_loop,
                   "autotune": tuning, "graph": g.params},
        "plain_comparison": plain_cmp,
        "profile_level_stride": stride,
        "level_steps_per_step": round(levels_per_step, 1),
        "per_level_us": round(ms_per_step * 1e3 / levels_per_step, 2) if levels_per_step else None,
        "reached_arc_gteps": None if ra is None else round(ra / (ms_per_step / 1e3) / 1e9, 3),
        "end_to_end": end_to_end,
        "p50_ms": round(float(q[0]), 3), "p99_ms": round(float(q[1]), 3),
        "roofline": roofline,
        "cpu_baseline": cpu, "kernels": kernels,
    }
    print(json.dumps(rec), flush=True)
    G.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
