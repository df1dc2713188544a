#!/usr/bin/env python
"""Benchmark of the Brandes betweenness-centrality hot path on one MI355X.

Default workload: directed R-MAT graph, scale 20 (n = 1,048,576), edge factor 16, quadrant
split (0.57, 0.19, 0.19, 0.05), self-loops and repeated pairs removed, seed 20; BC from 1,024
sources drawn uniformly without replacement (seed 2020), FP64 output, exact path counts.  One
step = one sampled-BC pass over those sources (forward sweep, backward sweep, accumulation for
each) with the graph already resident in HBM.  The same run also times the 1024 x 1024 lattice
with random edge orientation (1,024 sources) and reports it under `extra.lattice`.

Prints one JSON line: nominal GTEPS (sources x edges / s) as `value`, the roofline of the
search kernel (algorithmic bytes from exact per-call work counters over the kernel's
HIP-event time, against the 8 TB/s peak and against the bandwidth a STREAM-style kernel
reaches on the same GPU), and the CPU oracle timed on the same sources.

Other workloads (--workload): rmat16 (scale 16, edge factor 16, exact BC from all 65,536
sources), lattice (the lattice alone), batch (4,096 R-MAT graphs of scale 6..12, edge factor 8,
exact BC of each in one launch), serve (Poisson request stream), paper (the paper's three
strategies against the default path on BA digraphs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


KERNEL_OF_PATH = {0: "k_bc_global", 1: "k_bc_lds", 2: "k_msb", 7: "k_bc_deep"}
PATH_NAME = {0: "global", 1: "lds", 2: "batched", 7: "deep"}


def algorithmic_bytes(info, n):
    """Bytes the launch's design must move, from its exact work counters.

    One source per workgroup (paths 0, 1, 7): 96 B per reached vertex, 16 B per examined edge,
    24 B per shortest-path DAG edge, summed over sources.
    64-source batches (path 2): 144 B per level-list entry, 12 B per out-edge read for an
    entry in each sweep that reads it, 20 B per reached (vertex, source) pair (32-bit count
    read in each sweep and cleared, psi written), 16 B per DAG (edge, source) pair of a pushed
    level (32-bit count atomic, psi read), 16 B per vertex for every level-collect pass, plus
    the pulled levels' own reads (below).
    """
    if info["path"] == 2:
        # pulled forward levels: their entries' out-edges are not read forward; instead 20 B per
        # in-edge read (CSC row 4, level record of the in-neighbour 16), 8 B per vertex per pulled
        # level (its seen mask), and 12 B per DAG pair they find (count read 4, psi read 8)
        pushed = info["batch_edge_visits"] - info["batch_pull_skipped"]
        return (144 * info["batch_entries"] + 12 * info["batch_edge_visits"] + 12 * pushed
                + 20 * info["reached"] + 16 * (info["dag_edges"] - info["batch_pull_pairs"])
                + 12 * info["batch_pull_pairs"] + 16 * n * info["batch_scans"]
                + 20 * info["batch_pull_edges"] + 8 * n * info["batch_pull_levels"])
    return 96 * info["reached"] + 16 * info["examined"] + 24 * info["dag_edges"]


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1409_7764_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload, per_launch_scale):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they were taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except Exception:
        return None
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def _time_oracle(oracle, g, sources, m, threads, budget_s):
    """Sources per second of the oracle on a prefix of `sources`, grown until about half of
    `budget_s` is spent: (GTEPS, sources timed, seconds)."""
    k = min(len(sources), max(threads, 16))
    while True:
        t0 = time.perf_counter()
        oracle.bc(g, sources[:k], threads=threads)
        dt = time.perf_counter() - t0
        if dt >= budget_s / 2 or k >= len(sources):
            break
        # grow the sample towards the time budget
        k = int(min(len(sources), max(2 * k, k * budget_s / max(dt, 1e-3))))
    return k * m / dt / 1e9, k, dt


def cpu_baseline(n, u, v, sources, m, budget_s):
    """The CPU oracle, untuned, built -O3 -march=native on this host, on a bounded prefix of the
    benchmark's sources (all of them when they fit the budget): all host threads, and one
    thread on a smaller prefix (a quarter of the budget)."""
    import oracle
    try:
        lib = os.path.basename(oracle.use_native(True))
    except Exception as e:   # no compiler on this host: the generic -O3 build
        lib = f"{os.path.basename(oracle.use_native(False))} (native build failed: {e})"
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    threads = max(1, min(threads, oracle.max_threads() if oracle.max_threads() > 0 else threads))
    g = oracle.Graph(n, u, v)
    val, k, dt = _time_oracle(oracle, g, sources, m, threads, budget_s)
    val1, k1, dt1 = _time_oracle(oracle, g, sources, m, 1, budget_s / 4)
    return {"value": val, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{k} of the {len(sources)} sources (first {k} in benchmark order), "
                      f"{dt:.1f} s on {threads} threads of {cpu_info()}, {lib}",
            "single_thread": {"value": val1, "unit": "GTEPS", "cores": 1,
                              "sample": f"first {k1} sources, {dt1:.1f} s on 1 thread"}}


def stream_achievable(bcmi, sizes_gib=(1, 2, 4), reps=5):
    """Median copy and triad GB/s of the in-tree STREAM-style kernels at several array sizes
    (all far above the 256 MB MALL); `achievable` is the best of those medians."""
    runs = []
    for gib in sizes_gib:
        c, t = bcmi.bc_stream_probe(int(gib) << 30, reps)
        runs.append({"array_gib": gib, "copy_gbs": c, "triad_gbs": t})
    best = max(max(r["copy_gbs"], r["triad_gbs"]) for r in runs)
    return best, runs


WORKLOADS = {
    "rmat16": dict(cfg={"workload": "rmat16-exact", "graph": "R-MAT scale 16, edge factor 16, a=0.57 b=0.19 "
                        "c=0.19 d=0.05, seed 16, self-loops and duplicates removed", "sources": "all"}),
    "rmat20": dict(cfg={"workload": "rmat20-sampled1024", "graph": "R-MAT scale 20, edge factor 16, a=0.57 "
                        "b=0.19 c=0.19 d=0.05, seed 20, self-loops and duplicates removed",
                        "sources": "1024 uniform without replacement, seed 2020"}),
    "lattice": dict(cfg={"workload": "lattice1024-sampled1024", "graph": "1024x1024 lattice, random edge "
                         "orientation, seed 1", "sources": "1024 uniform without replacement, seed 1024"}),
}


def workload_input(gg, name):
    """(n, src, dst, sources, exact) of a single-graph workload."""
    if name == "rmat16":
        n, u, v = gg.rmat(16, 16, 16)
        return n, u, v, np.arange(n, dtype=np.uint32), True
    if name == "rmat20":
        n, u, v = gg.rmat(20, 16, 20)
        return n, u, v, gg.uniform_sources(n, 1024, 2020), False
    n, u, v = gg.grid_random_orientation(1024, 1024, 1)
    return n, u, v, gg.uniform_sources(n, 1024, 1024), False


def time_single(args, torch, bcmi, gg, name, achievable):
    """W untimed steps, then exactly K timed steps of one single-graph workload."""
    n, u, v, sources, exact = workload_input(gg, name)
    cfg = dict(WORKLOADS[name]["cfg"])
    t0 = time.perf_counter()
    g = bcmi.bc_build_csr(n, u, v)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    cfg.update({"n": n, "m": g.m})
    tune = None
    if args.tune:
        tune = bcmi.bc_tune(g)
    tun = bcmi.tuning(**{k: v for k, v in (tune or {}).items()}) if tune else None
    if args.strategy != "auto" or args.knob:
        base = dict(tune or {})
        if args.strategy != "auto":
            base.update({"batched": dict(batched=1), "per-source": dict(batched=-1)}[args.strategy])
        for kv in args.knob:
            key, val = kv.split("=")
            base[key] = int(val)
        tun = bcmi.tuning(**base)
        tune = base
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    d_src = torch.from_numpy(sources.view(np.int32)).cuda()

    def step():
        if exact:
            return bcmi.bc_exact(g, out=out, tuning=tun, info=True)[1]
        return bcmi.bc_sampled(g, d_src, out=out, tuning=tun, info=True)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    k = len(sources)
    kernel_ms = float(np.mean([i["kernel_ms"] for i in infos]))
    inf = infos[-1]
    nbytes = algorithmic_bytes(inf, n)
    achieved = nbytes / (kernel_ms / 1e3) / 1e9
    # the per-source accounting 16|E_s| + 32|D_s| + 92|R_s| summed over sources, whatever the
    # path: what one source at a time would move (a 64-source batch shares its edge reads)
    per_source = (16 * inf["examined"] + 32 * inf["dag_edges"] + 92 * inf["reached"]) / (kernel_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(cfg["workload"], 1),
            "achievable": achievable, "frac_of_achievable": achieved / achievable if achievable else None,
            "kernel": KERNEL_OF_PATH[inf["path"]],
            "kernel_ms": kernel_ms, "algorithmic_bytes_per_launch": nbytes,
            "per_source_convention_gbs": per_source}
    res = {
        "value": k * g.m / (ms_per_step / 1e3) / 1e9, "ms_per_step": ms_per_step,
        "dtype": "u32+f64" if inf["path"] == 2 else "u64+f64", "config": cfg, "roofline": roof,
        "extra": {
            "traversed_gteps": inf["examined"] / (ms_per_step / 1e3) / 1e9,
            "build_csr_ms": build_ms,
            "sources": k, "reached": inf["reached"], "examined": inf["examined"],
            "dag_edges": inf["dag_edges"], "levels_max": inf["levels_max"],
            "sigma_fp64_fallback_sources": inf["n_sigma_fp64_fallback"],
            "path": PATH_NAME[inf["path"]], "tuning": tune,
            "batch_entries": inf["batch_entries"], "batch_edge_visits": inf["batch_edge_visits"],
            "batch_scans": inf["batch_scans"], "batch_handoffs": inf["batch_handoffs"],
            "batch_cycles_fwd_bwd_reset": inf["batch_cycles"],
            "batch_pull_levels": inf["batch_pull_levels"], "batch_pull_edges": inf["batch_pull_edges"],
            "batch_pull_skipped": inf["batch_pull_skipped"], "batch_pull_pairs": inf["batch_pull_pairs"],
            "kernel_ms_all": [i["kernel_ms"] for i in infos],
        },
    }
    if args.plain_baseline:
        per = one_source_per_launch_ms(bcmi, torch, g, sources, 256)
        res["extra"]["one_launch_per_source_ms_estimated"] = per * k
        res["extra"]["speedup_vs_launch_per_source"] = per * k / ms_per_step
    g.free()
    return res, (n, u, v, sources, g.m)


def bench_single(args, torch, bcmi, gg):
    achievable, probe = (None, None)
    if not args.no_stream_probe:
        achievable, probe = stream_achievable(bcmi)
    res, (n, u, v, sources, m) = time_single(args, torch, bcmi, gg, args.workload, achievable)
    line = {
        "metric": "GTEPS (sources x edges / s), nominal, exact/sampled BC",
        "value": res["value"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": res["dtype"], "data": "synthetic", "config": res["config"], "roofline": res["roofline"],
        "extra": res["extra"],
    }
    line["extra"]["stream_probe"] = probe
    if args.workload == "rmat20" and not args.no_lattice:
        lat, _ = time_single(args, torch, bcmi, gg, "lattice", achievable)
        line["extra"]["lattice"] = {"value_gteps": lat["value"], "ms_per_step": lat["ms_per_step"],
                                    "config": lat["config"], "roofline": lat["roofline"],
                                    "sources": lat["extra"]["sources"], "levels_max": lat["extra"]["levels_max"],
                                    "sigma_fp64_fallback_sources": lat["extra"]["sigma_fp64_fallback_sources"],
                                    "path": lat["extra"]["path"], "kernel_ms_all": lat["extra"]["kernel_ms_all"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, u, v, sources, m, args.cpu_seconds)
    return line


def one_source_per_launch_ms(bcmi, torch, g, sources, reps):
    """Mean time of the plain path: one launch per source (bc_sampled with k = 1)."""
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    one = torch.zeros(1, dtype=torch.int32, device="cuda")
    tun = bcmi.tuning(batched=-1)
    bcmi.bc_sampled(g, one, out=out, tuning=tun)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sources[:reps]:
        one.fill_(int(s))
        bcmi.bc_sampled(g, one, out=out, tuning=tun)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / min(reps, len(sources))


def bench_paper(args, torch, bcmi, gg):
    """The paper's comparison (section III) on its own workload, BA digraphs: exact BC time of
    its three strategies (1 vertex-parallel, 2 edge-parallel, 3 host-synchronised levels) and of
    the default path, over graph size at density 10, over density at 5,000 vertices, and over
    workgroup size on 5,000 vertices / 49,950 edges."""

    def exact_ms(g, strategy, wg=None):
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        run = (lambda: bcmi.bc_exact(g, out=out)) if strategy == 0 else \
            (lambda: bcmi.bc_paper_strategy(g, strategy, wg or 256, out=out))
        run()
        torch.cuda.synchronize()
        reps = max(1, args.steps)
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    def row(n, beta, seed):
        g = bcmi.bc_build_csr(*gg.barabasi_albert(n, beta, seed))
        ms = {name: exact_ms(g, s) for name, s in [("bcmi", 0), ("vertex", 1), ("edge", 2), ("host_sync", 3)]}
        r = {"n": n, "m": g.m, "d": round(g.m / n, 2), "ms": {k: round(v, 3) for k, v in ms.items()},
             "speedup_over_host_sync": {k: round(ms["host_sync"] / v, 2) for k, v in ms.items()}}
        g.free()
        print(f"paper: n={n} m={r['m']} {r['ms']}", file=sys.stderr, flush=True)
        return r

    size = [row(n, 5, 100 + n) for n in (1000, 2000, 5000, 10000)]
    density = [row(5000, b, 200 + b) for b in (1, 2, 5, 10, 20, 30)]
    g = bcmi.bc_build_csr(*gg.barabasi_albert(5000, 5, 0))
    blocks = {name: {wg: round(exact_ms(g, strategy, wg), 3) for wg in (64, 128, 256, 512, 1024)}
              for name, strategy in [("vertex", 1), ("edge", 2), ("host_sync", 3)]}
    ref = {"n": g.n, "m": g.m, "bcmi_ms": exact_ms(g, 0)}
    g.free()
    value = ref["n"] * ref["m"] / (ref["bcmi_ms"] / 1e3) / 1e9
    return {"metric": "GTEPS (sources x edges / s), exact BC on the paper's BA digraph workload", "value": value,
            "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": ref["bcmi_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64+f64",
            "data": "synthetic",
            "config": {"workload": "paper-ba-n5000-m49950", "graph": "Barabasi-Albert digraph, n=5,000, "
                       "beta=5 (m=49,950), seed 0", "sources": "all"},
            "extra": {"graph_size_d10": size, "edge_density_n5000": density,
                      "workgroup_size_ms": blocks,
                      "strategies": {"vertex": "one workgroup per source, vertex-parallel levels",
                                     "edge": "one workgroup per source, edge-parallel levels",
                                     "host_sync": "whole grid per source, one launch per level, host-read flag",
                                     "bcmi": "default path of bc_exact"}}}


def bench_batch(args, torch, bcmi, gg):
    rng = np.random.default_rng(4096)
    scales = rng.integers(6, 13, size=4096)
    specs = [(int(s), 8, 4096_000 + i) for i, s in enumerate(scales)]
    graphs = []
    t0 = time.perf_counter()
    for sc, ef, seed in specs:
        n, u, v = gg.rmat(sc, ef, seed)
        graphs.append(bcmi.bc_build_csr(n, u, v))
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in graphs]

    def timed():
        for _ in range(args.warmup):
            bcmi.bc_batch(graphs, outs, info=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            infos.append(bcmi.bc_batch(graphs, outs, info=True)[1])
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, infos

    ms, infos = timed()
    tuned = None
    if args.tune:
        # the autotuner on the largest graph of each size class (floor(log2 n), round(log2 m/n));
        # bc_batch then resolves every graph's knobs from its class's entry
        default_ms, default_out = ms, [o.clone() for o in outs]
        reps = {}
        for g in graphs:
            key = (int(np.floor(np.log2(g.n))), int(round(np.log2(max(1.0, g.m / g.n)))))
            if key not in reps or g.n * g.m > reps[key].n * reps[key].m:
                reps[key] = g
        knobs = {f"n2^{k[0]} d2^{k[1]}": bcmi.bc_tune(g) for k, g in sorted(reps.items())}
        ms, infos = timed()
        worst = 0.0
        for a, b in zip(outs, default_out):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            nz = b != 0
            assert np.all(a[~nz] == 0), "tuned batch changed a structural zero"
            if nz.any():
                worst = max(worst, float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))))
        assert worst <= 1e-9, f"tuned batch differs from the default one by {worst}"
        tuned = {"default_ms": default_ms, "tuned_ms": ms, "speedup": default_ms / ms,
                 "max_rel_diff_vs_default": worst, "knobs_by_class": knobs}
    nominal = sum(g.n * g.m for g in graphs)
    per_graph_ms = per_source_ms = float("nan")
    if not args.skip_compare:
        # the same work as one exact launch per graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g, o in zip(graphs, outs):
            bcmi.bc_exact(g, out=o)
        torch.cuda.synchronize()
        per_graph_ms = (time.perf_counter() - t0) * 1e3
        # one launch per source, timed on a sample and scaled to every source
        sample_ms = []
        for g in graphs[:16]:
            sample_ms.append(one_source_per_launch_ms(bcmi, torch, g, np.arange(g.n), 32))
        per_source_ms = float(np.mean(sample_ms)) * sum(g.n for g in graphs)
    res = {"metric": "GTEPS (sources x edges / s), nominal, batched exact BC", "value": nominal / (ms / 1e3) / 1e9,
           "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64+f64", "data": "synthetic",
           "config": {"workload": "batch4096-rmat6to12-ef8", "graphs": 4096,
                      "sum_n": int(sum(g.n for g in graphs)), "sum_m": int(sum(g.m for g in graphs))},
           "extra": {"build_csr_ms_total": build_ms, "kernel_ms": infos[-1][0]["kernel_ms"], "autotune": tuned,
                     "one_exact_launch_per_graph_ms": per_graph_ms,
                     "one_launch_per_source_ms_estimated": per_source_ms,
                     "speedup_vs_launch_per_graph": per_graph_ms / ms,
                     "speedup_vs_launch_per_source": per_source_ms / ms}}
    for g in graphs:
        g.free()
    return res


def _serve_trace(bcmi, srv, reqs, outs, arrive, label):
    """Submits each request at its arrival time (seconds after the start), then polls every ticket
    to completion: (makespan seconds, infos)."""
    tickets = []
    t0 = time.perf_counter()
    for (g, S, _), out, at in zip(reqs, outs, arrive):
        while time.perf_counter() - t0 < at:
            pass
        tickets.append(bcmi.bc_serve_submit(srv, g, S, out))
    N = len(reqs)
    infos = [None] * N
    pending = set(range(N))
    last_print = time.perf_counter()
    while pending:
        for i in list(pending):
            inf = bcmi.bc_serve_poll(srv, tickets[i])
            if inf is not None:
                infos[i] = inf
                pending.discard(i)
        if time.perf_counter() - last_print > 20:
            print(f"serve {label}: {N - len(pending)}/{N} done", file=sys.stderr, flush=True)
            last_print = time.perf_counter()
        time.sleep(0.0005)
    return time.perf_counter() - t0, infos


def _latency_summary(infos, makespan, reqs):
    lat = np.array([i["t_done_ms"] - i["t_submit_ms"] for i in infos])
    work = sum(k * g.m for g, _, k in reqs)
    return {"requests": len(infos), "throughput_req_s": len(infos) / makespan, "makespan_s": makespan,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "nominal_gteps": work / makespan / 1e9}


def bench_serve(args, torch, bcmi, gg):
    """Poisson stream of BC requests over a pool of 64 resident R-MAT graphs (scale uniform on
    8..serve_max_scale, i.e. log-uniform n; edge factor uniform on 4..16), 70 % exact and 30 %
    on 256 sampled sources.  Two traces: (i) the stated arrival rate, which offers more work than
    one GPU serves (latency is then queueing), and (ii) the same kind of requests at 70 % of the
    capacity measured on (i).  Baselines on the same GPU, at the same accuracy (the same
    kernels): every request of (i) as one library call after another without the server, and
    one launch per source (timed on a sample of sources per graph, scaled to each request)."""
    rng = np.random.default_rng(5)
    pool = []
    for i in range(64):
        sc = int(rng.integers(8, args.serve_max_scale + 1))
        ef = int(rng.integers(4, 17))
        n, u, v = gg.rmat(sc, ef, 5000 + i)
        pool.append(bcmi.bc_build_csr(n, u, v))
    torch.cuda.synchronize()
    N = args.serve_requests
    arrive = np.cumsum(rng.exponential(1.0 / args.serve_rate, size=N))
    reqs = []
    for i in range(N):
        g = pool[int(rng.integers(0, len(pool)))]
        if rng.random() < 0.7:
            reqs.append((g, None, g.n))
        else:
            k = min(256, g.n)
            reqs.append((g, gg.uniform_sources(g.n, k, 77 + i), k))
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g, _, _ in reqs]
    srv = bcmi.bc_serve_create(200 << 30)
    for g, S, _ in reqs[:2]:   # warm-up: one request of each kind
        t = bcmi.bc_serve_submit(srv, g, S, torch.empty(g.n, dtype=torch.float64, device="cuda"))
        while bcmi.bc_serve_poll(srv, t) is None:
            time.sleep(0.001)
    makespan, infos = _serve_trace(bcmi, srv, reqs, outs, arrive, "stated rate")
    first = _latency_summary(infos, makespan, reqs)
    first["offered_rate_req_s"] = args.serve_rate
    capacity = first["throughput_req_s"]
    # (ii) rate-scaled: the first requests again, arriving at 70 % of the measured capacity
    N2 = min(N, args.serve_scaled_requests)
    rate2 = 0.7 * capacity
    arrive2 = np.cumsum(np.random.default_rng(55).exponential(1.0 / rate2, size=N2))
    makespan2, infos2 = _serve_trace(bcmi, srv, reqs[:N2], outs[:N2], arrive2, "scaled rate")
    second = _latency_summary(infos2, makespan2, reqs[:N2])
    second["offered_rate_req_s"] = rate2
    bcmi.bc_serve_destroy(srv)
    res = {"metric": "served BC requests: throughput and p50/p99 latency", "value": first["throughput_req_s"],
           "unit": "requests/s", "n_gpus": 1, "steps": 1, "warmup": 2, "ms_per_step": makespan * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64+f64",
           "data": "synthetic",
           "config": {"workload": f"served-poisson{args.serve_rate:g}-rmat8to{args.serve_max_scale}-ef4to16",
                      "requests": N, "exact_fraction": 0.7, "sampled_k": 256, "graph_pool": 64},
           "extra": {"stated_rate": first, "scaled_rate": second}}
    if not args.skip_compare:
        # one library call per request, one after another (no server, no continuous batching);
        # each call's service time also gives the latency a first-come-first-served queue of
        # such calls would have on the rate-scaled arrivals
        torch.cuda.synchronize()
        service = []
        t0 = time.perf_counter()
        for (g, S, _), out in zip(reqs, outs):
            t1 = time.perf_counter()
            if S is None:
                bcmi.bc_exact(g, out=out)
            else:
                bcmi.bc_sampled(g, S, out=out)
            torch.cuda.synchronize()
            service.append(time.perf_counter() - t1)
        seq = time.perf_counter() - t0
        free_at, lat2 = 0.0, []
        for at, sv in zip(arrive2, service[:N2]):
            start = max(at, free_at)
            free_at = start + sv
            lat2.append((free_at - at) * 1e3)
        res["extra"]["fifo_calls_scaled_rate"] = {"p50_ms": float(np.percentile(lat2, 50)),
                                                  "p99_ms": float(np.percentile(lat2, 99)),
                                                  "mean_ms": float(np.mean(lat2))}
        # one launch per source: per graph, a sample of single-source launches
        per_src = {}
        for g, _, _ in reqs:
            if id(g) not in per_src:
                per_src[id(g)] = one_source_per_launch_ms(bcmi, torch, g, np.arange(g.n), 16)
        plain_s = sum(k * per_src[id(g)] for g, _, k in reqs) / 1e3
        res["extra"]["one_call_per_request"] = {"makespan_s": seq, "throughput_req_s": N / seq,
                                                "speedup_of_server": seq / makespan}
        res["extra"]["one_launch_per_source_estimated"] = {"makespan_s": plain_s, "throughput_req_s": N / plain_s,
                                                           "speedup_of_server": plain_s / makespan,
                                                           "sample": "16 single-source launches per graph"}
    for g in pool:
        g.free()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20",
                    choices=["rmat16", "rmat20", "lattice", "batch", "serve", "paper"])
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="mean arrivals per second")
    ap.add_argument("--serve-max-scale", type=int, default=18)
    ap.add_argument("--serve-scaled-requests", type=int, default=128,
                    help="requests of the rate-scaled trace (70 %% of the measured capacity)")
    ap.add_argument("--tune", action="store_true", help="autotune launch knobs first (untimed)")
    ap.add_argument("--strategy", default="auto", choices=["auto", "batched", "per-source"])
    ap.add_argument("--knob", action="append", default=[], help="launch knob override, e.g. batch_wg_size=512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lattice", action="store_true", help="rmat20 workload: skip the lattice leg")
    ap.add_argument("--no-stream-probe", action="store_true",
                    help="skip the STREAM-style bandwidth probe (roofline.achievable is then null)")
    ap.add_argument("--skip-compare", action="store_true",
                    help="batch and serve workloads: skip the comparisons with plain launches")
    ap.add_argument("--plain-baseline", action="store_true",
                    help="also time the one-launch-per-source path on a sample of sources")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="time budget of the CPU oracle sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 2 GiB device-to-device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU (--gpus 1): the method would shard over sources with one "
              "final sum of the per-GPU BC arrays, and only the single-GPU share is run and reported.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1409_7764_amd import bcmi, graphgen as gg
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    bcmi.lib()
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batch":
        res = bench_batch(args, torch, bcmi, gg)
    elif args.workload == "serve":
        res = bench_serve(args, torch, bcmi, gg)
    elif args.workload == "paper":
        res = bench_paper(args, torch, bcmi, gg)
    else:
        res = bench_single(args, torch, bcmi, gg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
