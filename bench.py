"""Benchmark: exact betweenness centrality throughput on one MI355X.

One step = one full pass of the hot path over the workload: every source of
the graph through bc_compute (forward counting sweep, backward dependency
sweep, score fold), inputs resident in HBM.  The printed JSON line carries
GTEPS (sources x undirected edges / s), the roofline of the dominant kernel,
the one-source-per-launch form on a source sample, and the CPU oracle timed
on the host on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config rmat20p]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BC GTEPS (sources×edges/s) batched vs plain, 1 GPU; p50/p99 query latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str, sources_arg: int):
    import graphgen as gg
    if name == "rmat10":
        g, wl, prune = gg.workload_rmat10(), "rmat10_ef16_all_sources", False
    elif name == "rmat16":
        g, wl, prune = gg.workload_rmat16(), "rmat16_ef16_all_sources", False
    elif name == "rmat20p":
        g, wl, prune = gg.workload_rmat20_pendants(), "rmat20_ef16_plus30pct_pendants_all_sources_pruned", True
    elif name == "grid2048":
        g, wl, prune = gg.workload_roadlike_grid(), "grid2048_roadlike_all_sources", False
    elif name == "strip":
        # a 16384 x 4 lattice strip: a long diameter (16,386 levels) with counts that fit 64 bits
        g, wl, prune = gg.full_grid(16384, 4), "strip16384x4_lattice_all_sources", False
    else:
        raise SystemExit(f"unknown workload {name} (rmat10, rmat16, rmat20p, grid2048, strip)")
    if sources_arg < 0:
        sources_arg = DEFAULT_SOURCES.get(name, 0)
    src = None
    if sources_arg > 0:
        src = gg.sample(g.non_isolated(), min(sources_arg, len(g.non_isolated())), 44)
        wl = wl.replace("all_sources", f"{len(src)}_sampled_sources")
    return g, wl, prune, src


def alg_bytes(n: int, nnz: int, launches: int, st: dict) -> float:
    """Algorithmic bytes of a run: per launch the CSR streamed once per
    sweep (2 sweeps) and the score array read and written once; per source
    a 1-bit level test per directed edge of the reached set per sweep, one
    8-byte count forward and one 8-byte dependency term backward per DAG
    edge, and 40 bytes per reached vertex (level 4+4, count 8+8, dependency
    8+8, each written once and read once)."""
    per_launch = 2 * (4 * (n + 1) + 4 * nnz) + 16 * n
    return float(launches * per_launch + 2 * st["reached_nnz"] / 8 + 16 * st["dag_edges"] + 40 * st["reached"])


def alg_bytes_wg(n: int, launches: int, st: dict) -> float:
    """Algorithmic bytes of a per-workgroup run, where every source walks
    its own scalar state: per sweep and reached vertex its 8-byte row
    bounds, per sweep and reached directed edge the 4-byte column index and
    the neighbour's 4-byte level; per DAG edge an 8-byte count forward and
    an 8-byte dependency term backward; per reached vertex 48 bytes (level
    written, read and reset 4+4+4, count 8+8+8, dependency 8+8, queue slot
    4+4 minus the reads counted above as 12); the score array once per
    launch."""
    return float(launches * 16 * n + 2 * (8 * st["reached"] + 8 * st["reached_nnz"]) + 16 * st["dag_edges"]
                 + 48 * st["reached"])


def stream_copy_gbs(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM bandwidth: a device-to-device copy of nbytes timed with
    HIP events (median of reps), counted as bytes read plus bytes written."""
    import torch
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (float(np.median(ts)) / 1e3) / 1e9


def timed_compute(G, sources, stream, **opts):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    st = G.compute(sources, stream=stream, **opts)
    e1.record(stream)
    torch.cuda.synchronize()
    return st, e0.elapsed_time(e1)


KERNEL_SOURCES = {
    "batch_kernel": ["paper_1602_00963_amd/csrc/bc_batch.hip", "paper_1602_00963_amd/csrc/bc_common.h",
                     "paper_1602_00963_amd/csrc/bc_kernels.h"],
    "wg_kernel": ["paper_1602_00963_amd/csrc/bc_wg.hip", "paper_1602_00963_amd/csrc/bc_wg.h",
                  "paper_1602_00963_amd/csrc/bc_common.h"],
}
MODE_KERNEL = {"batched": "batch_kernel", "plain": "plain_kernel", "plain_scan": "scan_kernel",
               "per_workgroup": "wg_kernel"}


def kernel_sha(kernel: str = "batch_kernel") -> str:
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name: str, kernel: str = "batch_kernel"):
    """HBM bytes per launch of a kernel from committed rocprofv3 counter
    runs (FETCH_SIZE, WRITE_SIZE, each scaled by the same counter on a plain
    copy of known size); None unless the kernel source is unchanged since
    the counters were taken."""
    if kernel not in KERNEL_SOURCES:
        return None
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload_name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_sha") != kernel_sha(kernel):
        return None
    return t


def copy_calibration(nbytes: int, quiet: bool = False) -> None:
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    if not quiet:
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def _counter_rows(d: str):
    import csv
    import glob
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(max(f, key=os.path.getmtime)) as fh:  # the latest run in the directory
        return list(csv.DictReader(fh))


def summarize_counters(fetch_dir: str, write_dir: str, wl: str, copy_bytes: int, command: str,
                       kernel: str = "batch_kernel", last: int = 0) -> None:
    """Per-launch HBM traffic of a kernel from two rocprofv3 counter runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for the copy kernel of known size run in the same process.
    With last > 0 only the kernel's last `last` dispatches count (the timed
    step's, after warm-up launches of other sizes).  Writes
    profiles/traffic_<kernel>_<wl>.json and .md."""
    res = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        kern, copy = [], []
        for r in _counter_rows(d):
            if r["Counter_Name"] != name:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            if kernel in r["Kernel_Name"]:
                kern.append((int(r.get("Dispatch_Id") or 0), v))
            elif "copy" in r["Kernel_Name"].lower() and v > 0.5 * copy_bytes:
                copy.append(v)
        if not kern or not copy:
            raise SystemExit(f"{name}: missing {kernel} or copy dispatches")
        kern = [v for _, v in sorted(kern)]  # dispatch order
        if last > 0:
            kern = kern[-last:]
        scale = copy_bytes / float(np.median(copy))
        res[name] = {"kernel_bytes_per_launch_raw": float(np.mean(kern)), "dispatches": len(kern),
                     "copy_bytes_raw": float(np.median(copy)), "scale": scale,
                     "kernel_bytes_per_launch": float(np.mean(kern)) * scale}
    t = {"kernel": kernel, "workload": wl, "kernel_sha": kernel_sha(kernel),
         "bytes_per_launch": res["FETCH_SIZE"]["kernel_bytes_per_launch"] + res["WRITE_SIZE"]["kernel_bytes_per_launch"],
         "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"], "copy_bytes": copy_bytes, "command": command,
         "source": f"profiles/traffic_{kernel}_{wl}.md"}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wl}.json"), "w") as f:
        json.dump(t, f, indent=1)
    with open(os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wl}.md"), "w") as f:
        f.write(f"# HBM traffic of {kernel}, workload {wl}\n\n")
        f.write(f"Counter runs (one per counter, each followed in the same process by a copy of {copy_bytes} bytes):\n\n")
        f.write(f"    {command}\n\n")
        f.write(f"| counter | {kernel} KiB/dispatch (raw) | dispatches | copy raw bytes | scale | bytes/launch |\n")
        f.write("|---|---|---|---|---|---|\n")
        for name in ("FETCH_SIZE", "WRITE_SIZE"):
            r = res[name]
            f.write(f"| {name} | {r['kernel_bytes_per_launch_raw'] / 1024:.0f} | {r['dispatches']} | "
                    f"{r['copy_bytes_raw']:.4g} | {r['scale']:.4f} | {r['kernel_bytes_per_launch']:.4g} |\n")
        f.write(f"\nTraffic per launch: {t['bytes_per_launch']:.4g} bytes (kernel source sha {t['kernel_sha']}).\n")
    print(json.dumps(t), flush=True)


def summarize_trace(trace_dir: str, name: str, command: str) -> None:
    """Kernel-time summary (rocprofv3 --kernel-trace --stats) as markdown."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no kernel_stats.csv under {trace_dir}")
    with open(f[0]) as fh:
        rows = list(csv.DictReader(fh))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    out = os.path.join(ROOT, "profiles", f"{name}.md")
    with open(out, "w") as fo:
        fo.write(f"# rocprofv3 kernel statistics: {name}\n\n    {command}\n\n")
        fo.write("| kernel | calls | total ms | average us | min us | max us | % |\n|---|---|---|---|---|---|---|\n")
        for r in rows:
            nm = r.get("Name", "")
            short = nm if len(nm) < 70 else nm[:67] + "..."
            fo.write(f"| `{short}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")
        # kernels dispatched only a few times: every dispatch, in order (launches
        # of different sizes - a probe, a rerun - then stay apart from the step's)
        tf = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
        if tf:
            with open(max(tf, key=os.path.getmtime)) as fh:
                disp = [d for d in csv.DictReader(fh) if "bcx::" in d["Kernel_Name"]]
            by = {}
            for d in disp:
                by.setdefault(d["Kernel_Name"], []).append((int(d["Start_Timestamp"]),
                                                            (int(d["End_Timestamp"]) - int(d["Start_Timestamp"])) / 1e6,
                                                            d["Grid_Size_X"]))
            few = {k: v for k, v in by.items() if len(v) <= 12}
            if few:
                fo.write("\nDispatches in order (ms, grid threads):\n\n")
                for k, v in few.items():
                    short = k if len(k) < 70 else k[:67] + "..."
                    fo.write(f"- `{short}`: " + ", ".join(f"{ms:.2f} ({grid})" for _, ms, grid in sorted(v)) + "\n")
    print(open(out).read())


def serving_run(bcm, ctx, n_graphs: int, max_scale: int, n_queries: int, rhos, warmup_queries: int = 0,
                max_inflight: int = 4, seed: int = 5, budget_gb: float = 0.0):
    """Poisson stream of BC queries over resident graphs through the
    continuous-batching server: p50/p99 latency and GTEPS per offered load.
    Capacity (queries / s) is measured first in a closed loop on
    `warmup_queries` queries (all submitted at once); each rho then offers
    rho times that rate for `n_queries` queries (arrivals seeded)."""
    import threading
    import graphgen as gg
    specs = gg.serving_graph_specs(n_graphs, 5000, 12, max_scale)
    graphs = [gg.rmat(s, ef, sd) for s, ef, sd in specs]
    Gs = [bcm.Graph(ctx, g, validate=False) for g in graphs]
    log(f"serving: {len(graphs)} graphs resident, scales {sorted(s for s, _, _ in specs)}")
    rng = np.random.default_rng(seed)

    def draw(count, base):
        qs = []
        for i in range(count):
            gi = int(rng.integers(len(graphs)))
            cand = graphs[gi].non_isolated()
            k = int(min(len(cand), rng.integers(256, 8193)))
            qs.append((gi, gg.sample(cand, k, base + i)))
        return qs

    srv = bcm.Server(ctx, max_inflight=max_inflight, batch=256,
                     hbm_budget_bytes=int(budget_gb * (1 << 30)) if budget_gb > 0 else 0)
    warm = draw(max(8, warmup_queries or n_queries // 10), 100000)
    t0 = time.perf_counter()
    tk = [srv.submit(Gs[gi], S) for gi, S in warm]
    for t in tk:
        srv.wait(t)
    cap = len(warm) / (time.perf_counter() - t0)
    log(f"serving: closed loop {len(warm)} queries, capacity {cap:.2f} queries/s")
    out = {"graphs": len(graphs), "scales": [s for s, _, _ in specs], "efs": [e for _, e, _ in specs],
           "warmup_queries": len(warm), "closed_loop_qps": round(cap, 2), "loads": []}
    for rho in rhos:
        qs = draw(n_queries, 200000 + int(rho * 1000) * 10000)
        rate = rho * cap
        gaps = rng.exponential(1.0 / rate, size=len(qs))
        stats = [None] * len(qs)
        tickets = [None] * len(qs)

        def submitter():
            nxt = time.perf_counter()
            for i, (gi, S) in enumerate(qs):
                nxt += gaps[i]
                d = nxt - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(Gs[gi], S)

        s0 = srv.stats()
        th = threading.Thread(target=submitter)
        t0 = time.perf_counter()
        th.start()
        for i in range(len(qs)):
            while tickets[i] is None:
                time.sleep(0.0005)
            stats[i] = srv.wait(tickets[i])
            if (i + 1) % 250 == 0:
                log(f"serving rho={rho}: {i + 1}/{len(qs)} queries done")
        th.join()
        span = time.perf_counter() - t0
        s1 = srv.stats()
        lat = np.array([st["latency_ms"] for st in stats])
        te = sum(st["te"] for st in stats)
        busy = s1["busy_ms"] - s0["busy_ms"]
        mean_inf = ((s1["mean_inflight"] * s1["busy_ms"] - s0["mean_inflight"] * s0["busy_ms"]) / busy
                    if busy > 0 else 0.0)
        row = {"rho": rho, "queries": len(qs), "offered_qps": round(rate, 2),
               "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
               "gteps": round(te / span / 1e9, 3), "span_s": round(span, 2),
               "batches": s1["batches"] - s0["batches"], "mean_inflight": round(mean_inf, 3),
               "max_inflight_seen": s1["max_inflight_seen"]}
        log(f"serving: {row}")
        out["loads"].append(row)
    sst = srv.stats()
    srv.close()
    for G in Gs:
        G.close()
    out["server"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in sst.items()}
    head = next((r for r in out["loads"] if abs(r["rho"] - 0.8) < 1e-9), out["loads"][0])
    out.update({"rho": head["rho"], "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "gteps": head["gteps"]})
    return out


def overlap_stats(rows) -> dict:
    """Concurrency of kernel dispatches (kernel-trace rows with start/end
    timestamps and grid/workgroup sizes): time covered by k dispatches for
    each k, and the most dispatches and workgroups running at once.  A
    dispatch that starts when another ends does not overlap it."""
    ev = []
    for r in rows:
        wg = int(r["Grid_Size_X"]) // max(int(r["Workgroup_Size_X"]), 1)
        ev.append((int(r["Start_Timestamp"]), 1, wg))
        ev.append((int(r["End_Timestamp"]), -1, wg))
    ev.sort()  # at equal times, ends before starts
    cur = best = cur_wg = best_wg = 0
    cover = {}
    last = ev[0][0] if ev else 0
    for t, d, wg in ev:
        if cur > 0:
            cover[cur] = cover.get(cur, 0) + (t - last)
        cur += d
        cur_wg += d * wg
        best = max(best, cur)
        best_wg = max(best_wg, cur_wg)
        last = t
    return {"cover_ns": cover, "any_ns": sum(cover.values()),
            "multi_ns": sum(v for k, v in cover.items() if k >= 2), "most": best, "most_workgroups": best_wg,
            "streams": sorted({r["Stream_Id"] for r in rows}),
            "grids": sorted({int(r["Grid_Size_X"]) // max(int(r["Workgroup_Size_X"]), 1) for r in rows})}


def summarize_overlap(trace_dir: str, name: str, command: str) -> None:
    """Overlap of batch_kernel dispatches in a kernel trace.  Writes
    profiles/<name>.md."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no kernel_trace.csv under {trace_dir}")
    with open(f[0]) as fh:
        rows = [r for r in csv.DictReader(fh) if "batch_kernel" in r["Kernel_Name"]]
    o = overlap_stats(rows)
    any_ns, multi_ns = o["any_ns"], o["multi_ns"]
    out = os.path.join(ROOT, "profiles", f"{name}.md")
    with open(out, "w") as fo:
        fo.write(f"# Concurrent batch_kernel dispatches: {name}\n\n    {command}\n\n")
        fo.write(f"- dispatches: {len(rows)} on {len(o['streams'])} streams; workgroups per dispatch: {o['grids']}\n")
        fo.write(f"- time with >= 1 dispatch running: {any_ns / 1e6:.1f} ms\n")
        fo.write(f"- time with >= 2 running: {multi_ns / 1e6:.1f} ms ({100.0 * multi_ns / max(any_ns, 1):.1f}%)\n")
        fo.write(f"- most running at once: {o['most']}; most workgroups running at once: {o['most_workgroups']}\n")
        fo.write("- time by number running: "
                 + ", ".join(f"{k}: {v / 1e6:.1f} ms" for k, v in sorted(o["cover_ns"].items())) + "\n")
    print(open(out).read())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, m: int, budget_s: float, seed: int = 91):
    """The oracle (sequential Brandes per source, unpruned graph) timed on
    the host: on `cores` threads with a static split of a bounded sample of
    sources, and on one thread on a smaller sample."""
    import graphgen as gg
    import oracle
    nproc = os.cpu_count() or 1
    cores = min(nproc, 16)   # the GPU machine's CPU share for one GPU
    cand = g.non_isolated()
    probe = gg.sample(cand, min(len(cand), 2 * cores), seed)
    t0 = time.perf_counter()
    oracle.bc(g, probe, nthreads=cores)
    dt = max(time.perf_counter() - t0, 1e-3)
    k = int(min(len(cand), max(len(probe), len(probe) * budget_s / dt)))
    S = gg.sample(cand, k, seed + 1)
    t0 = time.perf_counter()
    oracle.bc(g, S, nthreads=cores)
    dt = time.perf_counter() - t0
    # one thread, about a quarter of the budget
    k1 = int(min(len(cand), max(1, k / cores * (budget_s / 4) / max(dt, 1e-3))))
    S1 = gg.sample(cand, k1, seed + 2)
    t0 = time.perf_counter()
    oracle.bc(g, S1, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": k * m / dt / 1e9, "unit": "GTEPS", "cores": cores, "kind": "oracle",
            "sample": f"{k} uniformly sampled sources of the same graph (seed {seed + 1}), sequential Brandes "
                      f"per source on the unpruned graph, static split over {cores} threads; {dt:.1f} s",
            "value_1thread": k1 * m / dt1 / 1e9,
            "sample_1thread": f"{k1} sources (seed {seed + 2}), one thread; {dt1:.1f} s",
            "nproc": nproc, "cpu_model": cpu_model()}


# Settings measured fastest on MI355X.  Batch width (sweep of 128..1024
# sources per launch): the scale-16 all-sources run gains from 1024, the
# scale-20 graph (ten times the vertices per level) does best at 256.
# Bottom-up threshold: on the R-MAT graphs no level goes bottom-up at the
# default threshold (a lower one, 4, is 20% slower on the scale-20 graph),
# and switching the test off (-1) spares the kernel its bookkeeping (+1%).
BEST_BATCH = {"rmat16": 1024}
BEST_ALPHA = {"rmat16": -1.0, "rmat20p": -1.0}
# Sources per step when none are given: the scale-20 graph is measured on a
# uniform sample (all its 1.1 M non-pruned sources would take about a minute
# and a half per step), as the paper extrapolates from a sample of sources;
# the lattice on its 8,192 sampled sources.
DEFAULT_SOURCES = {"rmat20p": 16384, "grid2048": 8192}
PLAIN_SAMPLE = {"rmat20p": 512, "grid2048": 64}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="rmat20p",
                    help="workload: rmat10, rmat16, rmat20p (default: scale 20 with pendants, pruned), grid2048")
    ap.add_argument("--sources", type=int, default=-1,
                    help="sample this many sources (0 = all; -1 = the workload's default: 16,384 on rmat20p, "
                         "8,192 on grid2048, all on the others)")
    ap.add_argument("--batch", type=int, default=0,
                    help="sources per launch (0 = the width measured fastest for the workload: "
                         "1024 on the scale-16 graph, 256 on the others)")
    ap.add_argument("--mode", default=None,
                    help="batched, plain, plain_scan, per_workgroup or auto (default: per_workgroup on "
                         "grid2048, batched on the others)")
    ap.add_argument("--order", default=None,
                    help="internal vertex order: degree or rcm (default: rcm on grid2048, degree on the others)")
    ap.add_argument("--alpha", type=float, default=None,
                    help="bottom-up threshold (0 = library default, < 0 = never; "
                         "unset = the workload's measured best: -1 on the R-MAT graphs)")
    ap.add_argument("--beta", type=float, default=0.0, help="bottom-up switch-back threshold (0 = none)")
    ap.add_argument("--grid-per-cu", type=int, default=0)
    ap.add_argument("--deg2", action="store_true")
    ap.add_argument("--no-prune", action="store_true",
                    help="run the scale-20 pendant workload without the 1-degree reduction")
    ap.add_argument("--prune-trees", action="store_true", help="iterate the 1-degree reduction")
    ap.add_argument("--autotune", type=int, default=-1,
                    help="tune batch/alpha/grid on this many sampled sources first (0 = off; -1 = 4,096 "
                         "when no batch or alpha is given)")
    ap.add_argument("--plain-sample", type=int, default=0,
                    help="sources timed one per launch (0 = 512 on rmat20p, 64 on grid2048, else 2,048)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-graph", type=int, default=64,
                    help="also time the plain leg with this many per-source launches per HIP graph (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, help="only run a copy of this many bytes")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--serving-full", action="store_true",
                    help="the full serving mix: 32 graphs of scale 12-20, 200 warm-up and 2,000 measured "
                         "queries at each load 0.5, 0.8, 0.95")
    ap.add_argument("--serving-graphs", type=int, default=8)
    ap.add_argument("--serving-max-scale", type=int, default=15)
    ap.add_argument("--serving-queries", type=int, default=200)
    ap.add_argument("--serving-warmup", type=int, default=0)
    ap.add_argument("--serving-rho", type=float, nargs="+", default=[0.8])
    ap.add_argument("--serving-inflight", type=int, default=4)
    ap.add_argument("--serving-budget-gb", type=float, default=0.0)
    ap.add_argument("--summarize-overlap", metavar="TRACE_DIR", help="write profiles/<--profile-name>.md")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="after the run, copy this many bytes (scales the traffic counters)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_<kernel>_<workload>.json from two counter runs (the kernel of --mode)")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR", help="write profiles/<--profile-name>.md")
    ap.add_argument("--profile-name", default="")
    ap.add_argument("--counter-last", type=int, default=0,
                    help="with --summarize-counters: count only the kernel's last N dispatches")
    ap.add_argument("--profile-command", default="")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.summarize_counters:
        _, wl, _, _ = workload(args.config, args.sources)
        mode = args.mode or ("per_workgroup" if args.config == "grid2048" else "batched")
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], wl, args.calibrate_copy,
                           args.profile_command, MODE_KERNEL[mode], args.counter_last)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.profile_name, args.profile_command)
        return
    if args.summarize_overlap:
        summarize_overlap(args.summarize_overlap, args.profile_name, args.profile_command)
        return
    if args.serving_full:
        args.serving_graphs, args.serving_max_scale, args.serving_queries = 32, 20, 2000
        args.serving_warmup, args.serving_rho = 200, [0.5, 0.8, 0.95]
        args.serving_budget_gb = args.serving_budget_gb or 200.0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        raise SystemExit(2)

    import torch
    import paper_1602_00963_amd as bcm

    if args.serving_only:
        ctx = bcm.Context(0)
        sv = serving_run(bcm, ctx, args.serving_graphs, args.serving_max_scale, args.serving_queries,
                         args.serving_rho, args.serving_warmup, args.serving_inflight,
                         budget_gb=args.serving_budget_gb)
        print(json.dumps({"metric": "BC serving: p50/p99 query latency and GTEPS, 1 GPU", "serving": sv}),
              flush=True)
        return
    g, wl, prune, sources = workload(args.config, args.sources)
    if args.no_prune and prune:
        prune, wl = False, wl.replace("_pruned", "_unpruned")
    if args.prune_trees:
        prune, wl = "trees", wl.replace("_pruned", "") + "_trees"
    if args.deg2:
        wl += "_deg2"
    if args.autotune < 0:
        args.autotune = 4096 if (args.batch == 0 and args.alpha is None) else 0
    if args.batch == 0:
        args.batch = BEST_BATCH.get(args.config, 256)
    if args.alpha is None:
        args.alpha = BEST_ALPHA.get(args.config, 0.0)
    if args.mode is None:
        args.mode = "per_workgroup" if args.config == "grid2048" else "batched"
    if args.order is None:
        args.order = "rcm" if args.config == "grid2048" else "degree"
    if args.plain_sample <= 0:
        args.plain_sample = PLAIN_SAMPLE.get(args.config, 2048)
    n, nnz, m = g.n, g.nnz, g.m
    log(f"workload {wl}: n={n} m={m}")
    ctx = bcm.Context(0)
    G = bcm.Graph(ctx, g, validate=False, prune=prune, order=args.order)
    stream = torch.cuda.Stream()
    opts = dict(mode=args.mode, batch=args.batch, deg1=bool(prune), deg2=args.deg2, alpha=args.alpha,
                grid_per_cu=args.grid_per_cu, beta=args.beta)
    tuned = None
    if args.autotune > 0 and args.mode == "batched":
        import graphgen as gg
        cand = g.non_isolated() if sources is None else sources
        t0 = time.perf_counter()
        tuned = G.autotune(gg.sample(cand, min(args.autotune, len(cand)), 17), budget_ms=60000.0, deg1=bool(prune),
                           deg2=args.deg2)
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
        log(f"autotune: {tuned}")
        opts.update(batch=0, alpha=0.0, grid_per_cu=0, beta=0.0)
    for i in range(args.warmup):
        st, ms = timed_compute(G, sources, stream, **opts)
        log(f"warmup {i}: {ms:.1f} ms, launches {st['launches']}")
    times, stats = [], []
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for i in range(args.steps):
        st, ms = timed_compute(G, sources, stream, **opts)
        times.append(ms)
        stats.append(st)
        log(f"step {i}: {ms:.1f} ms  {st['te'] / ms / 1e6:.2f} GTEPS  launches {st['launches']} "
            f"levels {st['levels']} bu {st['bottom_up_levels']} overflowed {st['overflowed']}")
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    st = stats[-1]
    ms_step = wall_ms / args.steps
    gteps = st["te"] / (ms_step / 1e3) / 1e9
    # the batched kernel's own time: HIP events recorded on the launch stream
    # around every launch, summed by the library (median step)
    kern_ms = float(np.median([s["kernel_ms"] for s in stats]))
    per_launch_ms = kern_ms / max(st["launches"], 1)
    tn = nnz if not prune else G.stats()["residual_nnz"]
    mode_run = st["mode"]  # the mode the library ran (resolves "auto")
    bytes_run = (alg_bytes_wg(n, st["launches"], st) if mode_run == "per_workgroup"
                 else alg_bytes(n, tn, st["launches"], st))
    achieved = bytes_run / (kern_ms / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64+f64", "data": "synthetic",
        "config": {"workload": wl, "n": n, "m": m, "sources": int(st["sources"]), "traversed": int(st["traversed"]),
                   "mode": mode_run, "vertex_order": args.order,
                   "batch": (tuned["batch"] if tuned else args.batch) if mode_run == "batched" else None,
                   "bottom_up_alpha": tuned["alpha"] if tuned else args.alpha,
                   "bottom_up_beta": tuned["beta"] if tuned else args.beta, "pruned": prune,
                   "deg2": args.deg2, "autotuned": tuned},
        "gteps_2m": round(2 * gteps, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel_sha": kernel_sha(MODE_KERNEL[mode_run]) if MODE_KERNEL[mode_run] in KERNEL_SOURCES
                     else None,
                     "kernel": MODE_KERNEL[mode_run],
                     "avg_launch_ms": round(per_launch_ms, 4), "launches": int(st["launches"]),
                     "kernel_ms_per_step": round(kern_ms, 2), "event_ms_per_step": round(float(np.median(times)), 2),
                     "launch_gap_us": round((float(np.median(times)) - kern_ms) * 1e3 / max(st["launches"], 1), 1),
                     "alg_bytes_per_launch": round(bytes_run / max(st["launches"], 1)),
                     "bytes_per_te": round(bytes_run / st["raw_te"], 3) if st["raw_te"] else None},
    }
    copy_gbs = stream_copy_gbs()
    out["roofline"]["stream_copy_GBs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_stream_copy"] = round(achieved / copy_gbs, 4)
    log(f"streaming copy: {copy_gbs:.0f} GB/s")
    # heuristics coverage of the graph over all sources (host), as the paper's heuristics table counts it
    cov = {}
    for name, kw in (("H0", {}), ("H1", dict(prune=True, deg1=True)), ("H2", dict(deg2=True)),
                     ("H3", dict(prune=True, deg1=True, deg2=True))):
        cov[name] = bcm.coverage_host(g.n, g.row_ptr, g.col_idx, **kw)
    out["coverage"] = cov
    tr = measured_traffic(wl, MODE_KERNEL[mode_run])
    if tr:
        # HBM bytes from the counters (FETCH_SIZE scaled by a streaming copy's reading, whose
        # 128-byte requests make the factor an upper bound for the kernel's 32-64-byte sectors;
        # the raw reading is the lower bound), beside the algorithmic bytes
        out["roofline"]["traffic"] = round(tr["bytes_per_launch"])
        raw = tr["fetch"]["kernel_bytes_per_launch_raw"] + tr["write"]["kernel_bytes_per_launch_raw"]
        out["roofline"]["traffic_raw"] = round(raw)
        out["roofline"]["traffic_GBs"] = round(tr["bytes_per_launch"] / (per_launch_ms / 1e3) / 1e9, 1)
        out["roofline"]["traffic_raw_GBs"] = round(raw / (per_launch_ms / 1e3) / 1e9, 1)
        out["roofline"]["traffic_source"] = tr["source"]
    if not args.no_plain and mode_run == "batched":
        import graphgen as gg
        cand = g.non_isolated() if sources is None else sources
        ps = gg.sample(cand, min(args.plain_sample, len(cand)), 7)
        pst, pms = timed_compute(G, ps, stream, mode="plain", deg1=bool(prune), alpha=args.alpha)
        pg = pst["te"] / (pms / 1e3) / 1e9
        pbytes = alg_bytes(n, tn, pst["launches"], pst)
        pk = pst["kernel_ms"]
        out["plain"] = {"gteps": round(pg, 3), "sample_sources": int(len(ps)), "ms": round(pms, 1),
                        "avg_launch_ms": round(pk / max(pst["launches"], 1), 4),
                        "launch_gap_us": round((pms - pk) * 1e3 / max(pst["launches"], 1), 1),
                        "achieved_GBs": round(pbytes / (pk / 1e3) / 1e9, 1)}
        out["batched_over_plain"] = round(gteps / pg, 2)
        log(f"plain: {pg:.2f} GTEPS on {len(ps)} sources")
        if args.plain_graph > 0:
            gst, gms = timed_compute(G, ps, stream, mode="plain", deg1=bool(prune), alpha=args.alpha,
                                     graph_launches=args.plain_graph)
            gg_te = gst["te"] / (gms / 1e3) / 1e9
            out["plain"].update({"hip_graph_launches": args.plain_graph, "gteps_hip_graph": round(gg_te, 3),
                                 "ms_hip_graph": round(gms, 1),
                                 "per_launch_us_hip_graph": round(gms * 1e3 / max(gst["launches"], 1), 1),
                                 "per_launch_us": round(pms * 1e3 / max(pst["launches"], 1), 1)})
            log(f"plain from HIP graphs of {args.plain_graph} launches: {gg_te:.2f} GTEPS")
    if not args.no_serving:
        out["serving"] = serving_run(bcm, ctx, args.serving_graphs, args.serving_max_scale, args.serving_queries,
                                     args.serving_rho, args.serving_warmup, args.serving_inflight,
                                     budget_gb=args.serving_budget_gb)
        log(f"serving: {out['serving']}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, m, args.cpu_budget)
        log(f"cpu: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        copy_calibration(args.calibrate_copy, quiet=True)


if __name__ == "__main__":
    main()
