#!/usr/bin/env python3
"""Louvain TEPS on one MI355X.

A step is one whole Louvain run (section 3.2 of Sahu, arXiv 2301.12390: passes of local moving
and aggregation until convergence, tolerance 0.01 declining x10 per pass, then the modularity of
the result) through the C ABI of liblouvain.so, on a graph already resident in HBM.

Default workload: R-MAT scale 25 (33,554,432 vertices, edge factor 16, a,b,c,d = 0.57, 0.19,
0.19, 0.05, symmetrised, self-loops and repeats removed, weights uniform 1..16, int64 offsets,
seed 1), generated on the GPU. TEPS = input arcs / run time.

Printed (stdout, one JSON line): the metric, the roofline of the dominant kernel (the LDS-table
move kernel, algorithmic bytes over its HIP-event-timed launches in the timed region), and the
CPU oracle timed on a bounded sample of the same workload. Progress goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Louvain TEPS (R-MAT s25); batched graphs/s vs one-by-one; serving p50/p99 ms"
HBM_PEAK_GBPS = 8000.0
CSRC = os.path.join(ROOT, "paper_2301_12390_amd", "csrc")
# the kernel whose roofline a workload reports: its source file and its PMC summary
PMC_KERNELS = {
    "k_move_lds": (os.path.join(CSRC, "lv_kernels.hip"),
                   os.path.join(ROOT, "profiles", "k_move_lds_rmat25_pmc.md")),
    "k_radix_onesweep": (os.path.join(CSRC, "lv_prep.hip"),
                         os.path.join(ROOT, "profiles", "k_radix_onesweep_prepare_rmat25_pmc.md")),
}


def lib_flags(args):
    """Library flags every workload passes (LV_GRAPH_REPLAY with --graph-replay)."""
    from paper_2301_12390_amd import LV_GRAPH_REPLAY
    return LV_GRAPH_REPLAY if getattr(args, "graph_replay", False) else 0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes of the LDS-table move kernel (what the method must move, not cache lines):
# per decided vertex: its row offset (o = 4 or 8 B, the input's offset width), C[v] 4, K[v] 8,
# Sigma[own] 8, csize[own] 4, csize[best] 4 and its decision 4 -> o + 32 B; per arc: neighbour
# id 4, weight 4, C[neighbour] 4 -> 12 B; per distinct candidate community: Sigma[c] 8 B.
BYTES_PER_VERTEX_BASE = 32
BYTES_PER_ARC = 12
BYTES_PER_CANDIDATE = 8


def save_graph(path, workload, g):
    import numpy as np
    with open(path, "wb") as f:
        hdr = {"workload": workload, "n": g.n, "nnz": g.nnz,
               "offsets": str(g.offsets.dtype).replace("torch.", ""),
               "weights": str(g.weights.dtype).replace("torch.", "")}
        b = json.dumps(hdr).encode()
        f.write(len(b).to_bytes(8, "little"))
        f.write(b)
        for t in (g.offsets, g.indices, g.weights):
            t.cpu().numpy().tofile(f)


def load_graph(path, workload, dev):
    import numpy as np
    import torch
    from graphgen import Csr
    with open(path, "rb") as f:
        hl = int.from_bytes(f.read(8), "little")
        hdr = json.loads(f.read(hl).decode())
        assert hdr["workload"] == workload, (hdr["workload"], workload)
        n, nnz = hdr["n"], hdr["nnz"]
        off = np.fromfile(f, dtype=hdr["offsets"], count=n + 1)
        idx = np.fromfile(f, dtype=np.int32, count=nnz)
        w = np.fromfile(f, dtype=hdr["weights"], count=nnz)
    return Csr(n, torch.from_numpy(off).to(dev), torch.from_numpy(idx).to(dev),
               torch.from_numpy(w).to(dev), workload)


def kernel_src_sha(kernel="k_move_lds"):
    return hashlib.sha256(open(PMC_KERNELS[kernel][0], "rb").read()).hexdigest()


def load_traffic(workload, kernel="k_move_lds"):
    """Measured HBM bytes per launch of the kernel from its committed rocprofv3 PMC summary
    (its ```json block), if it was taken on this workload with the current kernel source."""
    try:
        text = open(PMC_KERNELS[kernel][1]).read()
        d = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if d.get("workload") != workload or d.get("kernel_src_sha256") != kernel_src_sha(kernel):
        return None
    return d.get("bytes_per_launch")


# The kernels of each move tier and of aggregation, for the per-tier PMC summary.
TIER_KERNELS = {
    "fused": ("k_move_lds",),
    "wg": ("k_move_grp7", "k_move_wg"),
    "hub": ("k_hub_part", "k_hub_reduce", "k_hub_decide"),
    "agg": ("k_merge_lds", "k_merge_part", "k_merge_reduce", "k_count_members", "k_fill_members",
            "k_label_ranges", "k_super_rows"),
}
TIERS_PMC = os.path.join(ROOT, "profiles", "move_tiers_rmat25_pmc.md")


def tiers_src_sha():
    return hashlib.sha256(open(os.path.join(CSRC, "lv_kernels.hip"), "rb").read()).hexdigest()


def load_tier_traffic(workload, tier):
    """Measured HBM bytes per launch of a tier (its kernels' FETCH_SIZE + WRITE_SIZE per class
    step or per aggregation) from the committed per-tier PMC summary, if it was taken on this
    workload with the current kernel source."""
    try:
        text = open(TIERS_PMC).read()
        d = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if d.get("workload") != workload or d.get("kernel_src_sha256") != tiers_src_sha():
        return None
    return d["tiers"].get(tier, {}).get("bytes_per_launch")


def summarize_tiers_pmc(fetch_csv, write_csv, bench_json, out_path, command, workload, copy_mib):
    """Per-tier HBM traffic of two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of
    `bench.py --steps 1 --warmup 0`: each counter scaled by what it reads for the plain copy of
    copy_mib MiB, summed over the tier's kernels and divided by the tier's launches in the run."""
    import numpy as np
    per = {}
    for ctr, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _read_csv(path) if r["Counter_Name"] == ctr]
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                and int(r["Grid_Size"]) > 0]
        if not copy:
            raise SystemExit(f"{path}: no calibration copy dispatch")
        scale = copy_mib * 1024.0 / max(copy)
        by_kernel = {}
        for r in rows:
            by_kernel.setdefault(_short_name(r["Kernel_Name"]).replace("void ", ""), []).append(
                float(r["Counter_Value"]) * 1024 * scale)
        per[ctr] = {"copy_raw_kib": max(copy), "scale": scale, "by_kernel": by_kernel}
    bj = json.load(open(bench_json))
    tl = {t["tier"]: t for t in bj["roofline_tiers"]}

    def tier_of(name):
        for tier, ks in TIER_KERNELS.items():
            if any(name.startswith(k + "<") or name == k for k in ks):
                return tier
        return None

    tiers = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        for k, vals in per[ctr]["by_kernel"].items():
            t = tier_of(k)
            if t is None:
                continue
            tiers.setdefault(t, {"fetch": 0.0, "write": 0.0})
            tiers[t]["fetch" if ctr == "FETCH_SIZE" else "write"] += float(np.sum(vals))
    for t, v in tiers.items():
        n = tl[t]["launches"] if t in tl else 0
        v["launches"] = n
        v["bytes_per_launch"] = (v["fetch"] + v["write"]) / n if n else None
        v["algorithmic_bytes_per_launch"] = tl[t]["bytes_per_launch"] if t in tl else None
        v["measured_over_algorithmic"] = (v["bytes_per_launch"] / v["algorithmic_bytes_per_launch"]
                                          if n and v["algorithmic_bytes_per_launch"] else None)
    d = {"workload": workload, "kernel_src_sha256": tiers_src_sha(), "tiers": tiers,
         "calibration": {"copy_bytes": copy_mib << 20,
                         "fetch_raw_kib": per["FETCH_SIZE"]["copy_raw_kib"],
                         "fetch_scale": per["FETCH_SIZE"]["scale"],
                         "write_raw_kib": per["WRITE_SIZE"]["copy_raw_kib"],
                         "write_scale": per["WRITE_SIZE"]["scale"]}}
    lines = [f"# HBM traffic of the move tiers and of aggregation, {workload}", "",
             "Made by (one counter per run, then this summary):", "", "```", command, "```", "",
             f"Calibration: a plain device copy of {copy_mib} MiB reads FETCH_SIZE = "
             f"{per['FETCH_SIZE']['copy_raw_kib']:.0f} KiB and WRITE_SIZE = "
             f"{per['WRITE_SIZE']['copy_raw_kib']:.0f} KiB, so the counters are scaled by "
             f"{per['FETCH_SIZE']['scale']:.3f} and {per['WRITE_SIZE']['scale']:.3f}.", "",
             "A launch is one class step's kernels of a move tier, or one pass's aggregation.", "",
             "| tier | kernels | launches | measured MB / launch | algorithmic MB / launch | "
             "measured / algorithmic |", "|---|---|---:|---:|---:|---:|"]
    for t in ("fused", "wg", "hub", "agg"):
        if t not in tiers or not tiers[t]["launches"]:
            continue
        v = tiers[t]
        lines.append(f"| {t} | {', '.join(TIER_KERNELS[t])} | {v['launches']} | "
                     f"{v['bytes_per_launch'] / 1e6:.1f} | "
                     f"{v['algorithmic_bytes_per_launch'] / 1e6:.1f} | "
                     f"{v['measured_over_algorithmic']:.2f}x |")
    lines += ["", "| kernel | dispatches | fetch MB / dispatch | write MB / dispatch |",
              "|---|---:|---:|---:|"]
    fk, wk = per["FETCH_SIZE"]["by_kernel"], per["WRITE_SIZE"]["by_kernel"]
    for k in sorted(fk, key=lambda k: -sum(fk[k]))[:14]:
        lines.append(f"| `{k}` | {len(fk[k])} | {np.mean(fk[k]) / 1e6:.1f} | "
                     f"{np.mean(wk.get(k, [0.0])) / 1e6:.1f} |")
    lines += ["", "```json", json.dumps(d, indent=1), "```"]
    open(out_path, "w").write("\n".join(lines) + "\n")


def cpu_baseline(g, res_trace, seconds, substeps, n_arcs_input):
    """The oracle (plain C, OpenMP) on a bounded sample: the class steps of the first
    local-moving iteration of pass 0 on the same graph, as many as fit in ~`seconds`. Its arc
    rate is scaled to the whole run by the arcs the run's iterations scan."""
    import numpy as np
    import oracle as O

    t0 = time.perf_counter()
    og = O.Graph.from_csr(g)
    st = O.State(og)
    classes = O.class_lists(og.n, 0, substeps)
    deg = np.diff(og.off)
    prep = time.perf_counter() - t0
    log(f"oracle prepared in {prep:.1f}s")
    arcs = 0
    steps = 0
    t1 = time.perf_counter()
    for vs in classes:
        O.sync_step(og, st, vs)
        arcs += int(deg[vs].sum())
        steps += 1
        if time.perf_counter() - t1 >= seconds:
            break
    el = time.perf_counter() - t1
    rate = arcs / el
    scanned = sum(t["fused_arcs"] + t["wg_arcs"] + t["hub_arcs"] for t in res_trace)
    est_run = scanned / rate
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": n_arcs_input / est_run,
        "unit": "TEPS",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{steps} of {substeps} synchronous class steps of pass 0 iteration 0 "
                   f"({arcs} arcs, {el:.1f}s); run time estimated as the {scanned} arcs the "
                   f"run's local-moving iterations scan at that rate (aggregation excluded)"),
        "sample_seconds": round(el, 3),
        "arcs_per_second": rate,
    }


def _read_csv(path):
    import csv
    import gzip
    opener = gzip.open if path.endswith(".gz") else open
    with opener(path, "rt") as f:
        return list(csv.DictReader(f))


def _short_name(name):
    name = name.replace("lv::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0] if "(" in name else name


def summarize_stats(csv_path, out_path, command, title="R-MAT scale 25 Louvain runs"):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` kernel_stats.csv."""
    rows = _read_csv(csv_path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows if "lv::" in r["Name"])
    overlap = any("k_move_lds" in r["Name"] for r in rows)
    lines = [f"# Kernel time, {title}", "",
             "Made by:", "", "```", command, "```", "",
             f"Library kernels total: {total / 1e6:.1f} ms over all profiled runs "
             "(warm-up and timed steps)." + (
                 " The move kernels of a class step run concurrently on up to three streams, "
                 "so their durations overlap: shares are of summed kernel time, not of wall "
                 "time." if overlap else ""), "",
             "| kernel | calls | total ms | average us | share |",
             "|---|---:|---:|---:|---:|"]
    for r in rows:
        if "lv::" not in r["Name"]:
            continue
        t = float(r["TotalDurationNs"])
        lines.append(f"| `{_short_name(r['Name'])}` | {int(r['Calls'])} | {t / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {100 * t / total:.1f}% |")
    open(out_path, "w").write("\n".join(lines) + "\n")


def summarize_pmc(fetch_csv, write_csv, bench_json, out_path, command, workload, copy_mib,
                  kernel="k_move_lds"):
    """Markdown summary of the FETCH_SIZE and WRITE_SIZE passes: per-launch HBM bytes of
    `kernel`, each counter scaled by what it reads for the plain copy of copy_mib MiB."""
    import numpy as np
    per = {}
    for ctr, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _read_csv(path) if r["Counter_Name"] == ctr]
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                and int(r["Grid_Size"]) > 0]
        if not copy:
            raise SystemExit(f"{path}: no calibration copy dispatch")
        copy_kib = max(copy)
        scale = copy_mib * 1024.0 / copy_kib
        by_kernel = {}
        for r in rows:
            by_kernel.setdefault(_short_name(r["Kernel_Name"]), []).append(
                float(r["Counter_Value"]))
        per[ctr] = {"copy_raw_kib": copy_kib, "scale": scale, "by_kernel": by_kernel}
    key = [k for k in per["FETCH_SIZE"]["by_kernel"]
           if k.replace("void ", "").replace("(anonymous namespace)::", "").startswith(kernel)]
    fetch = np.concatenate([per["FETCH_SIZE"]["by_kernel"][k] for k in key])
    write = np.concatenate([per["WRITE_SIZE"]["by_kernel"][k] for k in key])
    fs, ws = per["FETCH_SIZE"]["scale"], per["WRITE_SIZE"]["scale"]
    fetch_b = float(fetch.mean()) * 1024 * fs
    write_b = float(write.mean()) * 1024 * ws
    bj = json.load(open(bench_json))
    alg = bj["roofline"]["algorithmic_bytes_per_launch"]
    d = {"workload": workload, "kernel": kernel, "kernel_src_sha256": kernel_src_sha(kernel),
         "launches": int(fetch.size),
         "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
         "bytes_per_launch": fetch_b + write_b,
         "algorithmic_bytes_per_launch": alg,
         "calibration": {"copy_bytes": copy_mib << 20,
                         "fetch_raw_kib": per["FETCH_SIZE"]["copy_raw_kib"], "fetch_scale": fs,
                         "write_raw_kib": per["WRITE_SIZE"]["copy_raw_kib"], "write_scale": ws}}
    lines = [f"# HBM traffic of {kernel}, {workload}", "",
             "Made by (one counter per run, then this summary):", "", "```", command, "```", "",
             f"Calibration: a plain device copy of {copy_mib} MiB reads FETCH_SIZE = "
             f"{per['FETCH_SIZE']['copy_raw_kib']:.0f} KiB and WRITE_SIZE = "
             f"{per['WRITE_SIZE']['copy_raw_kib']:.0f} KiB, so the counters are scaled by "
             f"{fs:.3f} and {ws:.3f}.", "",
             f"{kernel} over {fetch.size} launches: {fetch_b / 1e6:.1f} MB fetched and "
             f"{write_b / 1e6:.1f} MB written per launch, against {alg / 1e6:.1f} MB of "
             f"algorithmic bytes ({(fetch_b + write_b) / alg:.2f}x).", "",
             "| kernel | launches | fetch MB / launch | write MB / launch |",
             "|---|---:|---:|---:|"]
    fk = per["FETCH_SIZE"]["by_kernel"]
    wk = per["WRITE_SIZE"]["by_kernel"]
    tops = sorted(fk, key=lambda k: -sum(fk[k]))[:12]
    for k in tops:
        f = np.mean(fk[k]) * 1024 * fs / 1e6
        w = np.mean(wk.get(k, [0.0])) * 1024 * ws / 1e6
        lines.append(f"| `{k.replace('void ', '')}` | {len(fk[k])} | {f:.1f} | {w:.1f} |")
    lines += ["", "```json", json.dumps(d, indent=1), "```"]
    open(out_path, "w").write("\n".join(lines) + "\n")


def run_batched_bench(args, dev):
    """The batched workload: graphs/s of one louvain_run_batched call over the whole batch,
    against louvain_run called graph by graph (timed once over the whole batch)."""
    print(json.dumps(batched_measure(args, dev, args.steps, args.warmup,
                                     not args.no_cpu_baseline)), flush=True)


def batched_measure(args, dev, steps, warmup, with_cpu):
    """The batched workload's JSON record (see run_batched_bench)."""
    import torch

    import oracle as O
    from graphgen import batch_config, pack_graphs
    from paper_2301_12390_amd import Louvain

    t0 = time.perf_counter()
    graphs = batch_config(args.batch_count, device=dev)
    packed, vptr, aptr = pack_graphs(graphs, device=dev)
    torch.cuda.synchronize()
    G = len(graphs)
    log(f"generated {G} graphs: n={packed.n} nnz={packed.nnz} in "
        f"{time.perf_counter() - t0:.1f}s")
    lv = Louvain(0)
    for w in range(warmup):
        _, res = lv.run_batched(packed, vptr, aptr, substeps=args.substeps,
                                 flags=lib_flags(args))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        memb, res = lv.run_batched(packed, vptr, aptr, substeps=args.substeps,
                                 flags=lib_flags(args))
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    ms_per_step = el * 1000.0 / steps
    gps = G / (ms_per_step / 1000.0)
    log(f"batched: {ms_per_step:.1f} ms per batch, {gps:.1f} graphs/s")
    # one by one, over the same graphs already in HBM
    obo_gps, same = None, None
    if not args.no_one_by_one:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        q_single = []
        for g in graphs:
            _, r = lv.run(g, substeps=args.substeps, flags=lib_flags(args))
            q_single.append(r["qnum"])
        torch.cuda.synchronize()
        obo = time.perf_counter() - t2
        obo_gps = G / obo
        same = all(a == b["qnum"] for a, b in zip(q_single, res))
        log(f"one by one: {obo * 1000:.1f} ms, {obo_gps:.1f} graphs/s; identical Qnum: {same}")
    qs = [r["q"] for r in res]
    line = {
        "metric": METRIC,
        "value": gps,
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i64",
        "data": "synthetic",
        "config": {
            "workload": "batched",
            "graphs": G,
            "n": packed.n,
            "nnz": packed.nnz,
            "substeps": args.substeps,
            "teps": packed.nnz / (ms_per_step / 1000.0),
            "one_by_one_graphs_per_s": obo_gps,
            "speedup_vs_one_by_one": gps / obo_gps if obo_gps else None,
            "identical_to_one_by_one": same,
            "mean_q": sum(qs) / len(qs),
        },
        "roofline": None,
    }
    lv.close()
    if with_cpu:
        # the oracle's whole runs on the batch's graphs in order, until ~cpu_seconds
        done_arcs = 0
        k = 0
        t3 = time.perf_counter()
        for g in graphs:
            O.run(O.Graph.from_csr(g.to("cpu")), "sync", substeps=args.substeps)
            done_arcs += g.nnz
            k += 1
            if time.perf_counter() - t3 >= args.cpu_seconds:
                break
        el3 = time.perf_counter() - t3
        rate = done_arcs / el3
        line["cpu_baseline"] = {
            "value": G / (packed.nnz / rate),
            "unit": "graphs/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "kind": "oracle",
            "sample": (f"whole oracle runs on the first {k} graphs of the batch ({done_arcs} "
                       f"arcs, {el3:.1f}s); graphs/s estimated from that arc rate over the "
                       f"batch's {packed.nnz} arcs"),
        }
        log(f"cpu baseline: {line['cpu_baseline']['value']:.2f} graphs/s")
    return line


def run_serving_bench(args, dev):
    """Serving (see serving_measure), printed as its own JSON line."""
    print(json.dumps(serving_measure(args, dev)), flush=True)


def serving_measure(args, dev, seconds=None, servers=None):
    """Serving: Poisson arrivals of requests drawn from a pool of pre-generated graphs held in
    pinned host memory, submitted at their arrival times to the library's request server
    (louvain_server_*). Latency is arrival to membership in host memory (queueing, packing, H2D
    and D2H included), from the server's own clock. Every trace runs through three servers:
    continuous batching (--serve-slots runs in flight, each batching up to --serve-batch-arcs),
    batch-at-a-time (one slot that batches), and one-at-a-time FIFO (one slot, no batching)."""
    import numpy as np
    import torch

    from graphgen import serving_pool
    from paper_2301_12390_amd import Server

    t0 = time.perf_counter()
    pool = serving_pool(args.pool, device=dev)
    torch.cuda.synchronize()
    host = []
    for g in pool:
        host.append((g.n, g.offsets.to(torch.int64).cpu().pin_memory(),
                     g.indices.cpu().pin_memory(), g.weights.cpu().pin_memory()))
    sizes = [h[0] for h in host]
    arcs = [int(h[2].numel()) for h in host]
    del pool
    torch.cuda.empty_cache()
    log(f"request pool: {len(host)} graphs, n {min(sizes)}..{max(sizes)}, mean arcs "
        f"{sum(arcs) / len(arcs):.0f}, generated in {time.perf_counter() - t0:.1f}s")

    serve_seconds = args.serve_seconds if seconds is None else seconds

    def run_trace(rate, name, slots, batch_arcs):
        """One arrival trace (seeded per rate, the same for every server) through a server.
        Arrivals stop at serve_seconds; requests not done by twice that are counted
        unfinished (the server is then destroyed, which drops them)."""
        rng = np.random.default_rng(1000 + int(rate))
        arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * serve_seconds * 2) + 16))
        arr = arr[arr <= serve_seconds]
        which = rng.integers(0, len(host), size=arr.size)
        srv = Server(0, slots=slots, hbm_budget=int(args.serve_budget_gb * (1 << 30)),
                     batch_arcs=batch_arcs, substeps=args.substeps, flags=lib_flags(args))
        # warm-up: every slot's buffers and workspace grown on the largest pool graph
        big = int(np.argmax(arcs))
        for t in [srv.submit(*host[big]) for _ in range(slots)]:
            srv.wait(t)
        base = srv.stats()
        tickets = []
        start = srv.clock_ns()
        for i in range(arr.size):
            lag = arr[i] - (srv.clock_ns() - start) * 1e-9
            if lag > 0:
                time.sleep(lag)
            tickets.append(srv.submit(*host[int(which[i])]))
        deadline = start + int(serve_seconds * 2 * 1e9)
        lat, done_at, batches = [], [], []
        for i, t in enumerate(tickets):
            left_ms = (deadline - srv.clock_ns()) // 1_000_000
            r = srv.wait(t, timeout_ms=max(int(left_ms), 0))
            if r is None:
                break
            out = r[1]
            if out["status"] != 0:
                raise RuntimeError(f"request {i} failed: {out['error']}")
            lat.append((out["done_ns"] - (start + int(arr[i] * 1e9))) * 1e-6)
            done_at.append(out["done_ns"])
            batches.append(out["batch_graphs"])
        st = srv.stats()
        end = max(done_at) if done_at else srv.clock_ns()
        srv.close()
        el = (end - start) * 1e-9
        lat_ms = np.array(lat)
        rec = {
            "rate": rate, "server": name, "slots": slots, "batch_arcs": batch_arcs,
            "offered": int(arr.size), "completed": len(lat),
            "unfinished": int(arr.size - len(lat)),
            "completed_per_s": len(lat) / max(el, 1e-9),
            "p50_ms": float(np.percentile(lat_ms, 50)) if lat else None,
            "p99_ms": float(np.percentile(lat_ms, 99)) if lat else None,
            "runs": st["runs"] - base["runs"],
            "mean_batch": float(np.mean(batches)) if batches else None,
            "peak_running": st["peak_running"],
            "peak_held_gb": st["peak_held_bytes"] / 2**30,
            "seconds": el,
        }
        log(f"{name} rate {rate:g}/s: {rec['completed']} of {rec['offered']} done, "
            f"{rec['completed_per_s']:.1f}/s, p50 {rec['p50_ms']:.1f} ms, "
            f"p99 {rec['p99_ms']:.1f} ms, {rec['runs']} runs, mean batch "
            f"{rec['mean_batch']:.2f}, peak running {rec['peak_running']}")
        return rec

    all_servers = [("continuous", args.serve_slots, args.serve_batch_arcs),
                   ("batch_at_a_time", 1, args.serve_single_batch_arcs), ("fifo", 1, 0)]
    if servers is None:
        servers = ["continuous"] + ([] if args.no_fifo else ["batch_at_a_time", "fifo"])
    servers = [x for x in all_servers if x[0] in servers]
    per = {name: [] for name, _, _ in servers}
    for rate in [float(x) for x in args.rates.split(",")]:
        for name, slots, ba in servers:
            per[name].append(run_trace(rate, name, slots, ba))
    first = per["continuous"][0]
    line = {
        "metric": METRIC,
        "value": first["p99_ms"],
        "unit": "ms (p99 latency at the first rate)",
        "n_gpus": 1,
        "steps": len(per["continuous"]),
        "warmup": 1,
        "ms_per_step": first["p50_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i64",
        "data": "synthetic",
        "config": {
            "workload": "serving",
            "pool_graphs": len(host),
            "pool_mean_arcs": sum(arcs) / len(arcs),
            "serve_seconds": serve_seconds,
            "slots": args.serve_slots,
            "batch_arc_budget": args.serve_batch_arcs,
            "single_slot_batch_arc_budget": args.serve_single_batch_arcs,
            "hbm_budget_gb": args.serve_budget_gb,
            "substeps": args.substeps,
            "rates": per["continuous"],
            "batch_at_a_time_rates": per.get("batch_at_a_time", []),
            "fifo_rates": per.get("fifo", []),
        },
        "roofline": None,
    }
    return line


def run_sweep_bench(args, dev):
    """Tolerance and decline-factor sweep (section 3.2's parameter study): Q, time, iterations
    and passes of louvain_run for initial tolerance 10^-a and decline factor 10^b on the
    synthetic graphs, with the sequential asynchronous oracle's Q beside them where it is cheap
    (graphs of up to ~2e7 arcs)."""
    import torch

    import oracle as O
    from graphgen import config_graph
    from paper_2301_12390_amd import Louvain

    lv = Louvain(0)
    tols = [int(x) for x in args.sweep_tolerances.split(",")]
    decls = [int(x) for x in args.sweep_declines.split(",")]
    grid = [(a, 1) for a in tols] + [(2, b) for b in decls if b != 1]
    out = []
    for name in args.sweep_graphs.split(","):
        g = config_graph(name, device=dev)
        torch.cuda.synchronize()
        q_async = None
        if g.nnz <= args.sweep_async_arcs:
            _, ra = O.run(O.Graph.from_csr(g.to("cpu")), "async")
            q_async = ra["q"]
        rows = []
        for a, b in grid:
            lv.run(g, tolerance_exp10=a, decline_exp10=b, substeps=args.substeps)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r = lv.run(g, tolerance_exp10=a, decline_exp10=b, substeps=args.substeps)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1000.0
            rows.append({"tolerance": f"1e-{a}", "decline": 10 ** b, "q": r["q"],
                         "ms": ms, "passes": r["passes"], "iterations": r["iterations"],
                         "iterations_total": r["iterations_total"], "cap_hits": r["cap_hits"]})
            log(f"{name} tol 1e-{a} decline 1e{b}: Q {r['q']:.6f}, {ms:.1f} ms, "
                f"{r['iterations_total']} iterations in {r['passes']} passes")
        out.append({"graph": name, "n": g.n, "nnz": g.nnz, "q_async_oracle": q_async,
                    "runs": rows})
        del g
        torch.cuda.empty_cache()
    lv.close()
    base = next(r for r in out[-1]["runs"] if r["tolerance"] == "1e-2" and r["decline"] == 10)
    line = {
        "metric": METRIC,
        "value": out[-1]["nnz"] / (base["ms"] / 1000.0),
        "unit": "TEPS (last graph, tolerance 1e-2, decline 10)",
        "n_gpus": 1, "steps": len(grid), "warmup": 1, "ms_per_step": base["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i64",
        "data": "synthetic",
        "config": {"workload": "sweep", "substeps": args.substeps, "graphs": out},
        "roofline": None,
    }
    print(json.dumps(line), flush=True)


def run_table_bench(args, dev):
    """The per-config table of the baseline: for each --table-graphs workload, its size, W and
    SHA-256; the synchronous oracle (O1, --substeps classes, all host threads) and the
    sequential asynchronous oracle (O2, one core) timed on the host, each once after building
    its input; and the GPU run (median of 5 after one warm-up): time, TEPS, Q."""
    import statistics

    import torch

    import oracle as O
    from graphgen import config_graph, csr_sha256
    from paper_2301_12390_amd import Louvain

    lv = Louvain(0)
    rows = []
    for name in args.table_graphs.split(","):
        g = config_graph(name, device=dev)
        torch.cuda.synchronize()
        lv.run(g, substeps=args.substeps, flags=lib_flags(args))
        ms = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r = lv.run(g, substeps=args.substeps, flags=lib_flags(args))
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1000.0)
        gpu_ms = statistics.median(ms)
        log(f"{name}: GPU {gpu_ms:.2f} ms, Q {r['q']:.6f}; oracle runs next")
        gc = g.to("cpu")
        og = O.Graph.from_csr(gc)
        t0 = time.perf_counter()
        _, r1 = O.run(og, "sync", substeps=args.substeps)
        o1 = time.perf_counter() - t0
        log(f"{name}: synchronous oracle {o1:.1f} s")
        t0 = time.perf_counter()
        _, r2 = O.run(og, "async")
        o2 = time.perf_counter() - t0
        log(f"{name}: asynchronous oracle {o2:.1f} s")
        row = {"graph": name, "n": g.n, "nnz": g.nnz, "W": r["W"], "csr_sha256": csr_sha256(gc),
               "o1_s": o1, "o1_teps": g.nnz / o1, "o1_q": r1["q"],
               "o1_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "o2_s": o2, "o2_teps": g.nnz / o2, "o2_q": r2["q"],
               "gpu_ms": gpu_ms, "gpu_teps": g.nnz / (gpu_ms / 1000.0), "gpu_q": r["q"],
               "gpu_equals_o1": r["qnum"] == r1["qnum"]}
        rows.append(row)
        log(f"{name}: {row}")
        del g, gc, og
        torch.cuda.empty_cache()
    lv.close()
    print(json.dumps({"metric": METRIC, "config": {"workload": "table", "rows": rows}}),
          flush=True)


def calibration_copy(args, dev):
    """A plain device copy of --copy-calibration-mib MiB, the known-size reference that scales
    the FETCH_SIZE / WRITE_SIZE counters of a --pmc run."""
    import torch
    if args.copy_calibration_mib <= 0:
        return
    words = args.copy_calibration_mib * (1 << 18)
    src = torch.ones(words, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy of {args.copy_calibration_mib} MiB done")
    del src, dst
    torch.cuda.empty_cache()


# Algorithmic bytes of one stable scatter pass of the preparation sort, per arc: its 8-byte key
# read once and written once (the paper's recipe has no input weights, so no weight array is
# sorted; with input weights 4 more bytes each way).
PREP_SCATTER_BYTES_PER_ARC = 16


def run_prepare_bench(args, dev):
    """Graph preparation (section 3.1.2 and Table 1): a raw R-MAT edge list (repeats and
    self-loops included, as an edge-list file holds it) through louvain_prepare with the paper's
    recipe (reverse edges, unit weights, a loop on every vertex, repeats combined). A step is
    one louvain_prepare call on the edge list already in HBM."""
    import numpy as np
    import torch

    import oracle as O
    from graphgen import rmat_edges
    from paper_2301_12390_amd import LV_PREP_PAPER, Louvain
    from paper_2301_12390_amd.louvain import LV_PREP_TRACE

    t0 = time.perf_counter()
    tag = f"rmat{args.prep_scale}-edges"
    if args.graph_cache and os.path.exists(args.graph_cache):
        with open(args.graph_cache, "rb") as f:
            hdr = json.loads(f.read(int.from_bytes(f.read(8), "little")).decode())
            assert hdr["workload"] == tag, (hdr["workload"], tag)
            n, m = hdr["n"], hdr["m"]
            src = torch.from_numpy(np.fromfile(f, dtype=np.int32, count=m)).to(dev)
            dst = torch.from_numpy(np.fromfile(f, dtype=np.int32, count=m)).to(dev)
        log(f"loaded the {tag} list: n={n} m={m} in {time.perf_counter() - t0:.1f}s")
    else:
        n, u, v = rmat_edges(args.prep_scale, device=dev)
        src = u.to(torch.int32).contiguous()
        dst = v.to(torch.int32).contiguous()
        del u, v
        torch.cuda.synchronize()
        m = int(src.numel())
        log(f"generated the {tag} list: n={n} m={m} in {time.perf_counter() - t0:.1f}s")
        if args.graph_cache:
            with open(args.graph_cache, "wb") as f:
                b = json.dumps({"workload": tag, "n": n, "m": m}).encode()
                f.write(len(b).to_bytes(8, "little"))
                f.write(b)
                src.cpu().numpy().tofile(f)
                dst.cpu().numpy().tofile(f)
            log(f"saved to {args.graph_cache}")
    torch.cuda.empty_cache()
    if args.steps <= 0:
        return
    calibration_copy(args, dev)
    lv = Louvain(0)
    flags = LV_PREP_PAPER | LV_PREP_TRACE
    for w in range(args.warmup):
        g = lv.prepare(n, src, dst, flags=flags)
        log(f"warmup {w}: {g.stats['total_ms']:.1f} ms, nnz={g.nnz}")
        del g
    torch.cuda.synchronize()
    stats = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g = lv.prepare(n, src, dst, flags=flags)
        stats.append(g.stats)
        nnz = g.nnz
        del g
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    ms_per_step = el * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, "
        f"{m / (ms_per_step / 1000.0) / 1e9:.3f} G input edges/s")
    arcs = stats[0]["arcs"]
    passes = stats[0]["sort_passes"]
    scatter_ms = sum(s_["scatter_ms"] for s_ in stats)
    launches = passes * len(stats)
    avg_ms = scatter_ms / max(launches, 1)
    bytes_per_launch = PREP_SCATTER_BYTES_PER_ARC * arcs
    achieved = bytes_per_launch / (avg_ms / 1000.0) / 1e9 if avg_ms > 0 else 0.0
    traffic = load_traffic(f"prepare-rmat{args.prep_scale}", "k_radix_onesweep")
    phases = {k: sum(s_[k] for s_ in stats) / len(stats)
              for k in ("expand_ms", "hist_ms", "scan_ms", "scatter_ms", "emit_ms", "total_ms")}
    line = {
        "metric": METRIC,
        "value": m / (ms_per_step / 1000.0),
        "unit": "input edges/s (graph preparation)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"prepare-rmat{args.prep_scale}", "n": n, "edges": m,
                   "arcs_before_combining": arcs, "nnz": nnz,
                   "recipe": "reverse edges, unit weights, self-loop per vertex, repeats "
                             "combined (max)",
                   "key_bits": stats[0]["key_bits"], "sort_passes": passes,
                   "phase_ms_per_step": phases},
        "roofline": {
            "kernel": "k_radix_onesweep", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "traffic_gbps": (traffic / (avg_ms / 1000.0) / 1e9 if traffic and avg_ms > 0
                             else None),
            "avg_launch_ms": avg_ms, "launches": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
    }
    lv.close()
    if not args.no_cpu_baseline:
        # the oracle's preparation of the edge list's first k edges, k doubling until about a
        # third of cpu_seconds; without the n added loops, which would not shrink with k
        hs = src.cpu().numpy()
        hd = dst.cpu().numpy()
        k = 1 << 20
        done = 0
        el3 = 0.0
        while True:
            t3 = time.perf_counter()
            O.prepare(n, hs[:k], hd[:k], None, O.PREP_SYM | O.PREP_MAX)
            el3 = time.perf_counter() - t3
            done = k
            if el3 >= args.cpu_seconds / 3 or 2 * k > m:
                break
            k *= 2
        line["cpu_baseline"] = {
            "value": done / el3, "unit": "input edges/s (graph preparation)", "cores": 1,
            "kind": "oracle",
            "sample": (f"the oracle's preparation (reverse edges, combine repeats; the "
                       f"{n} added loops left out) of the first {done} edges of the same edge "
                       f"list ({el3:.1f}s, single-threaded sort)"),
        }
        log(f"cpu baseline: {done / el3 / 1e6:.2f} M edges/s")
    print(json.dumps(line), flush=True)


def run_colour_bench(args, dev, g):
    """Colour classes (LV_COLOR_CLASSES) on the workload graph: louvain_colour_classes for pass
    0 timed on its own (a step), then one whole run with colour classes beside one with hashed
    classes (Q, iterations, time)."""
    import torch

    from paper_2301_12390_amd import LV_COLOR_CLASSES, Louvain

    lv = Louvain(0)
    K = args.substeps
    for _ in range(args.warmup):
        lv.colour_classes(g, 0, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c, rounds = lv.colour_classes(g, 0, K)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    sizes = torch.bincount(c.to(torch.int64), minlength=K).cpu().tolist()
    log(f"colouring: {ms:.1f} ms, {rounds} rounds enqueued, class sizes {sizes}")
    runs = {}
    for name, fl in (("colour", LV_COLOR_CLASSES), ("hash", 0)):
        lv.run(g, substeps=K, flags=fl)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, r = lv.run(g, substeps=K, flags=fl)
        torch.cuda.synchronize()
        runs[name] = {"ms": (time.perf_counter() - t1) * 1000.0, "q": r["q"],
                      "passes": r["passes"], "iterations": r["iterations"]}
        log(f"run with {name} classes: {runs[name]}")
    lv.close()
    line = {
        "metric": METRIC, "value": g.n / (ms / 1000.0), "unit": "vertices coloured/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"colour-{args.workload}", "n": g.n, "nnz": g.nnz, "K": K,
                   "rounds_enqueued": rounds, "class_sizes": sizes, "runs": runs},
        "roofline": None,
    }
    print(json.dumps(line), flush=True)


def run_partition_bench(args, dev, g):
    """Partition and merge on the workload graph: louvain_run_partitioned for each P of
    --partitions beside the direct louvain_run (time, Q, the parts' and the merge's share)."""
    import torch

    from paper_2301_12390_amd import Louvain

    lv = Louvain(0)
    out = []
    for P in [int(x) for x in args.partitions.split(",")]:
        for _ in range(args.warmup):
            lv.run_partitioned(g, P=P, substeps=args.substeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, res, pr = lv.run_partitioned(g, P=P, substeps=args.substeps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        row = {"P": P, "ms": ms, "q": res["q"], "merge_ms": res["total_ms"],
               "merge_passes": res["passes"], "merge_iterations": res["iterations"],
               "part_communities": sum(p["n_communities"] for p in pr),
               "max_part_iterations": max(sum(p["iterations"]) for p in pr)}
        out.append(row)
        log(f"P={P}: {ms:.1f} ms, Q {res['q']:.6f}, merge {res['total_ms']:.1f} ms")
    for _ in range(args.warmup):
        lv.run(g, substeps=args.substeps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rd = lv.run(g, substeps=args.substeps)
    torch.cuda.synchronize()
    direct_ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    log(f"direct: {direct_ms:.1f} ms, Q {rd['q']:.6f}")
    lv.close()
    best = min(out, key=lambda r: r["ms"])
    line = {
        "metric": METRIC, "value": g.nnz / (best["ms"] / 1000.0),
        "unit": f"TEPS (partition and merge, P = {best['P']})", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i64",
        "data": "synthetic",
        "config": {"workload": f"partitioned-{args.workload}", "n": g.n, "nnz": g.nnz,
                   "substeps": args.substeps, "runs": out,
                   "direct": {"ms": direct_ms, "q": rd["q"], "iterations": rd["iterations"]}},
        "roofline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch-count", type=int, default=2048,
                    help="graphs of the batched workload")
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="batched: skip the graph-by-graph comparison run")
    ap.add_argument("--sweep-graphs", default="sbm10k,rmat22",
                    help="sweep: workloads to sweep (config names)")
    ap.add_argument("--sweep-tolerances", default="0,1,2,3,4,6,8,12",
                    help="sweep: initial tolerance exponents a (tolerance 10^-a), decline 10")
    ap.add_argument("--sweep-declines", default="1,2,3,4",
                    help="sweep: decline exponents b (factor 10^b) at tolerance 1e-2")
    ap.add_argument("--sweep-async-arcs", type=int, default=20000000,
                    help="sweep: largest graph (arcs) given the asynchronous oracle's Q")
    ap.add_argument("--table-graphs", default="sbm10k,rmat22",
                    help="table: workloads of the per-config baseline table")
    ap.add_argument("--rates", default="50,200,800",
                    help="serving: request rates (per second), comma separated")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="serving: seconds of arrivals per rate (the queue then drains)")
    ap.add_argument("--pool", type=int, default=32, help="serving: distinct request graphs")
    ap.add_argument("--no-fifo", action="store_true",
                    help="serving: skip the batch-at-a-time and one-at-a-time servers")
    ap.add_argument("--serve-slots", type=int, default=6,
                    help="serving: runs in flight at once in the continuous-batching server")
    ap.add_argument("--serve-single-batch-arcs", type=int, default=1 << 28,
                    help="serving: most arcs of one run of the batch-at-a-time server")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0,
                    help="serving: device memory budget of the server (GiB)")
    ap.add_argument("--serve-batch-arcs", type=int, default=1 << 25,
                    help="serving: most arcs of one run of the continuous-batching server")
    ap.add_argument("--prep-scale", type=int, default=25,
                    help="prepare: R-MAT scale of the raw edge list")
    ap.add_argument("--workload", default="rmat25",
                    help="rmat25 (default), rmat22, sbm10k, rmatNN, batched (the batch of "
                         "--batch-count SBM and lattice graphs, graphs/s), serving (Poisson "
                         "requests at --rates, p50/p99 latency), sweep (tolerance and "
                         "decline-factor study) or prepare (graph preparation of a raw R-MAT "
                         "edge list of --prep-scale)")
    ap.add_argument("--partitions", default="",
                    help="time partition and merge (louvain_run_partitioned) for these part "
                         "counts, comma separated, beside the direct run")
    ap.add_argument("--colour-bench", action="store_true",
                    help="time the colouring behind LV_COLOR_CLASSES on the workload graph, and "
                         "one run with colour classes beside one with hashed classes")
    ap.add_argument("--colour-classes", action="store_true",
                    help="vertex classes from the device colouring (LV_COLOR_CLASSES) instead "
                         "of the hash")
    ap.add_argument("--substeps", type=int, default=8,
                    help="vertex classes per local-moving iteration (1 = fully synchronous)")
    ap.add_argument("--no-trace", action="store_true",
                    help="time runs without LV_TRACE's per-kernel events (latency of small "
                         "graphs; no roofline)")
    ap.add_argument("--graph-replay", action="store_true",
                    help="replay small phases' iterations as captured HIP graphs "
                         "(LV_GRAPH_REPLAY) instead of launching every kernel directly")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload: skip the fully synchronous run, the batched "
                         "workload and the serving traces that the line also reports")
    ap.add_argument("--extra-serve-seconds", type=float, default=5.0,
                    help="default workload: seconds of arrivals per rate of its serving traces")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph-cache", default="",
                    help="file to load the workload graph from, or to save it to after "
                         "generating it (raw little-endian arrays)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB once (a plain "
                         "copy kernel of known size, to scale profiler byte counters)")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("KERNEL_STATS_CSV", "OUT_MD"),
                    help="write a markdown summary of a rocprofv3 --stats run and exit")
    ap.add_argument("--summarize-pmc", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON", "OUT_MD"),
                    help="write the k_move_lds HBM-traffic summary of two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE; with --copy-calibration-mib) and exit")
    ap.add_argument("--summarize-tiers-pmc", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON", "OUT_MD"),
                    help="write the per-tier HBM-traffic summary of two rocprofv3 --pmc runs "
                         "of bench.py --steps 1 --warmup 0 --no-extra (FETCH_SIZE, WRITE_SIZE; "
                         "with --copy-calibration-mib) and exit")
    ap.add_argument("--command", default="", help="command text recorded in a summary")
    ap.add_argument("--summary-title", default="R-MAT scale 25 Louvain runs",
                    help="what a --summarize-stats summary covers")
    ap.add_argument("--pmc-kernel", default="k_move_lds", choices=sorted(PMC_KERNELS),
                    help="kernel a --summarize-pmc summary covers")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, args.command, args.summary_title)
        return
    if args.summarize_tiers_pmc:
        summarize_tiers_pmc(*args.summarize_tiers_pmc, args.command, args.workload,
                            args.copy_calibration_mib or 1024)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.command, args.workload,
                      args.copy_calibration_mib or 1024, args.pmc_kernel)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from graphgen import config_graph
    from paper_2301_12390_amd import LV_COLOR_CLASSES, LV_TRACE, Louvain
    from paper_2301_12390_amd import build as lib_build

    if not os.path.exists(lib_build.LIB):
        lib_build.build()
    dev = torch.device("cuda:0")
    log(f"device {torch.cuda.get_device_name(0)}")
    if args.workload == "batched":
        run_batched_bench(args, dev)
        return
    if args.workload == "serving":
        run_serving_bench(args, dev)
        return
    if args.workload == "sweep":
        run_sweep_bench(args, dev)
        return
    if args.workload == "prepare":
        run_prepare_bench(args, dev)
        return
    if args.workload == "table":
        run_table_bench(args, dev)
        return
    t0 = time.perf_counter()
    if args.graph_cache and os.path.exists(args.graph_cache):
        g = load_graph(args.graph_cache, args.workload, dev)
        log(f"loaded {args.workload}: n={g.n} nnz={g.nnz} in {time.perf_counter() - t0:.1f}s")
    else:
        g = config_graph(args.workload, device=dev)
        torch.cuda.synchronize()
        log(f"generated {args.workload}: n={g.n} nnz={g.nnz} in {time.perf_counter() - t0:.1f}s")
        if args.graph_cache:
            save_graph(args.graph_cache, args.workload, g)
            log(f"saved to {args.graph_cache}")
    torch.cuda.empty_cache()
    if args.steps <= 0:
        return
    if args.colour_bench:
        run_colour_bench(args, dev, g)
        return
    if args.partitions:
        run_partition_bench(args, dev, g)
        return

    calibration_copy(args, dev)

    lv = Louvain(0)
    run_flags = ((0 if args.no_trace else LV_TRACE) |
                 (LV_COLOR_CLASSES if args.colour_classes else 0) |
                 lib_flags(args))
    for w in range(args.warmup):
        _, res = lv.run(g, substeps=args.substeps, flags=run_flags)
        log(f"warmup {w}: {res['total_ms']:.1f} ms, Q={res['q']:.6f}, passes={res['passes']}, "
            f"iterations={res['iterations']}")
    torch.cuda.synchronize()
    results = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        memb, res = lv.run(g, substeps=args.substeps, flags=run_flags)
        results.append(res)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1000.0 / args.steps
    teps = g.nnz / (ms_per_step / 1000.0)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {teps / 1e9:.3f} GTEPS")

    if args.no_trace:
        # latency runs: no per-kernel events, so no roofline
        line = {"metric": METRIC, "value": teps, "unit": "TEPS", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "i64", "data": "synthetic",
                "config": {"workload": args.workload, "n": g.n, "nnz": g.nnz,
                           "substeps": args.substeps, "graph_replay": args.graph_replay,
                           "passes": results[0]["passes"],
                           "iterations": results[0]["iterations"], "Q": results[0]["q"]},
                "roofline": None}
        lv.close()
        print(json.dumps(line), flush=True)
        return
    tiers = tier_rooflines(results, g.offsets.dtype == torch.int64)
    dom = max(tiers, key=lambda t: t["ms_total"])
    for t in tiers:
        t["traffic"] = load_tier_traffic(args.workload, t["tier"])
    traffic = dom["traffic"]
    r0 = results[0]
    scanned = sum(t["fused_arcs"] + t["wg_arcs"] + t["hub_arcs"] for t in r0["trace"])
    move_ms = sum(t["fused_ms"] + t["wg_ms"] + t["hub_ms"] for t in r0["trace"])
    move_teps = scanned / max(move_ms / 1000.0, 1e-12)
    wide = any(t["wide"] for r in results for t in r["trace"])

    line = {
        "metric": METRIC,
        "value": teps,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i128" if wide else "i64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n": g.n,
            "nnz": g.nnz,
            "W": r0["W"],
            "offsets": str(g.offsets.dtype).replace("torch.", ""),
            "tolerance": "1e-2, declining x10 per pass",
            "substeps": args.substeps,
            "classes": "colour" if args.colour_classes else "hash",
            "passes": r0["passes"],
            "iterations": r0["iterations"],
            "n_per_pass": r0["n_pass"],
            "arcs_per_pass": r0["nnz_pass"],
            "communities": r0["n_communities"],
            "Q": r0["q"],
        },
        "roofline": {
            "kernel": dom["kernel"],
            "bound": "hbm",
            "achieved": dom["achieved_gbps"],
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": dom["achieved_gbps"] / HBM_PEAK_GBPS,
            "traffic": traffic,
            "traffic_gbps": (traffic / (dom["avg_launch_ms"] / 1000.0) / 1e9
                             if traffic and dom["avg_launch_ms"] > 0 else None),
            "avg_launch_ms": dom["avg_launch_ms"],
            "launches": dom["launches"],
            "algorithmic_bytes_per_launch": dom["bytes_per_launch"],
        },
        "roofline_tiers": tiers,
        "breakdown_ms_per_step": {t["tier"]: t["ms_total"] / args.steps for t in tiers},
        "move_teps": move_teps,
    }
    del memb
    # the random-access ceiling, measured after the timed runs on a table the size of the
    # first pass's community records (16 bytes per vertex): the move tiers' gathers per second
    # set against it (the records of later passes are smaller, so this ceiling is the lowest
    # the run meets)
    table = 16 * g.n
    ceiling = lv.probe_gather(table, 1)
    line["gather_ceiling"] = {"probe": "louvain_probe_gather: 4.2M threads x 64 random "
                                       "4-byte gathers", "table_bytes": table, "slices": 1,
                              "gathers_per_s": ceiling,
                              "gathers_per_s_xcd_sliced": lv.probe_gather(table, 8)}
    for t in tiers:
        if "gathers_per_s" in t and ceiling > 0:
            t["gather_frac"] = t["gathers_per_s"] / ceiling
    # the whole move phase: every iteration's gathers (all tiers) over its wall time
    mg = sum(t["fused_arcs"] + t["wg_arcs"] + t["hub_arcs"] + t["candidates"]
             for r in results for t in r["trace"])
    mms = sum(t["iter_ms"] for r in results for t in r["trace"])
    if mms > 0 and ceiling > 0:
        line["move_phase_gathers"] = {"gathers": mg / len(results), "ms": mms / len(results),
                                      "gathers_per_s": mg / (mms / 1000.0),
                                      "frac_of_ceiling": mg / (mms / 1000.0) / ceiling}
    if "gathers_per_s" in dom and ceiling > 0:
        line["roofline_gather"] = {"kernel": dom["kernel"], "bound": "random gathers",
                                   "achieved": dom["gathers_per_s"], "peak": ceiling,
                                   "unit": "gathers/s", "frac": dom["gather_frac"]}
    log(f"gather ceiling: {ceiling / 1e9:.1f}e9/s over {table / 2**20:.0f} MiB; dominant tier "
        f"{dom['tier']} at {dom.get('gathers_per_s', 0) / 1e9:.1f}e9/s")
    if not args.no_extra:
        # the fully synchronous rule (one class per iteration) on the same graph, one run
        lv.run(g, substeps=1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, r1 = lv.run(g, substeps=1)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t1
        line["sync_k1"] = {"ms": el1 * 1000.0, "teps": g.nnz / el1, "q": r1["q"],
                           "passes": r1["passes"], "iterations": r1["iterations"],
                           "qnum_pass": [str(x) for x in r1["qnum_pass"]],
                           "cap_hits": r1["cap_hits"]}
        log(f"fully synchronous (K = 1): {line['sync_k1']['ms']:.1f} ms, Q {r1['q']:.6f}, "
            f"iterations {r1['iterations']}")
    lv.close()
    if not args.no_cpu_baseline:
        log("cpu baseline: copying the graph to the host")
        gc = g.to("cpu")
        del g
        torch.cuda.empty_cache()
        line["cpu_baseline"] = cpu_baseline(gc, r0["trace"], args.cpu_seconds, args.substeps,
                                            gc.nnz)
        log(f"cpu baseline: {line['cpu_baseline']['value'] / 1e6:.2f} MTEPS")
        del gc
    else:
        del g
    torch.cuda.empty_cache()
    if not args.no_extra:
        # the other two parts of the metric: batched graphs/s against one graph at a time, and
        # serving latency against a one-at-a-time FIFO server, on the same GPU
        b = batched_measure(args, dev, 3, 1, False)
        line["batched"] = {k: b["config"][k] for k in
                           ("graphs", "nnz", "one_by_one_graphs_per_s", "speedup_vs_one_by_one",
                            "identical_to_one_by_one", "mean_q")}
        line["batched"]["graphs_per_s"] = b["value"]
        line["batched"]["ms_per_batch"] = b["ms_per_step"]
        torch.cuda.empty_cache()
        sv = serving_measure(args, dev, seconds=args.extra_serve_seconds,
                             servers=("continuous", "fifo"))["config"]
        keep = ("rate", "completed_per_s", "p50_ms", "p99_ms", "offered", "completed",
                "unfinished", "mean_batch")
        line["serving"] = {
            "seconds_of_arrivals": sv["serve_seconds"], "pool_graphs": sv["pool_graphs"],
            "pool_mean_arcs": sv["pool_mean_arcs"],
            "continuous": [{k: r[k] for k in keep} for r in sv["rates"]],
            "one_at_a_time_fifo": [{k: r[k] for k in keep} for r in sv["fifo_rates"]],
        }
    print(json.dumps(line), flush=True)


# Algorithmic bytes of the move tiers (what the method must move, not cache lines): per decided
# vertex its row bounds (o = 8 B for the input's int64 offsets, 16 B for the start and end
# arrays of a super-vertex graph) and C[v] 4, K[v] 8, Sigma[own] 8, csize[own] 4,
# csize[best] 4, decision 4 -> o + 32 B; per arc neighbour id 4, weight 4, C[neighbour] 4 ->
# 12 B; per distinct candidate community Sigma[c] 8 B. Aggregation of a pass's graph: per arc
# neighbour id 4, weight 4, super id of the neighbour 4 -> 12 B; per vertex C 4 and super id
# 4 -> 8 B; per super-arc written id 4 and weight 4 -> 8 B.
AGG_BYTES_PER_ARC = 12
AGG_BYTES_PER_VERTEX = 8
AGG_BYTES_PER_SUPER_ARC = 8


def tier_rooflines(results, offsets_64):
    """Per move tier (one launch = one class step's kernels of the tier) and for aggregation
    (one launch = one pass's aggregation): algorithmic bytes per launch over the HIP-event time
    of the launch on the stream it ran on, summed over the timed runs. The three move tiers of
    a class step run concurrently on three streams, so each tier's time is stretched by the
    others and the rates are lower bounds of what each tier achieves alone."""
    acc = {k: {"ms": 0.0, "launches": 0, "bytes": 0.0, "gathers": 0.0}
           for k in ("fused", "wg", "hub", "agg")}
    for r in results:
        for t in r["trace"]:
            o = 8 if (t["pass"] == 0 and offsets_64) else (4 if t["pass"] == 0 else 16)
            hub_cand = t["candidates"] - t["fused_candidates"] - t["wg_candidates"]
            for key, v, a, c, ms, nl in (
                    ("fused", t["fused_vertices"], t["fused_arcs"], t["fused_candidates"],
                     t["fused_ms"], t["fused_launches"]),
                    ("wg", t["wg_vertices"], t["wg_arcs"], t["wg_candidates"], t["wg_ms"],
                     t["wg_launches"]),
                    ("hub", t["hub_vertices"], t["hub_arcs"], hub_cand, t["hub_ms"],
                     t["hub_launches"])):
                if nl <= 0:
                    continue
                acc[key]["ms"] += ms
                acc[key]["launches"] += nl
                acc[key]["bytes"] += ((o + BYTES_PER_VERTEX_BASE) * v + BYTES_PER_ARC * a
                                      + BYTES_PER_CANDIDATE * c)
                # random gathers: a neighbour's community per arc, a candidate's Sigma
                acc[key]["gathers"] += a + c
        for p in range(r["passes"] - 1):
            if r["aggregate_ms"][p] <= 0:
                continue
            acc["agg"]["ms"] += r["aggregate_ms"][p]
            acc["agg"]["launches"] += 1
            acc["agg"]["bytes"] += (AGG_BYTES_PER_ARC * r["nnz_pass"][p]
                                    + AGG_BYTES_PER_VERTEX * r["n_pass"][p]
                                    + AGG_BYTES_PER_SUPER_ARC * r["nnz_pass"][p + 1])
    names = {"fused": "k_move_lds", "wg": "k_move_grp7+k_move_wg",
             "hub": "k_hub_part+k_hub_reduce+k_hub_decide",
             "agg": "aggregation (k_merge_part, k_merge_lds, k_merge_reduce, ...)"}
    out = []
    for key, a in acc.items():
        if a["launches"] == 0:
            continue
        avg = a["ms"] / a["launches"]
        bpl = a["bytes"] / a["launches"]
        gbps = bpl / (avg / 1000.0) / 1e9 if avg > 0 else 0.0
        t = {"tier": key, "kernel": names[key], "ms_total": a["ms"],
             "launches": a["launches"], "avg_launch_ms": avg, "bytes_per_launch": bpl,
             "achieved_gbps": gbps, "frac": gbps / HBM_PEAK_GBPS}
        if a["gathers"] > 0 and avg > 0:
            t["gathers_per_launch"] = a["gathers"] / a["launches"]
            t["gathers_per_s"] = t["gathers_per_launch"] / (avg / 1000.0)
        out.append(t)
    return out


if __name__ == "__main__":
    main()
