"""Benchmark: VT/VV/TT relation entries per second on one MI355X.

One step = every cluster of the 128^3 Kuhn lattice (2,097,152 vertices,
12,290,298 tetrahedra, 2048 Morton clusters of 1024 vertices) built into HBM
with all three relations in one batched persistent launch.  The mesh streams
are resident in HBM before timing starts; copies to the host are not part of a
step.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    1: "32^3 Kuhn lattice (32,768 vertices, 178,746 tetrahedra), seed-permuted, 64 Morton clusters of 512 "
       "vertices; VT+VV+TT for every cluster in one batched launch",
    2: "128^3 Kuhn lattice (2,097,152 vertices, 12,290,298 tetrahedra), seed-permuted, 2048 Morton clusters of "
       "1024 vertices; VT+VV+TT for every cluster in one batched launch",
    3: "256^3 Kuhn lattice refined by 3 rounds of centroid splits of 5% of the tetrahedra in 8 Gaussian blobs "
       "(34,050,862 vertices, 151,309,188 tetrahedra), lognormal Morton clusters (median 512, sigma 1, 64..8192; "
       "40,579 clusters); VT+VV+TT for every cluster in one batched launch, autotuned launch classes",
    4: "the 256^3 refined mesh with a 16-Gaussian scalar field; batched build as for the refined mesh, then the "
       "serving workload (40 consumer threads, 4 GB HBM relation cache)",
}
KERNEL_SOURCES = ["paper_2507_15230_amd/csrc/gale_kernels.hip", "paper_2507_15230_amd/csrc/gale_layout.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "persistent_kernel_traffic_128cubed.json")
COPY_BYTES = 256 << 20


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per persistent launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def summarize_profile(kt_dir, fetch_dir, write_dir, out_md, out_json, cmd_kt, cmd_fetch, cmd_write):
    """Turn rocprofv3 CSV output into the committed text summary and the
    traffic record bench.py reads back."""
    stats = glob.glob(os.path.join(kt_dir, "**", "*kernel_stats.csv"), recursive=True)
    lines = ["# rocprofv3 kernel statistics: 128^3 lattice, 2048 clusters, VT+VV+TT batched", "",
             "Command: `%s`" % cmd_kt, "", "| kernel | calls | total ms | avg us | min us | max us |",
             "|---|---|---|---|---|---|"]
    avg_persistent = None
    for fn in stats:
        for r in csv.DictReader(open(fn)):
            name = r.get("Name") or r.get("KernelName") or ""
            calls = int(float(r.get("Calls", 0)))
            tot = float(r.get("TotalDurationNs", 0)) / 1e6
            avg = float(r.get("AverageNs", 0)) / 1e3
            mn = float(r.get("MinNs", 0)) / 1e3
            mx = float(r.get("MaxNs", 0)) / 1e3
            lines.append("| %s | %d | %.3f | %.1f | %.1f | %.1f |" % (name[:90], calls, tot, avg, mn, mx))
            if "gale_persistent_kernel" in name and ", true>" in name:
                avg_persistent = avg
    traffic = {}
    for tag, d in (("fetch", fetch_dir), ("write", write_dir)):
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            per = {}
            for r in csv.DictReader(open(fn)):
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
            traffic[tag] = per
    copy_name = None
    res = {"kernel_source_sha256": kernel_source_hash(), "commands": [cmd_kt, cmd_fetch, cmd_write]}
    if "fetch" in traffic and "write" in traffic:
        def pick(per, pred):
            for k, v in per.items():
                if pred(k):
                    return k, sum(v) / len(v)
            return None, None
        copy_name, copy_fetch = pick(traffic["fetch"], lambda k: "neg" in k.lower())
        _, copy_write = pick(traffic["write"], lambda k: k == copy_name)
        kname, k_fetch = pick(traffic["fetch"], lambda k: "gale_persistent_kernel" in k and ", true>" in k)
        _, k_write = pick(traffic["write"], lambda k: k == kname)
        if copy_fetch and copy_write and k_fetch is not None and k_write is not None:
            f_fac = COPY_BYTES / (copy_fetch * 1024.0)
            w_fac = COPY_BYTES / (copy_write * 1024.0)
            tb = k_fetch * 1024.0 * f_fac + k_write * 1024.0 * w_fac
            res.update({"copy_kernel": copy_name, "copy_bytes": COPY_BYTES, "copy_fetch_kib": copy_fetch,
                        "copy_write_kib": copy_write, "fetch_factor": f_fac, "write_factor": w_fac,
                        "kernel": kname, "fetch_kib_per_dispatch": k_fetch, "write_kib_per_dispatch": k_write,
                        "traffic_bytes_per_launch": tb, "avg_kernel_us": avg_persistent})
            lines += ["", "## HBM traffic (rocprofv3 --pmc, per dispatch)", "",
                      "Commands: `%s` and `%s`" % (cmd_fetch, cmd_write), "",
                      "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|",
                      "| %s | %.0f | %.0f |" % (kname[:90], k_fetch, k_write),
                      "| %s (%d MiB copy) | %.0f | %.0f |" % (copy_name[:60], COPY_BYTES >> 20, copy_fetch, copy_write),
                      "", "Scale factors from the copy (known bytes / counter): fetch %.3f, write %.3f." % (f_fac, w_fac),
                      "Traffic per persistent launch: %.1f MB." % (tb / 1e6)]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", out_md, out_json)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def output_bytes(entries: int, nv: int, nt: int, ncl: int) -> int:
    """Bytes a step must write: entries, offsets (VT, VV per vertex row + 1 per
    cluster, TT per tetrahedron row + 1 per cluster), row ids (vertex rows once,
    tetrahedron rows) and an 8-word header per block."""
    words = entries + (2 * nv + 2 * ncl) + (nt + ncl) + nv + nt + 8 * ncl
    return 4 * words


def cpu_baseline(mesh, budget_s: float = 15.0):
    """The oracle as it stands, single-threaded, on the first clusters of the
    same mesh until about budget_s seconds of block building."""
    import oracle
    t0 = time.perf_counter()
    orc = oracle.Oracle.of(mesh)
    t_setup = time.perf_counter() - t0
    entries = 0
    nclus = 0
    t1 = time.perf_counter()
    for k in range(mesh.nclusters):
        for rel in (1, 2, 4):
            _, _, e = orc.block(k, rel)
            entries += len(e)
        nclus += 1
        if time.perf_counter() - t1 > budget_s:
            break
    dt = time.perf_counter() - t1
    return {
        "value": entries / dt, "unit": "entries/s", "cores": 1, "kind": "oracle",
        "sample": "first %d of %d clusters, VT+VV+TT blocks, %.1f s of block building; "
                  "global VT/owner setup %.2f s excluded" % (nclus, mesh.nclusters, dt, t_setup),
    }


def serving_leg(mesh, args, pass_bytes: int):
    """Consumer threads (native, in the library) classify critical points
    cluster by cluster (Morton order, Zipf(1.1) re-access), first through the
    serving loop (continuous batching, HBM cache under a budget), then through
    synchronous plain per-cluster launches with no cache; per-access latency
    (submit -> ready) percentiles."""
    import meshgen
    from paper_2507_15230_amd import gale
    if mesh.scalar is not None:
        field = mesh.scalar
    else:
        n = int(round(mesh.nv ** (1.0 / 3.0)))
        field = meshgen.gauss_field(mesh.coords.astype(np.float64), n, np.random.default_rng(1))
    if args.serving_budget_mb:
        budget = args.serving_budget_mb << 20
    elif args.config == 4:
        budget = 4 << 30
    else:
        budget = pass_bytes // 2
    ncur = args.serving_clusters if args.serving_clusters >= 0 else (mesh.nclusters if args.config <= 2 else 4096)
    order = np.arange(min(ncur, mesh.nclusters), dtype=np.int32)  # cluster ids are in Morton order
    log("serving leg: %d consumers, budget %.0f MB" % (args.consumers, budget / 1e6))
    ctx = gale.Context(device=0, mode="serve", cache_budget_bytes=budget, max_inflight=4,
                       block_threads=args.block_threads)
    ctx.load(mesh.tets, mesh.cluster, mesh.nclusters)
    res = gale.consumer_run(ctx, mesh.tets, field, order, threads=args.consumers)
    st = ctx.stats()
    ctx.close()
    out = {
        "workload": "the benchmark mesh with its 16-Gaussian scalar field; %d native consumer threads, Morton "
                    "cursor, truncated Zipf(1.1) re-access, VT+VV+TT per access, critical points from VT and VV"
                    % args.consumers,
        "consumers": args.consumers, "cache_budget_bytes": int(budget), "max_inflight": 4,
        "cursor_clusters": int(order.shape[0]),
        "accesses": res["accesses"], "reaccesses": res["reaccesses"], "wall_s": res["wall_s"],
        "accesses_per_s": res["accesses"] / res["wall_s"],
        "p50_us": res["lat_p50_us"], "p99_us": res["lat_p99_us"], "mean_us": res["lat_mean_us"],
        "max_us": res["lat_max_us"],
        "cache_hits": st["cache_hits"], "cache_misses": st["cache_misses"], "evictions": st["evictions"],
        "batches": st["batches"], "mean_batch_clusters": st["mean_batch_clusters"],
        "entries_built_per_s": st["entries_built"] / res["wall_s"],
        "entries_delivered_per_s": st["entries_delivered"] / res["wall_s"],
        "stage_us": {"queue": st["stage_queue_us"], "build": st["stage_build_us"], "copy": st["stage_copy_us"]},
        "label_mismatches": res["mismatches"], "errors": res["errors"],
        "critical_points": {"minima": res["minima"], "maxima": res["maxima"], "saddles": res["saddles"]},
    }
    log("plain serving baseline")
    pctx = gale.Context(device=0, mode="direct", form="plain", block_threads=args.block_threads)
    pctx.load(mesh.tets, mesh.cluster, mesh.nclusters)
    pres = gale.consumer_run(pctx, mesh.tets, field, order, threads=args.consumers)
    pctx.close()
    out["plain"] = {"accesses": pres["accesses"], "wall_s": pres["wall_s"],
                    "accesses_per_s": pres["accesses"] / pres["wall_s"],
                    "p50_us": pres["lat_p50_us"], "p99_us": pres["lat_p99_us"], "mean_us": pres["lat_mean_us"],
                    "label_mismatches": pres["mismatches"], "errors": pres["errors"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--block-threads", type=int, default=1024)
    ap.add_argument("--lds-bytes", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="one gale_build per step instead of a graph replay")
    ap.add_argument("--autotune", type=int, default=-1,
                    help="pick the launch classes by timing (default: on for the refined configs 3-5)")
    ap.add_argument("--consumers", type=int, default=40)
    ap.add_argument("--serving-clusters", type=int, default=-1,
                    help="clusters the consumers' cursor walks (default: all on the lattices, 4096 on refined meshes)")
    ap.add_argument("--serving-budget-mb", type=int, default=0,
                    help="HBM cache budget of the serving leg; 0 = half of one full pass's block bytes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one %d MiB device copy (reference for the HBM byte counters)" % (COPY_BYTES >> 20))
    ap.add_argument("--summarize-profile", nargs=8, metavar=("KT", "FETCH", "WRITE", "MD", "JSON", "CMD_KT",
                                                           "CMD_FETCH", "CMD_WRITE"))
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(*args.summarize_profile)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (clusters are independent, so "
              "Morton ranges of cluster ids would go to separate GPUs with no per-request collective). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import meshgen
    from paper_2507_15230_amd import gale

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    log("generating config", args.config)
    mesh = meshgen.config(args.config)
    nv, nt, ncl = mesh.nv, mesh.nt, mesh.nclusters
    ids = np.arange(ncl, dtype=np.int32)

    if args.copy_calibration:
        # a plain read+write kernel of known size: dst = -src over COPY_BYTES
        src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    ctx = gale.Context(device=0, mode="direct", form="batched", block_threads=args.block_threads,
                       lds_bytes=args.lds_bytes, stream=stream.cuda_stream)
    log("loading")
    ctx.load(mesh.tets, mesh.cluster, ncl)
    st0 = ctx.stats()
    mesh_bytes = st0["device_mesh_bytes"]
    tuned = None
    if args.autotune == 1 or (args.autotune < 0 and args.config >= 3):
        log("autotune")
        chosen, cand = ctx.autotune(ids, 7, reps=2)
        tuned = {"launch_classes": chosen, "candidates_ms": {str(k): v for k, v in cand.items()},
                 "global_cu_share": ctx.stats()["global_cu_share"]}
    use_graph = not args.no_graph
    graph = ctx.graph_create(ids, 7) if use_graph else None

    def step():
        return ctx.graph_launch(graph) if use_graph else ctx.build(ids, 7, "batched")

    # warmup (a graph's steps share its buffer: release each before the next)
    log("warmup")
    for _ in range(max(1, args.warmup)):
        t = step()
        ctx.poll(t)
        ctx.release(t)
    e_before = ctx.stats()["entries_built"]

    # timed region: K steps back to back on the context stream.  The library
    # records HIP events around each step's launches on that stream; their
    # mean is the kernel time the roofline uses.
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tks = []
    for i in range(args.steps):
        tks.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for t in tks:
        ctx.poll(t)
    st_t = ctx.stats()
    entries_step = (st_t["entries_built"] - e_before) // args.steps
    for t in tks:
        ctx.release(t)
    if graph is not None:
        ctx.graph_destroy(graph)
    ms_kernel = st_t["kernel_ms_total"] / max(1, st_t["timed_launches"])
    ms_step = wall * 1000.0 / args.steps
    value = entries_step / (ms_step / 1000.0)
    alg_bytes = mesh_bytes + output_bytes(entries_step, nv, nt, ncl)
    achieved = alg_bytes / (ms_kernel / 1000.0) / 1e9

    plain = None
    if not args.no_plain:
        log("plain per-cluster launches")
        pctx = gale.Context(device=0, mode="direct", form="plain", block_threads=args.block_threads,
                            lds_bytes=args.lds_bytes, stream=stream.cuda_stream)
        pctx.load(mesh.tets, mesh.cluster, ncl)
        for t in [pctx.build(ids, 7, "plain")]:
            pctx.poll(t)
            pctx.release(t)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        t = pctx.build(ids, 7, "plain")
        pctx.poll(t)
        pdt = time.perf_counter() - p0
        pctx.release(t)
        pctx.close()
        plain = {"value": entries_step / pdt, "unit": "entries/s", "launches": 3 * ncl,
                 "ms_per_pass": pdt * 1000.0}

    serving = None
    if not args.no_serving:
        serving = serving_leg(mesh, args, output_bytes(entries_step, nv, nt, ncl))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(mesh)

    st = ctx.stats()
    ctx.close()
    out = {
        "metric": "VT/VV/TT relation entries/s",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS.get(args.config, "config %d" % args.config),
            "config_index": args.config,
            "seed": 0,
            "entries_per_step": int(entries_step),
            "clusters": ncl,
            "form": "batched, one hipGraph replay per step" if use_graph else "batched, one build call per step",
            "block_threads": args.block_threads,
            "autotune": tuned,
            "load_seconds": st0["load_seconds"],
            "global_path_blocks_per_step": int(st["global_path_blocks"] // max(1, st["requests"])),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "alg_bytes_per_launch": int(alg_bytes), "kernel_ms": ms_kernel,
        },
        "cpu_baseline": cpu,
        "plain": plain,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
