"""Benchmark: VT/VV/TT relation entries per second on one MI355X.

One step = every cluster of the workload's mesh built into HBM with all
three relations, as one hipGraph replay of the batched persistent launches
(the launch shapes read from the tune table the project's autotuner wrote, or
tuned on the spot).  The default workload is the 256^3 lattice refined in
Gaussian blobs (34,050,862 vertices, 151,309,188 tetrahedra, 40,579 lognormal
Morton clusters).  The mesh streams are resident in HBM before timing starts;
copies to the host are not part of a step.  Around the timed steps the run
also measures: the same build as one launch per (cluster, relation) ("plain"),
the serving loop with 40 consumer threads under an HBM cache budget against
synchronous plain per-cluster requests, and the CPU oracle on a bounded sample
(one thread, then every allowed host thread).  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C]
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TUNE_TABLE = os.path.join(ROOT, "paper_2507_15230_amd", "tune_mi355x.json")
WORKLOADS = {
    1: "32^3 Kuhn lattice (32,768 vertices, 178,746 tetrahedra), seed-permuted, 64 Morton clusters of 512 "
       "vertices; VT+VV+TT for every cluster in one batched launch",
    2: "128^3 Kuhn lattice (2,097,152 vertices, 12,290,298 tetrahedra), seed-permuted, 2048 Morton clusters of "
       "1024 vertices; VT+VV+TT for every cluster in one batched launch",
    3: "256^3 Kuhn lattice refined by 3 rounds of centroid splits of 5% of the tetrahedra in 8 Gaussian blobs "
       "(34,050,862 vertices, 151,309,188 tetrahedra), lognormal Morton clusters (median 512, sigma 1, 64..8192; "
       "40,579 clusters); VT+VV+TT for every cluster in one hipGraph-captured batched submit, tuned launch shapes",
    4: "the 256^3 refined mesh with a 16-Gaussian scalar field (config 3's mesh, own permutation); batched "
       "build as for config 3, then the serving workload (40 consumer threads, 4 GB HBM relation cache)",
    5: "384^3 Kuhn lattice refined by 2 rounds of centroid splits of 3% of the tetrahedra in 8 Gaussian blobs "
       "(77,758,730 vertices, 400,498,200 tetrahedra), lognormal Morton clusters (median 1024, sigma 1.2, "
       "64..8192; 42,669 clusters); VT+VV+TT for every cluster in one hipGraph-captured batched submit, then "
       "serving with 40 consumers under 8 / 32 / 128 GB cache budgets",
}
COPY_BYTES = 256 << 20
# the sources of the kernels a step runs: a committed traffic summary counts
# only while these are unchanged
KERNEL_SOURCES = ("gale_kernels.hip", "gale_stitch.hip", "gale_devutil.h", "gale_layout.h")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_15230_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(config_index: int):
    """HBM bytes of one step (FETCH_SIZE + WRITE_SIZE, calibrated by a plain
    copy) from the committed rocprofv3 summary of this workload, if it was
    taken on the current kernel sources; else None."""
    sha = kernel_source_sha()
    for fn in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))):
        try:
            d = json.load(open(fn))
        except (OSError, ValueError):
            continue
        if d.get("config_index") == config_index and d.get("kernel_source_sha256") == sha:
            return d.get("traffic_bytes_per_step"), os.path.relpath(fn, ROOT)
    return None, None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info() -> dict:
    """CPU model, logical CPUs, the CPUs this process may use, and RAM."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = 0
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "allowed_cpus": len(os.sched_getaffinity(0)),
            "ram_bytes": ram}


def alg_bytes(ctx, ncl: int, entries: int) -> tuple[int, dict]:
    """Algorithmic bytes of one step: every cluster's star and halo
    tetrahedra read once as four int32 vertex ids and an int32 tetrahedron id
    (20 B each), every entry written (4 B), the offsets (VT and VV per vertex
    row + 1, TT per tetrahedron row + 1) and the row ids (vertex rows once,
    tetrahedron rows)."""
    ns = nh = nv = nt = 0
    for k in range(ncl):
        i = ctx.cluster_info(k)
        ns += i["ns"]
        nh += i["nh"]
        nv += i["nV"]
        nt += i["nT"]
    b = 20 * (ns + nh) + 4 * entries + 4 * (2 * nv + nt + 3 * ncl) + 4 * (nv + nt)
    return b, {"star_tets": ns, "halo_tets": nh, "vertex_rows": nv, "tet_rows": nt}


def stream_bytes(mesh_bytes: int, entries: int, nv: int, nt: int, ncl: int) -> int:
    """Bytes as this library stores them: the compressed per-cluster streams
    (4 x uint16 local ids per tetrahedron where a cluster's table allows, the
    tetrahedron ids, the local vertex tables) read once, plus every output word
    (entries, offsets, row ids, an 8-word header per block)."""
    words = entries + (2 * nv + 2 * ncl) + (nt + ncl) + nv + nt + 8 * ncl
    return mesh_bytes + 4 * words


def cpu_baseline(mesh, budget_s: float = 12.0, seed: int = 0):
    """The oracle as it stands on a seeded random sample of the same mesh's
    clusters: first on one thread until about budget_s seconds of block
    building, then the same clusters on every allowed host thread (at most 16,
    the box's share), cluster-parallel."""
    import oracle
    t0 = time.perf_counter()
    orc = oracle.Oracle.of(mesh)
    t_setup = time.perf_counter() - t0
    order = np.random.default_rng(seed).permutation(mesh.nclusters)
    entries = 0
    done = []
    t1 = time.perf_counter()
    for k in order:
        for rel in (1, 2, 4):
            _, _, e = orc.block(int(k), rel)
            entries += len(e)
        done.append(int(k))
        if time.perf_counter() - t1 > budget_s:
            break
    dt1 = time.perf_counter() - t1
    threads = min(16, len(os.sched_getaffinity(0)))
    pairs = [(k, rel) for k in done for rel in (1, 2, 4)]
    t2 = time.perf_counter()
    res = orc.blocks(pairs, threads=threads)
    dtn = time.perf_counter() - t2
    assert sum(len(r[2]) for r in res) == entries
    sample = ("seeded random sample of %d of %d clusters (VT+VV+TT blocks, %d entries); global VT and owner setup "
              "%.1f s excluded" % (len(done), mesh.nclusters, entries, t_setup))
    return {
        "value": entries / dtn, "unit": "entries/s", "cores": threads, "kind": "oracle",
        "sample": sample + "; %d threads cluster-parallel, %.2f s" % (threads, dtn),
        "one_thread": {"value": entries / dt1, "unit": "entries/s", "cores": 1, "seconds": dt1},
        "host": host_info(),
    }


def serving_leg(mesh, budget: int, consumers: int, ncur: int, front_end: str = "single", plain: bool = True,
                prefetch: int = 0):
    """Consumer threads (native, in the library) classify critical points
    cluster by cluster (Morton order, Zipf(1.1) re-access) through the serving
    loop (continuous batching, HBM cache under `budget`); then, when `plain`,
    the same consumers with synchronous plain per-cluster launches and no
    cache.  Per-access latency (submit -> ready) percentiles and the paper's
    waiting-time stages."""
    import meshgen
    from paper_2507_15230_amd import gale
    if mesh.scalar is not None:
        field = mesh.scalar
    else:
        n = int(round(mesh.meta.get("n", round(mesh.nv ** (1.0 / 3.0)))))
        field = meshgen.gauss_field(mesh.coords.astype(np.float64), n, np.random.default_rng(1))
    order = np.arange(min(ncur, mesh.nclusters), dtype=np.int32)  # cluster ids are in Morton order
    log("serving: %d consumers, budget %.1f GB, front end %s, prefetch %d, %d clusters"
        % (consumers, budget / 1e9, front_end, prefetch, order.shape[0]))
    ctx = gale.Context(device=0, mode="serve", cache_budget_bytes=budget, max_inflight=4, front_end=front_end,
                       prefetch_depth=prefetch)
    ctx.load(mesh.tets, mesh.cluster, mesh.nclusters)
    res = gale.consumer_run(ctx, mesh.tets, field, order, threads=consumers)
    st = ctx.stats()
    ctx.close()
    w = res["wall_s"]
    out = {
        "consumers": consumers, "cache_budget_bytes": int(budget), "front_end": front_end,
        "prefetch_depth": prefetch, "max_inflight": 4, "cursor_clusters": int(order.shape[0]),
        "accesses": res["accesses"], "reaccesses": res["reaccesses"], "wall_s": w,
        "accesses_per_s": res["accesses"] / w,
        "p50_us": res["lat_p50_us"], "p99_us": res["lat_p99_us"], "mean_us": res["lat_mean_us"],
        "max_us": res["lat_max_us"],
        "cache_hits": st["cache_hits"], "cache_misses": st["cache_misses"], "evictions": st["evictions"],
        "prefetch": {k: st[k] for k in ("prefetch_built", "prefetch_hits", "prefetch_evicted", "demand_evictions")},
        "batches": st["batches"], "mean_batch_clusters": st["mean_batch_clusters"],
        "queue_depth_mean": st["queue_depth_mean"], "queue_depth_max": st["queue_depth_max"],
        "entries_built_per_s": st["entries_built"] / w, "entries_delivered_per_s": st["entries_delivered"] / w,
        "stages_mean_us": {"push": st["stage_push_us"], "in_queue": st["stage_queue_us"] - st["stage_push_us"],
                           "preparation": st["stage_prep_us"], "kernel_and_copy": st["stage_kernel_copy_us"],
                           "integration": st["stage_integration_us"]},
        "stages_max_thread_s": {"push": st["wait_push_s_max"], "in_queue": st["wait_queue_s_max"],
                                "preparation": st["wait_prep_s_max"], "kernel_and_copy": st["wait_kernel_copy_s_max"],
                                "integration": st["wait_integration_s_max"]},
        "label_mismatches": res["mismatches"], "errors": res["errors"],
        "critical_points": {"minima": res["minima"], "maxima": res["maxima"], "saddles": res["saddles"]},
    }
    if plain:
        log("serving: plain per-cluster baseline")
        pctx = gale.Context(device=0, mode="direct", form="plain")
        pctx.load(mesh.tets, mesh.cluster, mesh.nclusters)
        pres = gale.consumer_run(pctx, mesh.tets, field, order, threads=consumers)
        pctx.close()
        out["plain"] = {"accesses": pres["accesses"], "wall_s": pres["wall_s"],
                        "accesses_per_s": pres["accesses"] / pres["wall_s"],
                        "p50_us": pres["lat_p50_us"], "p99_us": pres["lat_p99_us"], "mean_us": pres["lat_mean_us"],
                        "label_mismatches": pres["mismatches"], "errors": pres["errors"]}
    return out


def simplices_leg(mesh, steps: int = 5) -> dict:
    """The edge and triangle relations (VE, VF, EF, ET, FT) of every cluster
    of `mesh`, built in the batched form into device memory: the lists' load
    time (enumeration on the host and upload) and relation entries per second
    over `steps` builds after one warm-up build."""
    from paper_2507_15230_amd import gale
    ctx = gale.Context(device=0, mode="direct", form="batched", simplex_lists=True)
    ctx.load(mesh.tets, mesh.cluster, mesh.nclusters)
    load_s = ctx.stats()["load_seconds"]
    e, _, f, _ = ctx.simplices()
    ids = np.arange(mesh.nclusters, dtype=np.int32)
    t = ctx.build(ids, gale.REL_EXT)
    ctx.poll(t)
    ctx.release(t)
    e0 = ctx.stats()["entries_built"]
    t0 = time.perf_counter()
    for _ in range(steps):
        t = ctx.build(ids, gale.REL_EXT)
        ctx.poll(t)
        ctx.release(t)
    dt = (time.perf_counter() - t0) / steps
    ent = (ctx.stats()["entries_built"] - e0) // steps
    ctx.close()
    return {"relations": "VE+VF+EF+ET+FT", "edges": int(e.shape[0]), "triangles": int(f.shape[0]),
            "load_seconds_with_lists": load_s, "entries_per_build": int(ent), "ms_per_build": dt * 1000.0,
            "entries_per_s": ent / dt,
            "note": "one gale_build per step (host staging and the header read-back included), device-resident output"}


def summarize_profile(out_md, title, cmd_kt, kt_dir, cmd_fetch=None, fetch_dir=None, cmd_write=None,
                      write_dir=None, kernel_ms=None, config_index=None, alg_bytes=None):
    """Turn rocprofv3 CSV output into a committed text summary: per-kernel
    statistics, the span of each step's persistent launches (first start to
    last end, from the kernel trace), and HBM traffic per step from
    FETCH_SIZE / WRITE_SIZE scaled by a plain copy of known size.  With
    config_index, the traffic also goes to <out_md>_traffic.json with the hash
    of the kernel sources, which the benchmark reads back."""
    lines = ["# " + title, "", "Command: `%s`" % cmd_kt, "", "| kernel | calls | total ms | avg us | min us | max us |",
             "|---|---|---|---|---|---|"]
    for fn in glob.glob(os.path.join(kt_dir, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            name = r.get("Name") or r.get("KernelName") or ""
            lines.append("| %s | %d | %.3f | %.1f | %.1f | %.1f |" % (
                name[:90], int(float(r.get("Calls", 0))), float(r.get("TotalDurationNs", 0)) / 1e6,
                float(r.get("AverageNs", 0)) / 1e3, float(r.get("MinNs", 0)) / 1e3, float(r.get("MaxNs", 0)) / 1e3))
    # steps: runs of persistent launches separated by the zero kernel that starts each graph replay
    spans = []
    for fn in glob.glob(os.path.join(kt_dir, "**", "*kernel_trace.csv"), recursive=True):
        rows = sorted(csv.DictReader(open(fn)), key=lambda r: int(r["Start_Timestamp"]))
        cur = None
        for r in rows:
            name = r["Kernel_Name"]
            if "gale_zero_kernel" in name:
                if cur:
                    spans.append(cur)
                cur = [None, None, 0]
            elif ("gale_persistent_kernel" in name or "gale_stitch_kernel" in name) and cur is not None:
                s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                cur[0] = s if cur[0] is None else min(cur[0], s)
                cur[1] = e if cur[1] is None else max(cur[1], e)
                cur[2] += 1
        if cur and cur[0] is not None:
            spans.append(cur)
    spans = [s for s in spans if s[0] is not None]
    if spans:
        d = [(s[1] - s[0]) / 1e6 for s in spans]
        lines += ["", "Steps (graph replays): %d; launches per step (persistent and stitch): %s; span of a step's "
                  "launches (first start to last end) mean %.3f ms, min %.3f, max %.3f." % (
                      len(spans), sorted(set(s[2] for s in spans)), sum(d) / len(d), min(d), max(d))]
        if kernel_ms:
            lines.append("HIP events around the same launches in the benchmark's own run: %.3f ms." % kernel_ms)
    if fetch_dir and write_dir:
        per = {}
        for tag, dd in (("fetch", fetch_dir), ("write", write_dir)):
            vals = {}
            for fn in glob.glob(os.path.join(dd, "**", "*counter_collection.csv"), recursive=True):
                for r in csv.DictReader(open(fn)):
                    vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
            per[tag] = vals
        copy = [k for k in per["fetch"] if "neg" in k.lower()]
        if copy and copy[0] in per["write"]:
            cf = sum(per["fetch"][copy[0]]) / len(per["fetch"][copy[0]])
            cw = sum(per["write"][copy[0]]) / len(per["write"][copy[0]])
            ff, wf = COPY_BYTES / (cf * 1024.0), COPY_BYTES / (cw * 1024.0)
            lines += ["", "## HBM traffic (rocprofv3 --pmc, KiB per dispatch)", "",
                      "Commands: `%s` and `%s`" % (cmd_fetch, cmd_write), "",
                      "| kernel | dispatches | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) |", "|---|---|---|---|"]
            tot = 0.0
            for k in sorted(per["fetch"]):
                if not ("gale_persistent_kernel" in k or "gale_stitch_kernel" in k) or k not in per["write"]:
                    continue
                f, w = per["fetch"][k], per["write"][k]
                lines.append("| %s | %d | %.0f | %.0f |" % (k[:90], len(f), sum(f) / len(f), sum(w) / len(w)))
                tot += sum(f) / len(f) * 1024 * ff + sum(w) / len(w) * 1024 * wf
            lines += ["| copy of %d MiB (%s) | | %.0f | %.0f |" % (COPY_BYTES >> 20, copy[0][:40], cf, cw), "",
                      "Scale factors (known bytes / counter): fetch %.3f, write %.3f." % (ff, wf),
                      "HBM traffic of one step (one dispatch of each persistent kernel and of the stitch): %.1f MB."
                      % (tot / 1e6)]
            if alg_bytes:
                lines.append("Algorithmic bytes of one step: %.1f MB (traffic / algorithmic = %.3f)." % (
                    alg_bytes / 1e6, tot / alg_bytes))
            if config_index is not None:
                tj = os.path.splitext(out_md)[0] + "_traffic.json"
                with open(tj, "w") as f:
                    json.dump({"config_index": int(config_index), "kernel_source_sha256": kernel_source_sha(),
                               "traffic_bytes_per_step": tot, "alg_bytes_per_step": alg_bytes,
                               "fetch_factor": ff, "write_factor": wf,
                               "commands": [cmd_fetch, cmd_write]}, f, indent=1)
                lines.append("Traffic record for the benchmark: `%s`." % os.path.relpath(tj, ROOT))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md)


def summarize_sq(out_md, title, cmd, sq_dir, kt_dir, clock_ghz=2.4, simds=1024):
    """Committed text summary of a rocprofv3 SQ counter run: per kernel the
    mean of each counter over its dispatches, and, with the kernel's mean
    duration from the kernel trace in kt_dir, how busy the vector and scalar
    issue were (a wave64 VALU instruction takes 4 cycles of a SIMD)."""
    vals = {}
    for fn in glob.glob(os.path.join(sq_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            k = r["Kernel_Name"]
            if "gale" not in k:
                continue
            vals.setdefault(k, {}).setdefault(r["Counter_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
            vals[k][r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    dur = {}
    for fn in glob.glob(os.path.join(kt_dir, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            dur[r["Name"]] = float(r["AverageNs"]) * 1e-9
    lines = ["# " + title, "", "Command: `%s`" % cmd, "",
             "Mean per dispatch; durations from the kernel trace of the same workload.", ""]
    for k in sorted(vals):
        c = {n: sum(d.values()) / len(d) for n, d in vals[k].items()}
        lines += ["## " + k[:90], "", "| counter | value |", "|---|---|"]
        lines += ["| %s | %.4g |" % (n, c[n]) for n in sorted(c)]
        t = dur.get(k)
        if t and c.get("SQ_INSTS_VALU"):
            cyc = t * clock_ghz * 1e9
            lines += ["", "Derived (mean duration %.3f ms, %d SIMDs at %.1f GHz):" % (t * 1e3, simds, clock_ghz), "",
                      "* VALU issue: %.0f %% of the SIMDs' cycles (4 cycles per wave64 instruction)."
                      % (100.0 * c["SQ_INSTS_VALU"] * 4 / (simds * cyc)),
                      "* SALU issue: %.0f %% of one scalar instruction per SIMD per cycle."
                      % (100.0 * c.get("SQ_INSTS_SALU", 0.0) / (simds * cyc)),
                      "* LDS: %.3g instructions, %.2f bank-conflict cycles per LDS instruction."
                      % (c.get("SQ_INSTS_LDS", 0.0), c.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(1.0, c.get("SQ_INSTS_LDS", 0.0))),
                      "* VALU / LDS / SALU instructions per wave: %.0f / %.0f / %.0f." % (
                          c["SQ_INSTS_VALU"] / max(1.0, c.get("SQ_WAVES", 1.0)),
                          c.get("SQ_INSTS_LDS", 0.0) / max(1.0, c.get("SQ_WAVES", 1.0)),
                          c.get("SQ_INSTS_SALU", 0.0) / max(1.0, c.get("SQ_WAVES", 1.0)))]
        lines.append("")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--block-threads", type=int, default=1024)
    ap.add_argument("--tile-entries", type=int, default=0,
                    help="VT entries per tile of clusters too large for LDS (0 = the library default, < 0 = no tiles)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-simplices", action="store_true",
                    help="skip the VE/VF/EF/ET/FT leg (on the 128^3 lattice, or the workload mesh for configs 1-2)")
    ap.add_argument("--tune-table", default=TUNE_TABLE, help="tune table read at load and written by autotune")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even if the table has an entry")
    ap.add_argument("--consumers", type=int, default=40)
    ap.add_argument("--serving-clusters", type=int, default=-1,
                    help="clusters the consumers' cursor walks (default: all on the lattices, 24,000 on the "
                         "refined meshes, enough to overflow a 4 GB cache)")
    ap.add_argument("--budgets-gb", default="",
                    help="comma-separated HBM cache budgets of the serving leg (default: 4 on configs 3-4, "
                         "8,32,128 on config 5, half a pass's block bytes on the lattices)")
    ap.add_argument("--front-ends", default="single,per_relation",
                    help="serving front ends to run (the first one also runs the plain baseline)")
    ap.add_argument("--prefetch", type=int, default=0, help="prefetch_depth of the serving leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one %d MiB device copy (reference for the HBM byte counters)" % (COPY_BYTES >> 20))
    ap.add_argument("--summarize-sq", nargs=5, metavar=("OUT_MD", "TITLE", "CMD", "SQ_DIR", "KT_DIR"),
                    help="summary of a rocprofv3 SQ counter run")
    ap.add_argument("--summarize-profile", nargs="+", metavar="ARG",
                    help="OUT_MD TITLE CMD_KT KT_DIR [CMD_FETCH FETCH_DIR CMD_WRITE WRITE_DIR [KERNEL_MS "
                         "[CONFIG ALG_BYTES]]]")
    args = ap.parse_args()
    if args.summarize_sq:
        summarize_sq(*args.summarize_sq)
        return
    if args.summarize_profile:
        a = args.summarize_profile
        kms = float(a[8]) if len(a) > 8 else None
        cfg_i = int(a[9]) if len(a) > 10 else None
        alg = float(a[10]) if len(a) > 10 else None
        summarize_profile(a[0], a[1], a[2], a[3], *(a[4:8] if len(a) >= 8 else []), kernel_ms=kms,
                          config_index=cfg_i, alg_bytes=alg)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU.  Clusters are independent, so several GPUs would each take a "
              "contiguous Morton range of cluster ids balanced by star + halo size, load only that range's "
              "streams, and serve requests routed by owner with no per-request collective; this build has no "
              "such path.  Run with --gpus 1.", file=sys.stderr)
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
    tg = time.perf_counter()
    mesh = meshgen.config(args.config)
    gen_s = time.perf_counter() - tg
    nv, nt, ncl = mesh.nv, mesh.nt, mesh.nclusters
    ids = np.arange(ncl, dtype=np.int32)
    log("generated in %.1f s: %d vertices, %d tetrahedra, %d clusters" % (gen_s, nv, nt, ncl))

    if args.copy_calibration:
        # a plain read+write kernel of known size: dst = -src over COPY_BYTES
        src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    ctx = gale.Context(device=0, mode="direct", form="batched", block_threads=args.block_threads,
                       stream=stream.cuda_stream, tune_table_path=args.tune_table, tile_entries=args.tile_entries)
    log("loading")
    ctx.load(mesh.tets, mesh.cluster, ncl)
    st0 = ctx.stats()
    log("loaded in %.1f s" % st0["load_seconds"])
    tuned = None
    if args.config >= 3 and (args.retune or not st0["tune_applied"]):
        log("autotune")
        chosen, cand = ctx.autotune(ids, 7, reps=2)
        tuned = {"source": "gale_autotune in this run", "launch_classes": chosen,
                 "candidates_ms": {str(k): v for k, v in cand.items()}}
    elif st0["tune_applied"]:
        tuned = {"source": "tune table"}
    if tuned is not None:
        tuned.update({"table": os.path.relpath(args.tune_table, ROOT),
                      "global_cu_share": ctx.stats()["global_cu_share"]})
        try:
            for e in json.load(open(args.tune_table))["entries"]:
                if e["nv"] == nv and e["nt"] == nt and e["nclusters"] == ncl and e["rel_mask"] == 7:
                    tuned["entry"] = e
        except (OSError, ValueError, KeyError):
            pass
    graph = ctx.graph_create(ids, 7)

    log("warmup")
    for _ in range(max(1, args.warmup)):
        t = ctx.graph_launch(graph)
        ctx.poll(t)
        ctx.release(t)
    e_before = ctx.stats()["entries_built"]

    # timed region: K graph replays back to back on the context stream.  The
    # library records HIP events around each step's launches on that stream;
    # their mean is the kernel time the roofline uses.
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tks = [ctx.graph_launch(graph) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for t in tks:
        ctx.poll(t)
    st_t = ctx.stats()
    entries_step = (st_t["entries_built"] - e_before) // args.steps
    for t in tks:
        ctx.release(t)
    ctx.graph_destroy(graph)
    ms_kernel = st_t["kernel_ms_total"] / max(1, st_t["timed_launches"])
    ms_step = wall * 1000.0 / args.steps
    value = entries_step / (ms_step / 1000.0)
    b_alg, parts = alg_bytes(ctx, ncl, entries_step)
    b_stream = stream_bytes(st0["device_mesh_bytes"], entries_step, nv, nt, ncl)
    achieved = b_alg / (ms_kernel / 1000.0) / 1e9
    log("step %.3f ms, kernels %.3f ms, %.2f G entries/s, %.1f%% of HBM peak"
        % (ms_step, ms_kernel, value / 1e9, 100 * achieved / HBM_PEAK_GBS))
    st = ctx.stats()

    plain = None
    if not args.no_plain:
        log("plain per-cluster launches")
        pctx = gale.Context(device=0, mode="direct", form="plain", block_threads=args.block_threads,
                            stream=stream.cuda_stream)
        pctx.load(mesh.tets, mesh.cluster, ncl)
        t = pctx.build(ids[: min(64, ncl)], 7, "plain")
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
                 "ms_per_pass": pdt * 1000.0, "batched_over_plain": value / (entries_step / pdt)}

    serving = None
    if not args.no_serving:
        if args.budgets_gb:
            budgets = [int(float(x) * (1 << 30)) for x in args.budgets_gb.split(",")]
        elif args.config == 5:
            budgets = [8 << 30, 32 << 30, 128 << 30]
        elif args.config >= 3:
            budgets = [4 << 30]
        else:
            budgets = [stream_bytes(0, entries_step, nv, nt, ncl) // 2]
        ncur = args.serving_clusters if args.serving_clusters >= 0 else (ncl if args.config <= 2 else 24000)
        fronts = [f for f in args.front_ends.split(",") if f]
        serving = {"workload": "the benchmark mesh with a 16-Gaussian scalar field; %d native consumer threads, "
                               "Morton cursor, truncated Zipf(1.1) re-access, VT+VV+TT per access, critical points "
                               "from VT and VV" % args.consumers, "runs": []}
        for bi, b in enumerate(budgets):
            for fi, fe in enumerate(fronts):
                serving["runs"].append(serving_leg(mesh, b, args.consumers, ncur, fe, plain=(bi == 0 and fi == 0),
                                                   prefetch=args.prefetch))

    simp = None
    if not args.no_simplices:
        log("edge / triangle relations")
        smesh = mesh if args.config <= 2 else meshgen.config(2)
        simp = simplices_leg(smesh)
        simp["workload"] = WORKLOADS[args.config if args.config <= 2 else 2].split(";")[0]
        del smesh

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(mesh)

    ctx.close()
    traffic, traffic_src = committed_traffic(args.config)
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
            "form": "batched, one hipGraph replay per step",
            "block_threads": args.block_threads,
            "autotune": tuned,
            "generate_seconds": gen_s,
            "load_seconds": st0["load_seconds"],
            "global_path_blocks_per_step": int(st["global_path_blocks"] // max(1, st["requests"])),
            "hybrid_path_blocks_per_step": int(st["hybrid_path_blocks"] // max(1, st["requests"])),
            "tile_entries": args.tile_entries,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
            "alg_bytes_per_step": int(b_alg), "alg_bytes_parts": parts, "kernel_ms": ms_kernel,
            "stream_bytes_per_step": int(b_stream),
            "stream_frac": b_stream / (ms_kernel / 1000.0) / 1e9 / HBM_PEAK_GBS,
        },
        "cpu_baseline": cpu,
        "plain": plain,
        "serving": serving,
        "simplices": simp,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
