#!/usr/bin/env python3
"""Benchmark of the minhash classifier hot path on one MI355X.

One step is one pass of the whole hot path over one batch: build the database
of the at-scale reference set (1,000 synthetic genomes, about 4 Gbp, already
resident in HBM: encode, canonical k-mers, h1, bottom-s sketches, inserts, cap)
and classify its read set (10M x 150 bp, 1% substitutions, 5% foreign reads:
sketch, lookup, sort, window counts, sliding window, top hits, LCA labels).

Printed JSON line: ``value`` is classified reads/s of the classification phase;
``build_gbp_per_s`` the build rate; both with inputs resident in HBM. The
``roofline`` object covers the kernel with the larger share of the step, timed
with HIP events on its launch stream; ``cpu_baseline`` times the CPU oracle on
a read sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DB build Gbp/s; reads/s classified; p50/p99 batch latency vs plain launch"
HBM_PEAK_GBS = 8000.0
K, WINDOW, SKETCH, CAP = 16, 128, 16, 254


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--total-bp", type=float, default=4.0e9)
    ap.add_argument("--reads", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=20_000,
                    help="reads classified by the CPU oracle (0 = skip the CPU baseline)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0 = min(16, host cores)")
    return ap.parse_args()


def cpu_baseline(g, reads, n_sample, threads, gpu_labels):
    """Oracle timing on a read sample: the oracle indexes only the features the
    sample looks up (exact for the sample), then classifies it."""
    import oracle
    t0 = time.perf_counter()
    feats = np.unique(oracle.query_features(reads.text, reads.offsets, K, WINDOW, SKETCH, 0,
                                            n_sample, False))
    odb = oracle.OracleDB(K, WINDOW, SKETCH, CAP)
    odb.set_filter(feats)
    t1 = time.perf_counter()
    odb.add_targets(g.text, g.lengths, g.taxa, threads=threads)
    odb.set_taxonomy(g.parents)
    t2 = time.perf_counter()
    labels, _ = odb.classify(reads.text, reads.offsets, first=0, count=n_sample,
                             threads=threads)
    t3 = time.perf_counter()
    mism = int((labels != gpu_labels[:n_sample]).sum())
    log(f"oracle: sketch scan {t2 - t1:.1f}s ({threads} threads), classify {n_sample} reads "
        f"{t3 - t2:.2f}s, label mismatches vs GPU: {mism}")
    return {
        "value": n_sample / (t3 - t2), "unit": "reads/s", "cores": threads, "kind": "oracle",
        "sample": (f"first {n_sample} reads of the read set, classified against the oracle "
                   "index restricted to the features those reads look up (built by sketching "
                   "every window of all genomes)"),
        "build_sketch_bp_per_s": float(g.lengths.sum()) / (t2 - t1),
        "build_sketch_cores": threads,
        "sample_label_mismatches_vs_gpu": mism,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the classifier here runs on a single MI355X "
              "and has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2106_08150_amd as mc
    from paper_2106_08150_amd import synth

    mc.lib()   # fails loudly without the HIP library
    t0 = time.perf_counter()
    g = synth.scale_genomes(total_bp=args.total_bp, progress=log)
    reads = synth.scale_reads(g, n=args.reads, progress=log)
    total_bp = int(g.lengths.sum())
    n = reads.n_records
    log(f"generated {g.lengths.size} genomes / {total_bp / 1e9:.3f} Gbp and {n} reads "
        f"in {time.perf_counter() - t0:.1f}s")

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    gtext = torch.from_numpy(g.text).to(dev)
    rtext = torch.from_numpy(reads.text).to(dev)
    roff = torch.from_numpy(reads.offsets.view(np.int64)).to(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    opts = mc.QueryOpts(4, 4, 0, 0, 0)
    torch.cuda.synchronize()

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        db = mc.Database(K, WINDOW, SKETCH, CAP)
        mc.mc_db_set_profiling(db.h, True)
        db.add_targets(gtext, g.lengths, g.taxa)
        db.set_taxonomy(g.parents)
        ev[1].record()
        mc.mc_classify_ex(db.h, rtext, roff, n, opts, labels)
        ev[2].record()
        return db, ev

    for i in range(args.warmup):
        db, _ = step()
        torch.cuda.synchronize()
        db.close()
        log(f"warmup step {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {wall:.3f}s")

    build_ms = np.mean([r[1][0].elapsed_time(r[1][1]) for r in runs])
    cls_ms = np.mean([r[1][1].elapsed_time(r[1][2]) for r in runs])
    kt = [mc.mc_db_kernel_times(r[0].h) for r in runs]

    def avg_ms(kind):
        n_launch = sum(x[kind]["launches"] for x in kt)
        return sum(x[kind]["ms"] for x in kt) / max(1, n_launch)

    st = runs[-1][0].stats()
    gpu_labels = labels.cpu().numpy().view(np.uint32)
    for r in runs:
        r[0].close()

    # algorithmic bytes per launch ("Measurement")
    slots = st["n_windows"] * SKETCH
    pairs = st["n_pairs_inserted"]
    q_feats = float(st["q_features"])      # one classify launch per database
    q_locs = float(st["q_locations"])
    kernels = {
        "sketch": {"name": "k_sketch<2,true>", "avg_ms": avg_ms("sketch"),
                   "algorithmic_bytes": total_bp + 8.0 * slots,
                   "per_unit": "1 B of text per base read + 8 B per sketch slot written"},
        "scatter": {"name": "k_scan_parts + k_scatter", "avg_ms": avg_ms("scatter"),
                    "algorithmic_bytes": 8.0 * slots + 8.0 * pairs,
                    "per_unit": "8 B per slot read + 8 B per pair written"},
        "insert": {"name": "k_insert", "avg_ms": avg_ms("insert"),
                   "algorithmic_bytes": 16.0 * pairs,
                   "per_unit": "8 B per pair read + 8 B per pair stored"},
        "classify": {"name": "k_classify<512,4,2>", "avg_ms": avg_ms("classify"),
                     "algorithmic_bytes": float(reads.text.size) + 8.0 * (n + 1) + 4.0 * n
                     + 64.0 * q_feats + 4.0 * q_locs,
                     "per_unit": ("read bytes + 8 B offset + 4 B label per read, 64 B per "
                                  "sketch element probe, 4 B per location gathered")},
    }
    for kk in kernels.values():
        kk["achieved_gbs"] = kk["algorithmic_bytes"] / (kk["avg_ms"] * 1e-3) / 1e9 \
            if kk["avg_ms"] > 0 else 0.0
    dom = max(kernels.values(), key=lambda x: x["avg_ms"])
    achieved = dom["achieved_gbs"]
    roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None}

    out = {
        "metric": METRIC,
        "value": n / (cls_ms * 1e-3),
        "unit": "reads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"at-scale reference set: {g.lengths.size} genomes in 100 clusters "
                         f"(2-15% divergence), {total_bp / 1e9:.3f} Gbp; {n} single-end "
                         "150 bp reads, 1% substitutions, 5% foreign"),
            "k": K, "window": WINDOW, "sketch_size": SKETCH, "max_locations": CAP,
            "top_m": 4, "min_hits": 4, "hit_diff": 0,
        },
        "build_gbp_per_s": total_bp / 1e9 / (build_ms * 1e-3),
        "phases_ms": {"build": build_ms, "classify": cls_ms},
        "kernels": kernels,
        "db": {k: st[k] for k in ("n_windows", "n_pairs_inserted", "n_pairs_stored", "n_buckets",
                                  "table_bytes", "probe_sum", "n_cap_candidates")},
        "query": {"features_per_read": q_feats / n, "locations_per_read": q_locs / n,
                  "probes_per_feature": st["q_probes"] / max(1, st["q_features"]),
                  "classified_frac": float((gpu_labels != mc.MC_UNCLASSIFIED).mean())},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if args.cpu_sample > 0:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, reads, min(args.cpu_sample, n), threads,
                                           gpu_labels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
