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
    ap.add_argument("--uneven-records", type=int, default=20_000_000,
                    help="records of the uneven-batch leg (0 = skip)")
    ap.add_argument("--served-batches", type=int, default=100,
                    help="batches of the served-form trace (0 = skip the served leg)")
    ap.add_argument("--served-loads", type=str, default="0.7,1.0,1.5,2.0",
                    help="offered loads, as fractions of the plain launch's back-to-back "
                         "throughput, at which served and plain forms are compared")
    return ap.parse_args()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE counters
    (scaled by the copy-kernel calibration), or None if they were taken on other sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_classify_scale_10M_reads.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for name in t["sources"]:
        with open(os.path.join(ROOT, "paper_2106_08150_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return t["traffic_bytes"] if h.hexdigest() == t["sources_sha256"] else None


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


def uneven_leg(args, g, gtext, torch, mc, synth):
    """Mixed single-end (U{50..250} bp) and paired (2 x 150 bp, fragment
    N(400, 50)) records in one offsets array: autotuned launch shape, then the
    classification captured in a HIP graph and replayed."""
    recs = synth.mixed_records(g, args.uneven_records, seed=301, progress=log)
    n = recs.n_records
    mates = int((np.diff(recs.offsets) > 0).sum())
    dev = gtext.device
    r = torch.from_numpy(recs.text).to(dev)
    o = torch.from_numpy(recs.offsets.view(np.int64)).to(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    db = mc.Database(K, WINDOW, SKETCH, CAP)
    db.add_targets(gtext, g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    opts = mc.QueryOpts(4, 4, 0, 400, 1)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    default_ms = timed(lambda: mc.mc_classify_ex(db.h, r, o, n, opts, labels))
    ref = labels.clone()
    m = min(n, 2_000_000)
    sub_o = o[:2 * m + 1].contiguous()
    cfg, _ = mc.mc_db_autotune(db.h, r, sub_o, m, opts, labels)
    graph = mc.ClassifyGraph(db.h, r, o, n, opts, labels)
    graph_ms = timed(graph.launch)
    same = bool(torch.equal(labels, ref))
    graph.close()
    db.close()
    log(f"uneven: {n} records ({mates} mates), default {default_ms:.2f} ms, tuned "
        f"{cfg} + graph {graph_ms:.2f} ms, identical {same}")
    return {
        "workload": (f"{n} records in one paired-layout offsets array: 50% single-end "
                     "U{50..250} bp, 50% pairs 2 x 150 bp (fragment N(400, 50)), 1% "
                     "substitutions, 5% foreign; insert_size 400"),
        "records": n, "mates": mates,
        "default_config_ms": default_ms,
        "tuned_config": {"list_capacity": cfg[0], "waves_per_block": cfg[1],
                         "max_blocks": cfg[2]},
        "graph_ms": graph_ms,
        "records_per_s": n / (graph_ms * 1e-3),
        "mates_per_s": mates / (graph_ms * 1e-3),
        "labels_identical_to_default": same,
    }


def served_leg(args, g, gtext, torch, mc, synth):
    """Served request loop vs plain per-batch launches on one arrival trace.

    Trace: Poisson arrivals, batch sizes log-uniform in [1e3, 1e6] reads of
    U{100..250} bp (1% substitutions, 5% foreign); every 50 batches an
    on-demand addition of 20 genomes (2 new clusters, about 80 Mbp) with the
    extended taxonomy. Both forms start from the same freshly built database;
    latency = arrival -> labels in host memory.
    """
    import threading
    nb = args.served_batches
    unit_t, sizes = synth.arrival_trace(nb, seed=401, lo=1e3, hi=1e6, rate_hz=1.0)
    reads = synth.sample_reads_varlen(g, int(sizes.sum()), 100, 250, seed=402, foreign=0.05)
    cuts = np.concatenate([[0], np.cumsum(sizes)])
    # batch inputs in pinned host memory, as a serving front end would receive them
    batches = []
    for i in range(nb):
        off = reads.offsets[cuts[i]:cuts[i + 1] + 1]
        txt = torch.from_numpy(reads.text[int(off[0]):int(off[-1])]).pin_memory()
        batches.append((txt, (off - off[0]).astype(np.uint64)))
    staging = max(int(t.numel()) + 16 * (o.size + 1) for t, o in batches)
    adds, base = {}, g
    for i in range(50, nb, 50):
        add, parents = synth.addition_genomes(base, 2, 10, 8e7, seed=4000 + i)
        adds[i] = (add, parents)
        base = synth.Genomes(base.text[:0], base.lengths[:0], base.taxa[:0], parents)
    log(f"served trace: {nb} batches, {int(sizes.sum())} reads, {len(adds)} additions")

    # table headroom for the planned additions (no growth while serving)
    add_pairs = sum(int(((a.lengths.astype(np.int64) - K) // (WINDOW - K + 1) + 1).sum())
                    * SKETCH for a, _ in adds.values())

    def fresh_db():
        db = mc.Database(K, WINDOW, SKETCH, CAP)
        wins = int(((g.lengths.astype(np.int64) - K) // (WINDOW - K + 1) + 1).sum())
        db.reserve(wins * SKETCH + add_pairs)
        db.add_targets(gtext, g.lengths, g.taxa)
        db.set_taxonomy(g.parents)
        return db

    dev = gtext.device

    def plain_run(arrivals):
        db = fresh_db()
        labels, lat = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, (txt, off) in enumerate(batches):
            if arrivals is not None:
                wait = t0 + arrivals[i] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            if i in adds:
                add, parents = adds[i]
                db.add_targets(add.text, add.lengths, add.taxa)
                db.set_taxonomy(parents)
            r = txt.to(dev, non_blocking=True)
            o = torch.from_numpy(off.view(np.int64)).to(dev)
            lab, _ = db.classify(r, o, off.size - 1)
            labels.append(lab.cpu().numpy().view(np.uint32).copy())
            lat.append((time.perf_counter() - t0 - (arrivals[i] if arrivals is not None else 0))
                       * 1e3)
        span = time.perf_counter() - t0
        db.close()
        return labels, np.array(lat), span

    # throughput of back-to-back plain launches sets the arrival rates
    _, _, span0 = plain_run(None)
    plain_tput = reads.n_records / span0

    def served_run(arrivals):
        db = fresh_db()
        srv = mc.Server(db, slots=4, staging_bytes=staging)
        tickets = [None] * nb
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        late = [0.0] * nb   # arrival -> submit returned, ms

        def feeder():
            for i, (txt, off) in enumerate(batches):
                wait = t0 + arrivals[i] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                if i in adds:
                    add, parents = adds[i]
                    srv.add_targets(add.text, add.lengths, add.taxa, parents=parents)
                t = srv.submit(txt, off)
                late[i] = (time.perf_counter() - t0 - arrivals[i]) * 1e3
                tickets[i] = t

        th = threading.Thread(target=feeder)
        th.start()
        labels, lat = [], []
        for i in range(nb):
            while tickets[i] is None:
                time.sleep(0.0002)
            lab, _, ms = srv.wait(tickets[i])
            labels.append(lab.copy())
            # from arrival, as for plain launches: the server's submit -> labels
            # time plus the time from arrival until submit returned (an upper
            # bound: the submit call itself counts twice)
            lat.append(ms + late[i])
        th.join()
        span = time.perf_counter() - t0
        srv.close()
        db.close()
        return labels, np.array(lat), span

    def pct(v, p):
        v = np.sort(np.asarray(v))
        return float(v[min(v.size - 1, max(0, int(np.ceil(p / 100 * v.size)) - 1))])

    def summary(lat, span):
        return {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(np.mean(lat)),
                "reads_per_s": reads.n_records / span}

    results, same_all = [], True
    for load in [float(x) for x in args.served_loads.split(",") if x]:
        rate = load * plain_tput / float(sizes.mean())
        arrivals = unit_t / rate
        p_lab, p_lat, p_span = plain_run(arrivals)
        s_lab, s_lat, s_span = served_run(arrivals)
        same = all(np.array_equal(a, b) for a, b in zip(s_lab, p_lab))
        same_all &= same
        results.append({"offered_load": load, "batches_per_s": rate,
                         "served": summary(s_lat, s_span), "plain": summary(p_lat, p_span),
                         "labels_identical": bool(same)})
        log(f"load {load:.2f}: served p50 {pct(s_lat, 50):.2f} p99 {pct(s_lat, 99):.2f} ms, "
            f"plain p50 {pct(p_lat, 50):.2f} p99 {pct(p_lat, 99):.2f} ms, identical {same}")
    return {
        "trace": (f"{nb} batches, Poisson arrivals, sizes log-uniform 1e3..1e6 reads of "
                  f"100-250 bp (1% substitutions, 5% foreign), {len(adds)} addition(s) of 20 "
                  "genomes; the database is the at-scale set with headroom reserved; inputs "
                  "in pinned host memory; latency = arrival -> labels in host memory"),
        "reads": int(reads.n_records),
        "slots": 4,
        "plain_back_to_back_reads_per_s": plain_tput,
        "loads": results,
        "labels_identical": bool(same_all),
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
        "scatter": {"name": "k_scan_parts + k_scatter + k_hist2 + k_scan2 + k_scatter2",
                    "avg_ms": avg_ms("scatter"),
                    "algorithmic_bytes": 8.0 * slots + 8.0 * pairs + 24.0 * pairs,
                    "per_unit": ("8 B per slot read + 8 B per pair written (partitions), 8 B per "
                                 "pair read (slice histogram), 8 B read + 8 B written per pair "
                                 "(slices)")},
        "insert": {"name": "k_insert_slices + k_insert (deferred)", "avg_ms": avg_ms("insert"),
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
                "traffic": measured_traffic(dom["name"])}

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
    if args.uneven_records > 0:
        out["uneven"] = uneven_leg(args, g, gtext, torch, mc, synth)
    if args.served_batches > 0:
        out["served"] = served_leg(args, g, gtext, torch, mc, synth)
    if args.cpu_sample > 0:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, reads, min(args.cpu_sample, n), threads,
                                           gpu_labels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
