#!/usr/bin/env python3
"""Benchmark of the minhash classifier hot path on one MI355X.

One step is one pass of the whole hot path over one batch: build the database
of the at-scale reference set (1,000 synthetic genomes, about 4 Gbp, already
resident in HBM: encode, canonical k-mers, h1, bottom-s sketches, inserts, cap)
and classify its read set (10M x 150 bp, 1% substitutions, 5% foreign reads:
sketch, lookup, sort, window counts, sliding window, top hits, LCA labels).
The printed JSON line's ``value`` is classified reads/s of that step's
classification phase; ``build_gbp_per_s`` its build rate; both with inputs
resident in HBM and timed with HIP events.

Besides the steps, the same line carries:

* ``uneven``: 20M mixed single-end / paired records in one offsets array,
  autotuned launch shape, captured in a HIP graph;
* ``served``: the served request loop against plain per-batch launches on one
  Poisson arrival trace (10 Gbp resident set, on-demand genome additions);
* ``large``: the large single-GPU configuration: a 30 Gbp reference set built
  in full (timed, device-resident and including the copy from pinned host
  memory), its kernel classification rate, and 100M reads streamed through the
  served loop (and through plain per-batch launches) with the database
  resident;
* ``roofline`` (dominant kernel against the 8 TB/s HBM peak, plus the build and
  classify kernels against the measured random-access ceilings) and
  ``cpu_baseline`` (the CPU oracle on a read sample of the same workload, at 1
  thread and at the host's core share).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DB build Gbp/s; reads/s classified; p50/p99 batch latency vs plain launch"
HBM_PEAK_GBS = 8000.0
# Random-access ceilings measured on one MI355X with libmc_peaks
# (python -m paper_2106_08150_amd.peaks; 16 GiB working sets)
CEIL_LINES128_GPS = 38.44e9      # random 128-byte line reads / s
CEIL_CAS_GPS = 16.99e9           # random 64-bit atomic CAS / s
CEIL_COPY_GBS = 5155.89          # streaming copy, read + write bytes / s (GB/s)
K, WINDOW, SKETCH, CAP = 16, 128, 16, 254


T_START = time.perf_counter()


def log(msg: str) -> None:
    print(f"[bench {time.perf_counter() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--total-bp", type=float, default=4.0e9)
    ap.add_argument("--reads", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=20_000,
                    help="reads classified by the CPU oracle (0 = skip the CPU baseline)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="0 = min(16, host cores): the host share of one GPU")
    ap.add_argument("--uneven-records", type=int, default=20_000_000,
                    help="records of the uneven-batch leg (0 = skip)")
    ap.add_argument("--served-batches", type=int, default=100,
                    help="batches of the served-form trace (0 = skip the served leg)")
    ap.add_argument("--served-loads", type=str, default="0.7,1.0,1.5,2.0",
                    help="offered loads, as fractions of the plain launch's back-to-back "
                         "throughput, at which served and plain forms are compared")
    ap.add_argument("--served-gbp", type=float, default=10.0,
                    help="reference set of the served leg: this many Gbp in 250 clusters of 10 "
                         "(0 = the at-scale set)")
    ap.add_argument("--large-gbp", type=float, default=30.0,
                    help="large reference set (7,500 genomes in 750 clusters, 1-20%% "
                         "divergence) of this many Gbp (0 = skip the large leg)")
    ap.add_argument("--large-reads", type=int, default=100_000_000,
                    help="150 bp reads streamed through the served loop in the large leg")
    ap.add_argument("--large-batch", type=int, default=1_000_000,
                    help="reads per batch of the large leg's stream")
    ap.add_argument("--large-kernel-reads", type=int, default=10_000_000,
                    help="reads of the stream classified device-resident in one launch "
                         "(the kernel rate)")
    ap.add_argument("--large-builds", type=int, default=2,
                    help="timed device-resident builds of the large set (after a warm-up)")
    ap.add_argument("--large-shape", type=str, default="auto",
                    help="launch shape of the large leg: 'auto' (mc_db_autotune on the first 2M "
                         "reads) or list capacity, waves per workgroup, largest grid")
    ap.add_argument("--served-parity", type=int, default=2000,
                    help="records of the served trace checked against the (feature-filtered) "
                         "oracle on the database after all its on-demand additions, plus a "
                         "table slice (0 = skip; the oracle's scan of 10 Gbp takes about a "
                         "minute of host time)")
    ap.add_argument("--large-parity", type=int, default=2000,
                    help="reads of the large stream checked against the (feature-filtered) "
                         "oracle, plus a table slice (0 = skip; the oracle's scan of 30 Gbp "
                         "takes about three minutes of host time)")
    ap.add_argument("--launch-shape", type=str, default="256,4,16384",
                    help="classification launch shape of the main leg: list capacity, waves "
                         "per workgroup, largest grid (the shape mc_db_autotune picks on this "
                         "workload)")
    return ap.parse_args()


def windows_of(lengths) -> int:
    L = np.asarray(lengths, dtype=np.int64)
    return int(np.where(L >= K, (L - K) // (WINDOW - K + 1) + 1, 0).sum())


def pct(v, p):
    v = np.sort(np.asarray(v))
    return float(v[min(v.size - 1, max(0, int(np.ceil(p / 100 * v.size)) - 1))])


def host_info(threads):
    """Host identity for the CPU baseline: core count and CPU model."""
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "threads_used": threads, "cpu_model": model}


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


# ------------------------------------------------------------ CPU oracle --
def cpu_baseline(g, reads, n_sample, threads, gpu_labels):
    """The oracle on a read sample: it indexes only the features the sample
    looks up (exact for the sample; pinned against the unfiltered oracle in
    tests/test_oracle_filter.py), then classifies the sample at `threads`
    threads and a tenth of it at one thread. Its unfiltered build rate is
    timed at one thread on the first genomes."""
    import oracle
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
    n1 = max(1, n_sample // 10)
    odb.classify(reads.text, reads.offsets, first=0, count=n1, threads=1)
    t4 = time.perf_counter()
    mism = int((labels != gpu_labels[:n_sample]).sum())
    # unfiltered build, one thread, on the first genomes (about 60 Mbp)
    n_g = int(np.searchsorted(np.cumsum(g.lengths.astype(np.int64)), 6e7)) + 1
    sub = g.offsets[n_g]
    full = oracle.OracleDB(K, WINDOW, SKETCH, CAP)
    t5 = time.perf_counter()
    full.add_targets(g.text[:int(sub)], g.lengths[:n_g], g.taxa[:n_g], threads=1)
    t6 = time.perf_counter()
    log(f"oracle: filtered scan {t2 - t1:.1f}s ({threads} threads), classify {n_sample} reads "
        f"{t3 - t2:.2f}s, {n1} reads at 1 thread {t4 - t3:.2f}s, full build of "
        f"{int(sub) / 1e6:.0f} Mbp at 1 thread {t6 - t5:.1f}s; label mismatches vs GPU: {mism}")
    return {
        "value": n_sample / (t3 - t2), "unit": "reads/s", "cores": threads, "kind": "oracle",
        "sample": (f"first {n_sample} reads of the at-scale read set, classified against the "
                   "oracle index restricted to the features those reads look up (built by "
                   "sketching every window of all genomes)"),
        "reads_per_s_1_thread": n1 / (t4 - t3),
        "build_bp_per_s_1_thread": float(sub) / (t6 - t5),
        "build_sample": f"unfiltered oracle build of the first {n_g} genomes ({int(sub)} bp)",
        "filtered_scan_bp_per_s": float(g.lengths.sum()) / (t2 - t1),
        "host": host_info(threads),
        "sample_label_mismatches_vs_gpu": mism,
    }


def oracle_sample_parity(g, reads, sample, gl, gt, slice_hi, gf, gloc, threads):
    """Feature-filtered oracle on a read sample and a table slice (features
    <= slice_hi); returns (record mismatches, table slice equal)."""
    import oracle
    feats = [oracle.query_features(reads.text, reads.offsets, K, WINDOW, SKETCH, int(i), 1, False)
             for i in sample]
    odb = oracle.OracleDB(K, WINDOW, SKETCH, CAP)
    odb.set_filter(np.unique(np.concatenate(feats)))
    odb.set_filter_range(0, slice_hi)
    # the genomes in pieces of about 2 Gbp (target ids run on), with a line each
    off = g.offsets.astype(np.int64)
    cuts = np.searchsorted(off, np.arange(0, off[-1], 2e9))[1:].tolist() + [g.lengths.size]
    a = 0
    for b in cuts:
        if b <= a:
            continue
        odb.add_targets(g.text[off[a]:off[b]], g.lengths[a:b], g.taxa[a:b], threads=threads)
        log(f"oracle: scanned {b}/{g.lengths.size} genomes")
        a = b
    odb.set_taxonomy(g.parents)
    of, oloc = odb.dump()
    keep = of <= slice_hi
    table_ok = bool(np.array_equal(gf, of[keep]) and np.array_equal(gloc, oloc[keep]))
    bad = 0
    for j, i in enumerate(sample):
        ol, ot = odb.classify(reads.text, reads.offsets, first=int(i), count=1)
        bad += int(ol[0] != gl[j] or not np.array_equal(ot[0], gt[j]))
    return bad, table_ok


# --------------------------------------------------------- served forms --
def plain_run(torch, mc, db, batches, adds, arrivals):
    """Sequential per-batch launches: copy in, classify, labels back, one batch
    at a time. Returns labels, latencies (arrival -> labels in host memory, ms)
    and the span (s)."""
    dev = torch.device("cuda", 0)
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
    return labels, np.array(lat), time.perf_counter() - t0


def served_run(torch, mc, db, batches, adds, arrivals, staging, slots=4, stage_log=None):
    """The served loop on the same arrivals (None: back to back): a feeder
    thread submits each batch at its arrival time; latency = arrival ->
    labels in host memory."""
    nb = len(batches)
    srv = mc.Server(db, slots=slots, staging_bytes=staging)
    tickets = [None] * nb
    late = [0.0] * nb   # arrival -> submit returned, ms
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    arr = arrivals if arrivals is not None else np.zeros(nb)

    def feeder():
        for i, (txt, off) in enumerate(batches):
            wait = t0 + arr[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            if i in adds:
                add, parents = adds[i]
                srv.add_targets(add.text, add.lengths, add.taxa, parents=parents)
            t = srv.submit(txt, off)
            late[i] = (time.perf_counter() - t0 - arr[i]) * 1e3
            tickets[i] = t

    th = threading.Thread(target=feeder)
    th.start()
    labels, lat, stages = [], [], []
    for i in range(nb):
        while tickets[i] is None:
            time.sleep(0.0002)
        lab, _, tm = srv.wait_times(tickets[i])
        labels.append(lab.copy())
        # from arrival, as for plain launches: the server's submit -> labels
        # time plus the time from arrival until submit returned (an upper
        # bound: the submit call itself counts twice)
        lat.append(tm["total_ms"] + late[i])
        tm["submit_late_ms"] = late[i]
        tm["records"] = int(batches[i][1].size - 1)
        stages.append(tm)
    th.join()
    span = time.perf_counter() - t0
    srv.close()
    if stage_log is not None:
        stage_log.extend(stages)
    return labels, np.array(lat), span


def slowest_stages(stages, lat, n=3):
    """Stage split of the n slowest batches (ms), slowest first."""
    order = np.argsort(lat)[::-1][:n]
    keys = ("records", "submit_late_ms", "admit_ms", "copy_ms", "launch_ms", "finish_ms",
            "gpu_kernels_ms", "gpu_copy_back_ms")
    return [{k: (round(stages[i][k], 3) if k != "records" else stages[i][k]) for k in keys}
            for i in order]


def summary(lat, span, n_reads):
    return {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(np.mean(lat)),
            "max_ms": float(np.max(lat)), "reads_per_s": n_reads / span}


# ------------------------------------------------------------------ legs --
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
    # one launch shape for all records, tuned
    cfg, _ = mc.mc_db_autotune(db.h, r, sub_o, m, opts, labels)
    flat_ms = timed(lambda: mc.mc_classify_ex(db.h, r, o, n, opts, labels))
    same = bool(torch.equal(labels, ref))
    # size classes: single-end records (at most 3 windows) and pairs, each
    # class with its own tuned shape
    mc.mc_db_set_routing(db.h, [3], [cfg, cfg])
    mc.mc_db_autotune(db.h, r, sub_o, m, opts, labels)
    _, class_shapes = mc.mc_db_get_routing(db.h)
    routed_ms = timed(lambda: mc.mc_classify_ex(db.h, r, o, n, opts, labels))
    same &= bool(torch.equal(labels, ref))
    if flat_ms <= routed_ms:   # the graph replays the faster plan
        mc.mc_db_set_routing(db.h, [], [cfg])
    graph = mc.ClassifyGraph(db.h, r, o, n, opts, labels)
    graph_ms = timed(graph.launch)
    same &= bool(torch.equal(labels, ref))
    graph.close()
    db.close()
    del r, o, labels, ref
    log(f"uneven: {n} records ({mates} mates), default {default_ms:.2f} ms, tuned {cfg} "
        f"{flat_ms:.2f} ms, size classes {class_shapes} {routed_ms:.2f} ms, graph "
        f"{graph_ms:.2f} ms, identical {same}")
    return {
        "workload": (f"{n} records in one paired-layout offsets array: 50% single-end "
                     "U{50..250} bp, 50% pairs 2 x 150 bp (fragment N(400, 50)), 1% "
                     "substitutions, 5% foreign; insert_size 400"),
        "records": n, "mates": mates,
        "default_config_ms": default_ms,
        "tuned_config": {"list_capacity": cfg[0], "waves_per_block": cfg[1],
                         "max_blocks": cfg[2]},
        "tuned_ms": flat_ms,
        "size_classes": {"max_windows": [3], "tuned_shapes": [list(x) for x in class_shapes],
                         "ms": routed_ms},
        "graph_plan": "size classes" if routed_ms < flat_ms else "one tuned shape",
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
        # the new genomes in pinned host memory, as a loader would leave them
        # (both forms copy them from there)
        text = torch.from_numpy(add.text).pin_memory()
        add = synth.Genomes(text.numpy(), add.lengths, add.taxa, add.parents)
        adds[i] = (add, parents)
        base = synth.Genomes(base.text[:0], base.lengths[:0], base.taxa[:0], parents)
    log(f"served trace: {nb} batches, {int(sizes.sum())} reads, {len(adds)} additions")
    # table headroom for the planned additions (no growth while serving)
    add_pairs = sum(windows_of(a.lengths) * SKETCH for a, _ in adds.values())

    def fresh_db():
        db = mc.Database(K, WINDOW, SKETCH, CAP)
        db.reserve(windows_of(g.lengths) * SKETCH + add_pairs)
        db.add_targets(gtext, g.lengths, g.taxa)
        db.set_taxonomy(g.parents)
        return db

    def plain(arrivals):
        db = fresh_db()
        out = plain_run(torch, mc, db, batches, adds, arrivals)
        db.close()
        return out

    def served(arrivals, stage_log=None):
        db = fresh_db()
        out = served_run(torch, mc, db, batches, adds, arrivals, staging, stage_log=stage_log)
        db.close()
        return out

    # throughput of back-to-back plain launches sets the arrival rates
    _, _, span0 = plain(None)
    plain_tput = reads.n_records / span0
    results, same_all = [], True
    for load in [float(x) for x in args.served_loads.split(",") if x]:
        rate = load * plain_tput / float(sizes.mean())
        arrivals = unit_t / rate
        p_lab, p_lat, p_span = plain(arrivals)
        stages = []
        s_lab, s_lat, s_span = served(arrivals, stages)
        same = all(np.array_equal(a, b) for a, b in zip(s_lab, p_lab))
        same_all &= same
        slow_plain = np.argsort(p_lat)[::-1][:3]
        results.append({"offered_load": load, "batches_per_s": rate,
                        "served": summary(s_lat, s_span, reads.n_records),
                        "plain": summary(p_lat, p_span, reads.n_records),
                        "served_slowest": slowest_stages(stages, s_lat),
                        "plain_slowest": [{"records": int(batches[i][1].size - 1),
                                           "ms": round(float(p_lat[i]), 3)}
                                          for i in slow_plain],
                        "labels_identical": bool(same)})
        log(f"load {load:.2f}: served p50 {pct(s_lat, 50):.2f} p99 {pct(s_lat, 99):.2f} ms, "
            f"plain p50 {pct(p_lat, 50):.2f} p99 {pct(p_lat, 99):.2f} ms, identical {same}")
    parity = None
    if args.served_parity > 0 and adds:
        parity = served_parity(args, g, gtext, reads, adds, add_pairs, torch, mc)
    return {
        "oracle_parity": parity,
        "trace": (f"{nb} batches, Poisson arrivals, sizes log-uniform 1e3..1e6 reads of "
                  f"100-250 bp (1% substitutions, 5% foreign), {len(adds)} addition(s) of 20 "
                  f"genomes; the database: {g.lengths.size} genomes, "
                  f"{float(g.lengths.sum()) / 1e9:.2f} Gbp, with headroom reserved; inputs "
                  "in pinned host memory; latency = arrival -> labels in host memory"),
        "reads": int(reads.n_records),
        "slots": 4,
        "plain_back_to_back_reads_per_s": plain_tput,
        "loads": results,
        "labels_identical": bool(same_all),
    }


def records_subset(reads, sample):
    """Text and u64 offsets of the single-end records `sample` of `reads`."""
    off = reads.offsets.astype(np.int64)
    pieces = [reads.text[off[i]:off[i + 1]] for i in sample]
    o = np.zeros(len(pieces) + 1, np.int64)
    o[1:] = np.cumsum([p.size for p in pieces])
    return np.concatenate(pieces), o


def served_parity(args, g, gtext, reads, adds, add_pairs, torch, mc):
    """The served leg's database after every on-demand addition (built the
    way the served loop grows it: the reference set, then each addition with
    its extended taxonomy) against the feature-filtered oracle on all those
    genomes: a sample of the trace's records (labels and top hits) and a slice
    of the table (features <= 2^20 - 1)."""
    from paper_2106_08150_amd import synth
    dev = gtext.device
    db = mc.Database(K, WINDOW, SKETCH, CAP)
    db.reserve(windows_of(g.lengths) * SKETCH + add_pairs)
    db.add_targets(gtext, g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    texts, lens, taxa, parents = [g.text], [g.lengths], [g.taxa], g.parents
    for i in sorted(adds):
        add, par = adds[i]
        db.add_targets(add.text, add.lengths, add.taxa)
        db.set_taxonomy(par)
        texts.append(add.text)
        lens.append(add.lengths)
        taxa.append(add.taxa)
        parents = par
    full = synth.Genomes(np.concatenate(texts), np.concatenate(lens), np.concatenate(taxa),
                         parents)
    sample = np.sort(np.random.default_rng(11).choice(reads.n_records, args.served_parity,
                                                      replace=False))
    txt, off = records_subset(reads, sample)
    lab, top = db.classify(torch.from_numpy(txt).to(dev), torch.from_numpy(off).to(dev),
                           sample.size, with_top=True)
    torch.cuda.synchronize()
    gl = lab.cpu().numpy().view(np.uint32)
    gt = top.cpu().numpy().view(np.uint32)
    slice_hi = (1 << 20) - 1
    gf, gloc = db.dump(0, slice_hi)
    st = db.stats()
    db.close()
    t0 = time.perf_counter()
    bad, table_ok = oracle_sample_parity(full, reads, sample, gl, gt, slice_hi, gf, gloc,
                                         min(16, os.cpu_count() or 1))
    log(f"served: oracle parity after {len(adds)} addition(s) on {sample.size} records: "
        f"{bad} mismatches, table slice equal {table_ok}")
    return {"sample_records": int(sample.size), "mismatches": bad,
            "genomes": int(full.lengths.size), "gbp": float(full.lengths.sum()) / 1e9,
            "additions": len(adds), "table_slice_features_le": slice_hi,
            "table_slice_pairs": int(gf.size), "table_slice_equal": table_ok,
            "n_pairs_stored": st["n_pairs_stored"], "oracle_s": time.perf_counter() - t0}


def large_leg(args, g, stream, torch, mc):
    """The large single-GPU configuration: full builds of the large reference
    set (timed device-resident, and once including the copy of the genomes
    from pinned host memory), the classification kernel's rate on the first
    reads of the stream (device-resident, one launch), then the whole stream
    through the served loop and through plain per-batch launches with the
    database resident, on the same arrivals; labels must agree everywhere."""
    dev = torch.device("cuda", 0)
    total_bp = int(g.lengths.sum())
    props = torch.cuda.get_device_properties(dev)
    mc.mc_set_cached_memory_limit(props.total_memory // 2)   # builds reuse device blocks
    # genomes in pinned host memory, as a loader would leave them
    pinned = torch.empty(g.text.size, dtype=torch.uint8, pin_memory=True)
    pinned.numpy()[:] = g.text
    gtext = torch.empty(g.text.size, dtype=torch.uint8, device=dev)
    db = None

    def build(copy_in):
        nonlocal db
        if db is not None:
            db.close()
            db = None
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        if copy_in:
            gtext.copy_(pinned, non_blocking=True)
        e[1].record()
        db = mc.Database(K, WINDOW, SKETCH, CAP)
        mc.mc_db_set_profiling(db.h, True)
        db.add_targets(gtext, g.lengths, g.taxa)
        db.set_taxonomy(g.parents)
        e[2].record()
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[2]), e[1].elapsed_time(e[2]), mc.mc_db_kernel_times(db.h)

    with_copy, _, _ = build(True)          # also the warm-up
    del pinned
    log(f"large: build incl. copy from pinned host memory {with_copy:.1f} ms")
    builds, kts = [], []
    for i in range(args.large_builds):
        _, ms, kt = build(False)
        builds.append(ms)
        kts.append(kt)
        log(f"large: build {i + 1}: {ms:.1f} ms")
    mc.mc_set_cached_memory_limit(0)
    del gtext
    torch.cuda.empty_cache()

    # kernel rate: the first reads of the stream, device-resident, one launch
    nk = min(args.large_kernel_reads, stream.n_records)
    rt = torch.from_numpy(stream.text[:nk * 150]).to(dev)
    ro = torch.from_numpy(stream.offsets[:nk + 1].view(np.int64)).to(dev)
    klab = torch.empty(nk, dtype=torch.int32, device=dev)
    opts = mc.QueryOpts(4, 4, 0, 0, 0)
    if args.large_shape == "auto":
        m = min(nk, 2_000_000)
        shape, _ = mc.mc_db_autotune(db.h, rt, ro[:m + 1].contiguous(), m, opts, klab)
        log(f"large: autotuned launch shape {shape}")
    else:
        shape = tuple(int(x) for x in args.large_shape.split(","))
        mc.mc_db_set_launch_config(db.h, *shape)
    m = min(nk, 2_000_000)
    st0 = db.stats()
    cls = []
    for i in range(1 + 3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mc.mc_classify_ex(db.h, rt, ro, nk, opts, klab)
        e1.record()
        torch.cuda.synchronize()
        if i:
            cls.append(e0.elapsed_time(e1))
    kt_cls = mc.mc_db_kernel_times(db.h)
    st = db.stats()
    kernel_labels = klab.cpu().numpy().view(np.uint32).copy()
    log(f"large: kernel classify {nk} reads {np.mean(cls):.2f} ms")
    # the condensed layout (bucket table kept): conversion time, kernel rate
    torch.cuda.synchronize()
    t_c = time.perf_counter()
    db.condense()
    condense_ms = (time.perf_counter() - t_c) * 1e3
    cst = db.stats()
    if args.large_shape == "auto":
        cshape, _ = mc.mc_db_autotune(db.h, rt, ro[:m + 1].contiguous(), m, opts, klab)
    else:
        cshape = shape
    ccls = []
    for i in range(1 + 3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mc.mc_classify_ex(db.h, rt, ro, nk, opts, klab)
        e1.record()
        torch.cuda.synchronize()
        if i:
            ccls.append(e0.elapsed_time(e1))
    cond_same = bool(np.array_equal(klab.cpu().numpy().view(np.uint32), kernel_labels))
    condensed = {"condense_ms": condense_ms, "condensed_bytes": cst["condensed_bytes"],
                 "launch_shape": list(cshape), "kernel_classify_ms": float(np.mean(ccls)),
                 "kernel_reads_per_s": nk / (np.mean(ccls) * 1e-3),
                 "labels_identical_to_bucket_table": cond_same}
    log(f"large: condensed layout in {condense_ms:.0f} ms ({cst['condensed_bytes'] / 1e9:.1f} GB), "
        f"kernel classify {np.mean(ccls):.2f} ms, identical {cond_same}")
    del rt, ro, klab

    # the stream: batches in pinned host memory (views of one pinned buffer)
    B = args.large_batch
    nbat = (stream.n_records + B - 1) // B
    pinned_stream = torch.empty(stream.text.size, dtype=torch.uint8, pin_memory=True)
    pinned_stream.numpy()[:] = stream.text
    batches = []
    for i in range(nbat):
        a, b = i * B, min(stream.n_records, (i + 1) * B)
        batches.append((pinned_stream[a * 150:b * 150],
                        (stream.offsets[a:b + 1] - stream.offsets[a]).astype(np.uint64)))
    staging = max(int(t.numel()) + 16 * (o.size + 1) for t, o in batches)
    p_lab0, _, p_span0 = plain_run(torch, mc, db, batches, {}, None)
    plain_tput = stream.n_records / p_span0
    s_lab0, s_lat0, s_span0 = served_run(torch, mc, db, batches, {}, None, staging)
    rng = np.random.Generator(np.random.PCG64(503))
    load = 0.9
    arrivals = np.cumsum(rng.exponential(1.0, size=nbat)) / (load * plain_tput / B)
    p_lab, p_lat, p_span = plain_run(torch, mc, db, batches, {}, arrivals)
    s_lab, s_lat, s_span = served_run(torch, mc, db, batches, {}, arrivals, staging)
    same = all(np.array_equal(a, b) for a, b in zip(s_lab, p_lab))
    same &= all(np.array_equal(a, b) for a, b in zip(s_lab0, p_lab0))
    same &= all(np.array_equal(a, b) for a, b in zip(p_lab, p_lab0))
    kb = (nk + B - 1) // B
    same &= bool(np.array_equal(np.concatenate(p_lab0[:kb])[:nk], kernel_labels))
    del batches, pinned_stream
    log(f"large: stream {stream.n_records} reads: plain back-to-back {plain_tput / 1e6:.1f}M/s, "
        f"served back-to-back {stream.n_records / s_span0 / 1e6:.1f}M/s; at {load} x plain: "
        f"served p50 {pct(s_lat, 50):.1f} p99 {pct(s_lat, 99):.1f} ms, plain p50 "
        f"{pct(p_lat, 50):.1f} p99 {pct(p_lat, 99):.1f} ms; labels identical {same}")
    parity = None
    if args.large_parity > 0:
        gl = np.concatenate(s_lab)
        sample = np.sort(np.random.default_rng(7).choice(stream.n_records, args.large_parity,
                                                         replace=False))
        # labels and top hits of the sample records from one more launch
        rows = stream.text.reshape(-1, 150)[sample]
        sub = torch.from_numpy(np.ascontiguousarray(rows).reshape(-1)).to(dev)
        so = torch.from_numpy(np.arange(sample.size + 1, dtype=np.int64) * 150).to(dev)
        lab, top = db.classify(sub, so, sample.size, with_top=True)
        torch.cuda.synchronize()
        gsl = lab.cpu().numpy().view(np.uint32)
        gst = top.cpu().numpy().view(np.uint32)
        slice_hi = (1 << 20) - 1
        gf, gloc = db.dump(0, slice_hi)
        t0 = time.perf_counter()
        bad, table_ok = oracle_sample_parity(g, stream, sample, gsl, gst, slice_hi, gf, gloc,
                                             min(16, os.cpu_count() or 1))
        parity = {"sample_reads": int(sample.size), "mismatches": bad,
                  "stream_labels_equal": bool(np.array_equal(gsl, gl[sample])),
                  "table_slice_features_le": slice_hi, "table_slice_pairs": int(gf.size),
                  "table_slice_equal": table_ok, "oracle_s": time.perf_counter() - t0}
        log(f"large: oracle parity on {sample.size} reads: {bad} mismatches, table slice "
            f"equal {table_ok}")
    db.close()
    stage = {k: float(np.mean([x[k]["ms"] for x in kts])) for k in ("sketch", "scatter", "insert")}
    q_feats = st["q_features"] - st0["q_features"]
    q_probes = st["q_probes"] - st0["q_probes"]
    q_locs = st["q_locations"] - st0["q_locations"]
    cls_ms = float(np.mean(cls))
    k_ms = kt_cls["classify"]["ms"] / max(1, kt_cls["classify"]["launches"])
    return {
        "workload": (f"large reference set: {g.lengths.size} genomes in 750 clusters (1-20% "
                     f"divergence), {total_bp / 1e9:.3f} Gbp; {stream.n_records} single-end "
                     "150 bp reads, 1% substitutions, 5% foreign, streamed in batches of "
                     f"{B}"),
        "build_ms": float(np.mean(builds)),
        "build_gbp_per_s": total_bp / 1e9 / (np.mean(builds) * 1e-3),
        "build_incl_h2d_ms": with_copy,
        "build_incl_h2d_gbp_per_s": total_bp / 1e9 / (with_copy * 1e-3),
        "build_stage_ms": stage,
        "build_pairs_per_s": st["n_pairs_inserted"] / (np.mean(builds) * 1e-3),
        "kernel_reads": nk,
        "kernel_classify_ms": cls_ms,
        "kernel_reads_per_s": nk / (cls_ms * 1e-3),
        "kernel_launch_shape": list(shape),
        "classify_kernel_ms": k_ms,
        "classify_lines_per_s": q_probes / 4 / (k_ms * 1e-3),
        "classify_frac_of_line128_ceiling": q_probes / 4 / (k_ms * 1e-3) / CEIL_LINES128_GPS,
        "stream": {
            "reads": int(stream.n_records), "batches": nbat,
            "plain_back_to_back_reads_per_s": plain_tput,
            "served_back_to_back_reads_per_s": stream.n_records / s_span0,
            "served_back_to_back": summary(s_lat0, s_span0, stream.n_records),
            "offered_load": load,
            "served": summary(s_lat, s_span, stream.n_records),
            "plain": summary(p_lat, p_span, stream.n_records),
            "inputs": "batches in pinned host memory; latency = arrival -> labels in host memory",
        },
        "labels_identical": bool(same),
        "db": {k: st[k] for k in ("n_windows", "n_pairs_inserted", "n_pairs_stored", "n_features",
                                  "n_buckets", "table_bytes", "load_factor")},
        "query": {"features_per_read": q_feats / (4 * nk), "locations_per_read": q_locs / (4 * nk),
                  "probes_per_feature": q_probes / max(1, q_feats),
                  "large_pass_records_per_launch":
                      (st["q_large_records"] - st0["q_large_records"]) / 4,
                  "hbm_pass_records_per_launch": (st["q_hbm_records"] - st0["q_hbm_records"]) / 4,
                  "classified_frac": float((kernel_labels != mc.MC_UNCLASSIFIED).mean())},
        "oracle_parity": parity,
        "condensed": condensed,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the classifier here runs on a single MI355X "
              "and has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import paper_2106_08150_amd as mc
    from paper_2106_08150_amd import synth

    if not os.path.exists(mc.LIB_PATH):   # fail loudly without the HIP library (loaded below,
        mc.lib()                          # after the forked generators and torch)
    t0 = time.perf_counter()
    # every input is generated before the process touches the GPU (the large
    # sets by forked workers)
    g_large = stream = g_served = None
    if args.large_gbp > 0:
        g_large = synth.large_genomes(total_bp=args.large_gbp * 1e9, progress=log)
        stream = synth.stream_reads(g_large, args.large_reads, seed=502, progress=log)
        log(f"large set: {g_large.lengths.size} genomes, {g_large.lengths.sum() / 1e9:.3f} Gbp, "
            f"{stream.n_records} reads ({time.perf_counter() - t0:.1f}s)")
    if args.served_batches > 0 and args.served_gbp > 0:
        g_served = synth.large_genomes(seed=403, total_bp=args.served_gbp * 1e9, n_clusters=250,
                                       per_cluster=10, div_lo=0.02, div_hi=0.15, level1=50,
                                       progress=log)
    g = synth.scale_genomes(total_bp=args.total_bp, progress=log)
    reads = synth.scale_reads(g, n=args.reads, progress=log)
    total_bp = int(g.lengths.sum())
    n = reads.n_records
    log(f"generated every input in {time.perf_counter() - t0:.1f}s")

    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    mc.lib()
    props = torch.cuda.get_device_properties(dev)
    g_pinned = torch.empty(g.text.size, dtype=torch.uint8, pin_memory=True)
    g_pinned.numpy()[:] = g.text
    gtext = torch.empty(g.text.size, dtype=torch.uint8, device=dev)
    gtext.copy_(g_pinned)
    rtext = torch.from_numpy(reads.text).to(dev)
    roff = torch.from_numpy(reads.offsets.view(np.int64)).to(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    opts = mc.QueryOpts(4, 4, 0, 0, 0)
    shape = tuple(int(x) for x in args.launch_shape.split(","))
    cls_kernel = f"k_classify<{shape[0]},{shape[1]},2>"
    torch.cuda.synchronize()

    # the steps rebuild the same database: its device blocks are reused from
    # one step to the next instead of being unmapped and mapped again
    mc.mc_set_cached_memory_limit(props.total_memory // 2)
    live = []   # at-scale database handles alive: at most one at any time

    def step(keep=False, copy_in=False):
        """Build + classify; returns (build ms, classify ms, kernel times). Only
        numbers leave the step: its database is closed before it returns (the
        last one is kept in `live` for its statistics)."""
        assert not live, "an at-scale database is still alive"
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        if copy_in:
            gtext.copy_(g_pinned, non_blocking=True)
        db = mc.Database(K, WINDOW, SKETCH, CAP)
        live.append(db)
        mc.mc_db_set_launch_config(db.h, *shape)
        mc.mc_db_set_profiling(db.h, True)
        db.add_targets(gtext, g.lengths, g.taxa)
        db.set_taxonomy(g.parents)
        ev[1].record()
        mc.mc_classify_ex(db.h, rtext, roff, n, opts, labels)
        ev[2].record()
        kt = mc.mc_db_kernel_times(db.h)   # waits for the step's launches
        ev[2].synchronize()
        out = (ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), kt)
        if not keep:
            live.pop().close()
        return out

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    runs = [step(keep=(i == args.steps - 1)) for i in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {wall:.3f}s")

    build_ms = float(np.mean([r[0] for r in runs]))
    cls_ms = float(np.mean([r[1] for r in runs]))
    kt = [r[2] for r in runs]

    def avg_ms(kind):
        n_launch = sum(x[kind]["launches"] for x in kt)
        return sum(x[kind]["ms"] for x in kt) / max(1, n_launch)

    st = live[0].stats()
    gpu_labels = labels.cpu().numpy().view(np.uint32)
    # the same classification from the condensed layout of the last step's table
    db = live[0]
    torch.cuda.synchronize()
    t_c = time.perf_counter()
    db.condense()
    condense_ms = (time.perf_counter() - t_c) * 1e3
    cbytes = db.stats()["condensed_bytes"]
    c_ms = []
    for i in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mc.mc_classify_ex(db.h, rtext, roff, n, opts, labels)
        e1.record()
        torch.cuda.synchronize()
        if i:
            c_ms.append(e0.elapsed_time(e1))
    condensed = {"condense_ms": condense_ms, "condensed_bytes": cbytes,
                 "classify_ms": float(np.mean(c_ms)),
                 "reads_per_s": n / (np.mean(c_ms) * 1e-3),
                 "launch_shape": list(shape),
                 "labels_identical_to_bucket_table":
                     bool(np.array_equal(labels.cpu().numpy().view(np.uint32), gpu_labels))}
    log(f"condensed layout: {condense_ms:.0f} ms, {cbytes / 1e9:.2f} GB, classify "
        f"{np.mean(c_ms):.2f} ms")
    live.pop().close()
    # one more build that starts from the genomes in pinned host memory
    h2d_build_ms = step(copy_in=True)[0]
    del g_pinned
    mc.mc_set_cached_memory_limit(0)   # later legs keep nothing idle

    # algorithmic bytes per launch ("Measurement")
    slots = st["n_windows"] * SKETCH
    pairs = st["n_pairs_inserted"]
    q_feats = float(st["q_features"])      # one classify launch per database
    q_locs = float(st["q_locations"])
    q_probes = float(st["q_probes"])
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
        "classify": {"name": cls_kernel, "avg_ms": avg_ms("classify"),
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
    cls_s = kernels["classify"]["avg_ms"] * 1e-3
    build_s = build_ms * 1e-3
    roofline = {
        "bound": "hbm", "kernel": dom["name"], "achieved": achieved,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": measured_traffic(dom["name"]),
        # the same work against the measured random-access and streaming ceilings
        "random_access": {
            "classify_lines_per_s": q_probes / cls_s,
            "classify_frac_of_line128_ceiling": q_probes / cls_s / CEIL_LINES128_GPS,
            "build_pairs_per_s": pairs / build_s,
            "build_frac_of_cas_ceiling": pairs / build_s / CEIL_CAS_GPS,
            "insert_pairs_per_s": pairs / (kernels["insert"]["avg_ms"] * 1e-3),
            "build_stream_gbs_at_2_7_bytes_per_bp": 2.7 * total_bp / build_s / 1e9,
            "build_frac_of_copy_ceiling": (2.7 * total_bp / build_s / 1e9) / CEIL_COPY_GBS,
            "ceilings": {"line128_per_s": CEIL_LINES128_GPS, "cas_per_s": CEIL_CAS_GPS,
                         "copy_gbs": CEIL_COPY_GBS,
                         "source": "profiles/memory_ceilings_mi355x.md"},
        },
    }

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
            "launch_shape": list(shape),
            "top_m": 4, "min_hits": 4, "hit_diff": 0,
        },
        "build_gbp_per_s": total_bp / 1e9 / build_s,
        "build_incl_h2d_gbp_per_s": total_bp / 1e9 / (h2d_build_ms * 1e-3),
        "phases_ms": {"build": build_ms, "classify": cls_ms, "build_incl_h2d": h2d_build_ms},
        "kernels": kernels,
        "db": {k: st[k] for k in ("n_windows", "n_pairs_inserted", "n_pairs_stored", "n_features",
                                  "n_buckets", "table_bytes", "load_factor", "probe_sum",
                                  "n_cap_candidates")},
        "query": {"features_per_read": q_feats / n, "locations_per_read": q_locs / n,
                  "probes_per_feature": q_probes / max(1, q_feats),
                  "large_pass_records": st["q_large_records"],
                  "hbm_pass_records": st["q_hbm_records"],
                  "classified_frac": float((gpu_labels != mc.MC_UNCLASSIFIED).mean())},
        "roofline": roofline,
        "condensed": condensed,
        "cpu_baseline": None,
    }
    if args.uneven_records > 0:
        out["uneven"] = uneven_leg(args, g, gtext, torch, mc, synth)
    del rtext, roff, labels
    if args.served_batches > 0:
        if g_served is not None:
            del gtext   # the served leg's reference set replaces the at-scale one on the device
            torch.cuda.empty_cache()
            gs = torch.from_numpy(g_served.text).to(dev)
            out["served"] = served_leg(args, g_served, gs, torch, mc, synth)
            del gs
        else:
            out["served"] = served_leg(args, g, gtext, torch, mc, synth)
            del gtext
    else:
        del gtext
    torch.cuda.empty_cache()
    if g_large is not None:
        out["large"] = large_leg(args, g_large, stream, torch, mc)
        torch.cuda.empty_cache()
    if args.cpu_sample > 0:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, reads, min(args.cpu_sample, n), threads,
                                           gpu_labels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
