"""HIP path vs the CPU oracle, element by element, through the C ABI.

Integer work throughout, so the bar is bit-exact: per-window sketches, the
stored (feature, location) pairs, per-record top hits and labels.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2106_08150_amd as mc
from paper_2106_08150_amd import synth

pytestmark = pytest.mark.gpu

UNCL = 0xFFFFFFFF
SENTINEL_KMER = "ATATACTCGGAAGAAT"   # canonical 16-mer whose h1 is 0xFFFFFFFF


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def dev_u8(torch, arr):
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    return torch.from_numpy(a.copy()).cuda() if a.size else torch.zeros(1, dtype=torch.uint8,
                                                                           device="cuda")


def dev_off(torch, off):
    return torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).cuda()


def build_both(torch, g, k=16, w=128, s=16, cap=254, splits=None, path=None):
    gdb = mc.Database(k, w, s, cap)
    if path:
        mc.mc_db_set_insert_path(gdb.h, **path)
    odb = orc.OracleDB(k, w, s, cap)
    off = g.offsets
    for a, b in (splits or [(0, g.lengths.size)]):
        txt = g.text[int(off[a]):int(off[b])]
        gdb.add_targets(dev_u8(torch, txt), g.lengths[a:b], g.taxa[a:b])
        odb.add_targets(txt, g.lengths[a:b], g.taxa[a:b], threads=8)
    gdb.set_taxonomy(g.parents)
    odb.set_taxonomy(g.parents)
    return gdb, odb


def assert_same_table(gdb, odb):
    gf, gl = gdb.dump()
    of, ol = odb.dump()
    assert gf.size == of.size
    assert np.array_equal(gf, of)
    assert np.array_equal(gl, ol)


def classify_both(torch, gdb, odb, reads, paired=False, **opts):
    r = dev_u8(torch, reads.text)
    o = dev_off(torch, reads.offsets)
    n = reads.n_records
    labels, top = gdb.classify(r, o, n, paired=paired, with_top=True, **opts)
    torch.cuda.synchronize()
    gl = labels.cpu().numpy().view(np.uint32)
    gt = top.cpu().numpy().view(np.uint32)
    ol, ot = odb.classify(reads.text, reads.offsets, paired=paired, threads=8, **opts)
    return gl, gt, ol, ot


def assert_same_results(gl, gt, ol, ot):
    bad = np.nonzero((gl != ol) | (gt != ot).any(axis=(1, 2)))[0]
    assert bad.size == 0, (f"{bad.size} records differ, first {bad[:5]}: "
                           f"gpu {gl[bad[:3]]} {gt[bad[:3]]} oracle {ol[bad[:3]]} {ot[bad[:3]]}")


# ------------------------------------------------------------ sketches ----
@pytest.mark.parametrize("k,w,s", [(16, 128, 16), (16, 127, 16), (4, 20, 3), (5, 5, 1),
                                   (16, 40, 25), (12, 75, 64), (16, 271, 16), (1, 64, 2)])
def test_window_sketches(torch, k, w, s):
    rng = np.random.default_rng(k * 1000 + w)
    seqs = []
    for L in [0, 1, k - 1, k, k + 1, w, w + 1, 3 * w - 7, 5000]:
        t = rng.choice(np.frombuffer(b"ACGTacgtN", np.uint8), size=L,
                       p=[0.24, 0.24, 0.24, 0.24, 0.01, 0.01, 0.01, 0.005, 0.005])
        seqs.append(t.astype(np.uint8))
    seqs.append(np.frombuffer(b"A" * 700, np.uint8))
    seqs.append(np.frombuffer(("NN" + SENTINEL_KMER + "NN").encode(), np.uint8))
    lengths = np.array([x.size for x in seqs], np.uint64)
    text = np.concatenate(seqs)
    db = mc.Database(k, w, s, 254)
    nw = [orc.num_windows(int(L), k, w) for L in lengths]
    tot = max(1, sum(nw))
    counts = torch.zeros(tot, dtype=torch.int32, device="cuda")
    feats = torch.zeros(tot * s, dtype=torch.int32, device="cuda")
    mc.mc_db_sketch(db.h, dev_u8(torch, text), lengths, counts, feats)
    torch.cuda.synchronize()
    counts = counts.cpu().numpy().view(np.uint32)
    feats = feats.cpu().numpy().view(np.uint32)
    gw = 0
    for x, n_w in zip(seqs, nw):
        want = orc.sketch_windows(x, k, w, s)
        assert len(want) == n_w
        for j in range(n_w):
            got = feats[(gw + j) * s:(gw + j) * s + counts[gw + j]].tolist()
            assert got == want[j], (k, w, s, x.size, j)
        gw += n_w


# ---------------------------------------------------------- tiny config ----
@pytest.fixture(scope="module")
def tiny(torch):
    g = synth.tiny_genomes()
    gdb, odb = build_both(torch, g)
    reads = synth.tiny_reads(g)
    return g, gdb, odb, reads


def test_tiny_table(tiny):
    _, gdb, odb, _ = tiny
    assert_same_table(gdb, odb)
    st = gdb.stats()
    assert st["n_pairs_stored"] == odb.num_pairs
    assert st["n_windows"] == 8 * 885


def test_tiny_classification(torch, tiny):
    _, gdb, odb, reads = tiny
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads)
    assert_same_results(gl, gt, ol, ot)
    # sanity: most reads are labelled with a species or genus
    assert (gl != UNCL).mean() > 0.5


@pytest.mark.parametrize("top_m,min_hits,hit_diff",
                         [(1, 1, 0), (2, 1, 1), (4, 1, 3), (4, 4, 0), (2, 4, 3), (1, 4, 1),
                          (8, 2, 2)])
def test_parameter_grid(torch, tiny, top_m, min_hits, hit_diff):
    g, gdb, odb, _ = tiny
    reads = synth.sample_reads(g, 1500, 100, seed=top_m * 100 + min_hits * 10 + hit_diff)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, top_m=top_m, min_hits=min_hits,
                                   hit_diff=hit_diff)
    assert_same_results(gl, gt, ol, ot)


def test_batch_split_and_stream_determinism(torch, tiny):
    _, gdb, _, reads = tiny
    r = dev_u8(torch, reads.text)
    o = dev_off(torch, reads.offsets)
    full, _ = gdb.classify(r, o, reads.n_records)
    parts = []
    s = torch.cuda.Stream()
    for a, b in [(0, 1), (1, 4000), (4000, 10000)]:
        with torch.cuda.stream(s):
            lab, _ = gdb.classify(r, o[a:b + 1].contiguous(), b - a, stream=s)
        parts.append(lab)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(full, torch.cat(parts))


# -------------------------------------------------------- cap handling ----
def test_cap_stress_repeated_genomes(torch):
    g = synth.repeated_genome(300, 20_000, seed=21)
    gdb, odb = build_both(torch, g)
    assert_same_table(gdb, odb)
    f, _ = gdb.dump()
    _, counts = np.unique(f, return_counts=True)
    assert counts.max() == 254
    # reads from the repeats: 16 features x 254 locations -> large-list pass
    reads = synth.sample_reads(g, 300, 100, seed=5, error=0.0)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, top_m=8, min_hits=1)
    assert_same_results(gl, gt, ol, ot)
    assert mc.mc_db_query_status(gdb.h) == 0


def test_sentinel_feature_over_cap(torch):
    """Feature 0xFFFFFFFF stored more often than the cap: its capped-away
    entries must not read as empty slots, or the chains of other features
    that run through those buckets would end early."""
    rng = np.random.default_rng(23)
    base = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, 20_000)]
    island = np.frombuffer(b"N" * 120 + SENTINEL_KMER.encode() + b"N" * 120, np.uint8)
    one = np.concatenate([base[:9_000], island, base[9_000:]])
    n = 300
    g = synth.Genomes(np.tile(one, n), np.full(n, one.size, np.uint64),
                      np.arange(1, n + 1, dtype=np.uint32), np.zeros(n + 1, np.uint32))
    gdb, odb = build_both(torch, g)
    assert_same_table(gdb, odb)
    f, _ = gdb.dump(0xFFFFFFFF, 0xFFFFFFFF)
    assert f.size == 254
    reads = synth.sample_reads(g, 300, 100, seed=9, error=0.0)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, top_m=8, min_hits=1)
    assert_same_results(gl, gt, ol, ot)


@pytest.mark.parametrize("cap", [1, 3, 17])
def test_small_caps_and_incremental_adds(torch, cap):
    g = synth.tiny_genomes(length=30_000)
    gdb, odb = build_both(torch, g, cap=cap, splits=[(0, 3), (3, 4), (4, 8)])
    assert_same_table(gdb, odb)
    reads = synth.sample_reads(g, 2000, 100, seed=cap)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, min_hits=1)
    assert_same_results(gl, gt, ol, ot)


def test_table_growth_keeps_entries(torch):
    """Many small adds force several rehashes of the table."""
    g = synth.clustered_genomes(4, 5, 2e6, seed=31, median_bp=1e5, clip=(2e4, 3e5))
    gdb, odb = build_both(torch, g, splits=[(i, i + 1) for i in range(20)])
    assert gdb.stats()["n_rehash"] >= 1
    assert_same_table(gdb, odb)


# ------------------------------------------------------------ edge cases --
def test_edge_case_reads(torch, tiny):
    g, gdb, odb, _ = tiny
    g0 = g.genome(0)
    S = 113
    pieces = [
        b"", b"ACGT", g0[500:515].tobytes(), g0[500:516].tobytes(), g0[500:628].tobytes(),
        g0[5 * S:5 * S + 128].tobytes(), g0[1000:1129].tobytes(),
        g0[2000:2100].tobytes().lower(), (g0[3000:3050].tobytes() + b"N" + g0[3051:3100].tobytes()),
        b"N" * 100, g0[4000:4250].tobytes(), g0[7000:8000].tobytes(),
        synth.reverse_complement_text(g0[9000:9150]).tobytes(),
    ]
    off = np.zeros(len(pieces) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in pieces])
    reads = synth.Reads(np.frombuffer(b"".join(pieces), np.uint8), off)
    for opts in [dict(min_hits=1), dict(), dict(top_m=1, hit_diff=2)]:
        gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, **opts)
        assert_same_results(gl, gt, ol, ot)
    assert gl[0] == UNCL and gl[1] == UNCL and gl[9] == UNCL


def test_paired_records(torch, tiny):
    g, gdb, odb, _ = tiny
    recs = synth.mixed_records(g, 600, seed=9)
    # add a few records with an empty mate 1 or both mates empty
    extra = [(b"", g.genome(2)[100:250].tobytes()), (b"", b""), (g.genome(3)[0:20].tobytes(), b"")]
    text = recs.text.tobytes()
    off = list(recs.offsets.tolist())
    for m1, m2 in extra:
        text += m1
        off.append(len(text))
        text += m2
        off.append(len(text))
    reads = synth.Reads(np.frombuffer(text, np.uint8), np.array(off, np.uint64), paired=True)
    for ins in [0, 400, 1000]:
        gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, paired=True, insert_size=ins,
                                       min_hits=2)
        assert_same_results(gl, gt, ol, ot)


def test_homopolymer_and_sentinel_feature(torch):
    seqs = [b"A" * 5000, ("N" * 40 + SENTINEL_KMER + "N" * 40).encode(), SENTINEL_KMER.encode(),
            b"ACGT" * 700]
    lengths = np.array([len(x) for x in seqs], np.uint64)
    text = np.frombuffer(b"".join(seqs), np.uint8)
    g = synth.Genomes(text, lengths, np.array([1, 2, 2, 1], np.uint32),
                      np.array([0, 0, 0], np.uint32))
    gdb, odb = build_both(torch, g)
    assert_same_table(gdb, odb)
    f, _ = gdb.dump(0xFFFFFFFF, 0xFFFFFFFF)
    assert f.size == 2            # the all-ones feature is stored, twice
    rd = [SENTINEL_KMER.encode(), b"A" * 100, b"ACGT" * 30, b"T" * 60]
    off = np.zeros(len(rd) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in rd])
    reads = synth.Reads(np.frombuffer(b"".join(rd), np.uint8), off)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, min_hits=1, top_m=4)
    assert_same_results(gl, gt, ol, ot)
    assert gl[0] == 2


def test_long_records_match_oracle(torch):
    """Records whose candidate lists exceed the LDS passes (16,384 locations)
    take the HBM-list pass and still equal the oracle: on 300 identical
    genomes every feature holds 254 locations, so 2 x 600 bp mates gather
    12 windows x 16 x 254 = 48,768 locations, 2 x 1,000 bp mates 73,152 and a
    5,000 bp read 44 windows' worth; short records around them take the
    fast and large-list passes in the same launch."""
    g = synth.repeated_genome(300, 20_000, seed=21)
    gdb, odb = build_both(torch, g)
    g0 = g.genome(0)
    pieces = [g0[0:100], g0[:0], g0[1000:1600], g0[5000:5600],        # short; 2 x 600
              g0[100:250], g0[300:450],                                # 2 x 150
              g0[2000:3000], synth.reverse_complement_text(g0[4000:5000]),   # 2 x 1,000
              g0[7000:12000], g0[:0],                                  # 5,000 bp single
              g0[15000:18000], g0[:0],                                 # 3,000 bp single
              g0[300:400], g0[:0]]                                     # short
    off = np.zeros(len(pieces) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in pieces])
    reads = synth.Reads(np.concatenate(pieces), off, paired=True)
    for opts in (dict(min_hits=1), dict(min_hits=1, insert_size=2500, top_m=8),
                 dict(hit_diff=40, top_m=3)):
        print(f"long records, options {opts}", flush=True)
        gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, paired=True, **opts)
        assert_same_results(gl, gt, ol, ot)
        assert mc.mc_db_query_status(gdb.h) == 0
    assert (gl[1:5] != UNCL).all()


def test_record_beyond_hbm_list_capacity_is_reported(torch):
    """A record with more than 2^20 candidate locations (a 40 kbp read on 300
    identical genomes: about 1.4M) is reported and left unclassified; the
    records around it still match the oracle."""
    g = synth.repeated_genome(300, 20_000, seed=21)
    gdb, odb = build_both(torch, g)
    g0 = g.genome(0)
    pieces = [g0[0:100], np.concatenate([g0, g0]), g0[500:650]]
    off = np.zeros(len(pieces) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in pieces])
    reads = synth.Reads(np.concatenate(pieces), off)
    r = dev_u8(torch, reads.text)
    o = dev_off(torch, reads.offsets)
    labels, top = gdb.classify(r, o, 3, min_hits=1, with_top=True)
    torch.cuda.synchronize()
    gl = labels.cpu().numpy().view(np.uint32)
    gt = top.cpu().numpy().view(np.uint32)
    assert mc.mc_db_query_status(gdb.h) == 1
    assert gl[1] == UNCL and (gt[1, :, 0] == UNCL).all() and (gt[1, :, 1] == 0).all()
    keep = np.array([0, 2])
    sub = synth.Reads(np.concatenate([pieces[0], pieces[2]]),
                      np.array([0, 100, 250], np.uint64))
    ol, ot = odb.classify(sub.text, sub.offsets, min_hits=1)
    assert_same_results(gl[keep], gt[keep], ol, ot)


# ------------------------------------------------- several tiles, ragged --
def test_clustered_midsize(torch):
    g = synth.clustered_genomes(5, 6, 3e6, seed=41, median_bp=1e5, clip=(3e3, 4e5))
    gdb, odb = build_both(torch, g)
    assert_same_table(gdb, odb)
    reads = synth.sample_reads(g, 5000, 150, seed=42, foreign=0.05)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads)
    assert_same_results(gl, gt, ol, ot)
    recs = synth.mixed_records(g, 1000, seed=43)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, recs, paired=True, insert_size=400)
    assert_same_results(gl, gt, ol, ot)


INSERT_MODES = {
    "slices": {},
    "staged": {"stage_entries": 512},
    "direct": {"direct": 1},
    "global": {"global_insert": 1, "part_mb": 1},
    "fine1024": {"slice_shift": 5, "fine_bits": 10},
    "chunks": {"chunk_slots": 20000},
}


@pytest.mark.parametrize("mode", list(INSERT_MODES))
def test_insert_modes_agree(torch, mode):
    """Every insert path stores the oracle's pairs, over two add calls (the
    second fills buckets the first left partly full): the slice-local insert
    (default), the same with a 512-pair staging buffer (many rounds a slice),
    its direct path (LDS fill counters, one store a pair), the
    global-counter insert used for tables too large for LDS slices (1 MiB
    partitions), slices of 32 buckets with 1024 slices per partition (the
    largest level-2 scatter, as the largest tables use), and an add built in
    chunks of about 20,000 pair slots (every chunk after the first inserts
    into a table that already holds entries)."""
    g = synth.clustered_genomes(4, 5, 2e6, seed=47, median_bp=1e5, clip=(3e3, 3e5))
    db, odb = build_both(torch, g, splits=[(0, 7), (7, 20)], path=INSERT_MODES[mode])
    assert_same_table(db, odb)
    reads = synth.sample_reads(g, 3000, 150, seed=48)
    gl, gt, ol, ot = classify_both(torch, db, odb, reads)
    assert_same_results(gl, gt, ol, ot)


@pytest.mark.parametrize("mode", ["slices", "direct"])
def test_sparse_fresh_table(torch, mode):
    """A first insert into a table far larger than its pairs (load factor
    1e-4, so most slices hold no pair): the insert that clears the new table
    as it writes must leave every other slot empty and every other counter
    zero; a second add then grows the table by a rehash."""
    g = synth.tiny_genomes(length=30_000)
    gdb = mc.Database(16, 128, 16, 254)
    if INSERT_MODES[mode]:
        mc.mc_db_set_insert_path(gdb.h, **INSERT_MODES[mode])
    gdb.reserve(0, 1e-4)
    odb = orc.OracleDB(16, 128, 16, 254)
    off = g.offsets
    for a, b in [(0, 5), (5, g.lengths.size)]:
        txt = g.text[int(off[a]):int(off[b])]
        gdb.add_targets(dev_u8(torch, txt), g.lengths[a:b], g.taxa[a:b])
        odb.add_targets(txt, g.lengths[a:b], g.taxa[a:b], threads=8)
        of, _ = odb.dump()
        assert gdb.stats()["n_pairs_stored"] == of.size
    assert gdb.stats()["n_buckets"] > 1 << 20
    gdb.set_taxonomy(g.parents)
    odb.set_taxonomy(g.parents)
    assert_same_table(gdb, odb)
    reads = synth.sample_reads(g, 1000, 100, seed=5)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads, min_hits=1)
    assert_same_results(gl, gt, ol, ot)


def test_failed_add_is_rolled_back(torch):
    """An add that fails after its inserts ran (forced from the host) leaves
    no entry of its targets: the table equals the one before the call (its
    slots turned into tombstones), the target count is unchanged, and the same
    genomes added again afterwards give the oracle's table and results."""
    g = synth.clustered_genomes(3, 4, 1.2e6, seed=51, median_bp=1e5, clip=(3e3, 3e5))
    off = g.offsets
    gdb = mc.Database()
    gdb.add_targets(dev_u8(torch, g.text[:int(off[5])]), g.lengths[:5], g.taxa[:5])
    f0, l0 = gdb.dump()
    st0 = gdb.stats()
    mc.mc_db_set_insert_path(gdb.h, fail_after=1)
    with pytest.raises(mc.MCError) as e:
        gdb.add_targets(dev_u8(torch, g.text[int(off[5]):]), g.lengths[5:], g.taxa[5:])
    assert e.value.code == mc.MC_ERR_TABLE_FULL
    f1, l1 = gdb.dump()
    assert np.array_equal(f0, f1) and np.array_equal(l0, l1)
    st1 = gdb.stats()
    assert st1["n_targets"] == 5 and st1["n_pairs_stored"] == st0["n_pairs_stored"]
    assert st1["n_tombstones"] > 0 and st1["n_features"] == st0["n_features"]
    gdb.add_targets(dev_u8(torch, g.text[int(off[5]):]), g.lengths[5:], g.taxa[5:])
    gdb.set_taxonomy(g.parents)
    odb = orc.OracleDB()
    odb.add_targets(g.text, g.lengths, g.taxa, threads=8)
    odb.set_taxonomy(g.parents)
    assert_same_table(gdb, odb)
    st2 = gdb.stats()
    assert st2["n_features"] == odb.num_features and st2["n_pairs_stored"] == odb.num_pairs
    assert 0 < st2["load_factor"] < 1
    reads = synth.sample_reads(g, 2000, 150, seed=52, foreign=0.05)
    gl, gt, ol, ot = classify_both(torch, gdb, odb, reads)
    assert_same_results(gl, gt, ol, ot)


def test_addition_waits_for_classification_in_flight(torch):
    """A classification queued on a side stream is not disturbed by an
    addition issued right after it without any host synchronisation: it sees
    the table as it was, and the next one sees the new targets."""
    g = synth.tiny_genomes(length=60_000)
    off = g.offsets
    gdb = mc.Database()
    gdb.add_targets(dev_u8(torch, g.text[:int(off[4])]), g.lengths[:4], g.taxa[:4])
    gdb.set_taxonomy(g.parents)
    reads = synth.sample_reads(g, 200_000, 100, seed=53)
    r = dev_u8(torch, reads.text)
    o = dev_off(torch, reads.offsets)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        lab, top = gdb.classify(r, o, reads.n_records, with_top=True, stream=side)
    gdb.add_targets(dev_u8(torch, g.text[int(off[4]):]), g.lengths[4:], g.taxa[4:])
    side.synchronize()
    gl = lab.cpu().numpy().view(np.uint32)
    gt = top.cpu().numpy().view(np.uint32)
    before = orc.OracleDB()
    before.add_targets(g.text[:int(off[4])], g.lengths[:4], g.taxa[:4], threads=8)
    before.set_taxonomy(g.parents)
    ol, ot = before.classify(reads.text, reads.offsets, first=0, count=20_000, threads=8)
    assert_same_results(gl[:20_000], gt[:20_000], ol, ot)
    after = orc.OracleDB()
    after.add_targets(g.text, g.lengths, g.taxa, threads=8)
    after.set_taxonomy(g.parents)
    small = synth.sample_reads(g, 3000, 100, seed=54)
    gl, gt, ol, ot = classify_both(torch, gdb, after, small)
    assert_same_results(gl, gt, ol, ot)


def test_invalid_taxonomy_and_state(torch):
    db = mc.Database()
    with pytest.raises(mc.MCError):
        db.set_taxonomy(np.array([1, 0], np.uint32))          # no root (cycle)
    with pytest.raises(mc.MCError):
        db.set_taxonomy(np.array([0, 1], np.uint32))          # two roots
    with pytest.raises(mc.MCError):
        db.set_taxonomy(np.array([0, 5], np.uint32))          # out of range
    with pytest.raises(mc.MCError):
        db.set_taxonomy(np.array([0, 2, 1], np.uint32))       # cycle off the root
    g = synth.tiny_genomes(length=2000)
    db.add_targets(dev_u8(torch, g.text), g.lengths, g.taxa)
    r = dev_u8(torch, g.text[:100])
    o = dev_off(torch, np.array([0, 100], np.uint64))
    with pytest.raises(mc.MCError):       # taxonomy not set
        db.classify(r, o, 1)
    db.set_taxonomy(np.array([0, 0, 0], np.uint32))   # taxa 3..10 outside
    with pytest.raises(mc.MCError):
        db.classify(r, o, 1)
    # a sequence with 2^18 + 1 windows: rejected before any byte is read
    lengths = np.array([(1 << 18) * 113 + 16], np.uint64)
    taxa = np.zeros(1, np.uint32)
    buf = dev_u8(torch, np.zeros(16, np.uint8))
    rc = mc.lib().mc_db_add_targets_device(db.h, buf.data_ptr(), mc._np_ptr(lengths),
                                           mc._np_ptr(taxa), 1, None)
    assert rc == mc.MC_ERR_CAPACITY
