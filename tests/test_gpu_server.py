"""Served form: results identical alone and in the mix; ordered additions.

Batches of uneven size and layout are submitted to a server with several
in-flight slots so that their copies and kernels overlap; every batch's labels
and top hits must equal those of the same batch classified alone (tolerance
0), and the oracle's. A genome addition queued between batches must be seen by
every later batch and by no earlier one.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2106_08150_amd as mc
from paper_2106_08150_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def plain(torch, db, reads, paired, **opts):
    r = torch.from_numpy(np.ascontiguousarray(reads.text)).cuda()
    o = torch.from_numpy(reads.offsets.view(np.int64).copy()).cuda()
    lab, top = db.classify(r, o, reads.n_records, paired=paired, with_top=True, **opts)
    torch.cuda.synchronize()
    return lab.cpu().numpy().view(np.uint32), top.cpu().numpy().view(np.uint32)


def sub_batch(reads, a, b):
    off = reads.offsets[a:b + 1]
    return synth.Reads(reads.text[int(off[0]):int(off[-1])].copy(), off - off[0], False)


def test_results_identical_alone_and_in_the_mix(torch):
    g = synth.tiny_genomes()
    db = mc.Database()
    db.add_targets(torch.from_numpy(g.text.copy()).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    reads = synth.tiny_reads(g, n=40_000, seed=77)
    cuts = [0, 1, 101, 5101, 25101, 25401, 25418, 33418, 40000]
    batches = [(sub_batch(reads, a, b), False) for a, b in zip(cuts[:-1], cuts[1:])]
    batches.append((synth.mixed_records(g, 3000, seed=5), True))
    alone = [plain(torch, db, r, p, insert_size=400 if p else 0) for r, p in batches]

    srv = mc.Server(db, slots=3)
    tickets = [srv.submit(r.text, r.offsets, paired=p, with_top=True,
                          insert_size=400 if p else 0) for r, p in batches]
    for i, ((lab0, top0), t) in enumerate(zip(alone, tickets)):
        if i % 2:
            lab, top, ms = srv.wait(t)
        else:   # the stage split of a batch's latency adds up to it
            lab, top, tm = srv.wait_times(t)
            ms = tm["total_ms"]
            stages = tm["admit_ms"] + tm["copy_ms"] + tm["launch_ms"] + tm["finish_ms"]
            assert abs(stages - ms) < 1e-3 and min(tm.values()) >= 0
        assert ms >= 0
        assert np.array_equal(lab, lab0) and np.array_equal(top, top0)
    st = srv.stats()
    assert st["batches"] == len(batches)
    assert st["records"] == sum(r.n_records for r, _ in batches)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    srv.close()

    # the oracle agrees on a mixed sample
    odb = orc.OracleDB()
    odb.add_targets(g.text, g.lengths, g.taxa)
    odb.set_taxonomy(g.parents)
    r, _ = batches[3]
    ol, ot = odb.classify(r.text, r.offsets, first=0, count=2000)
    assert np.array_equal(alone[3][0][:2000], ol) and np.array_equal(alone[3][1][:2000], ot)


def test_additions_are_ordered_with_batches(torch):
    g = synth.tiny_genomes(length=40_000)
    # first 5 genomes at start, genomes 5..7 added while serving
    off = g.offsets
    first = synth.Genomes(g.text[:int(off[5])].copy(), g.lengths[:5], g.taxa[:5], g.parents)
    db = mc.Database()
    db.add_targets(first.text, first.lengths, first.taxa)
    db.set_taxonomy(first.parents)
    reads = synth.sample_reads(g, 6000, 100, seed=3)

    before = mc.Database()
    before.add_targets(first.text, first.lengths, first.taxa)
    before.set_taxonomy(g.parents)
    after = mc.Database()
    after.add_targets(g.text, g.lengths, g.taxa)
    after.set_taxonomy(g.parents)
    want_before = plain(torch, before, reads, False)
    want_after = plain(torch, after, reads, False)
    assert not np.array_equal(want_before[0], want_after[0])

    srv = mc.Server(db, slots=4)
    t1 = srv.submit(reads.text, reads.offsets, with_top=True)
    t2 = srv.submit(reads.text, reads.offsets, with_top=True)
    ta = srv.add_targets(g.text[int(off[5]):], g.lengths[5:], g.taxa[5:], parents=g.parents)
    t3 = srv.submit(reads.text, reads.offsets, with_top=True)
    for t in (t1, t2):
        lab, top, _ = srv.wait(t)
        assert np.array_equal(lab, want_before[0]) and np.array_equal(top, want_before[1])
    assert srv.wait(ta)[0] is None
    lab, top, _ = srv.wait(t3)
    assert np.array_equal(lab, want_after[0]) and np.array_equal(top, want_after[1])
    assert srv.stats()["additions"] == 1
    srv.close()


def test_budget_rejects_oversized_batch(torch):
    g = synth.tiny_genomes(length=5000)
    db = mc.Database()
    db.add_targets(g.text, g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    srv = mc.Server(db, slots=1, memory_budget=4096)
    reads = synth.sample_reads(g, 1000, 100, seed=1)
    with pytest.raises(mc.MCError):
        srv.submit(reads.text, reads.offsets)
    small = sub_batch(reads, 0, 5)
    lab, _, _ = srv.wait(srv.submit(small.text, small.offsets))
    assert lab.size == 5
    srv.close()


def test_ticket_waited_twice_is_rejected(torch):
    g = synth.tiny_genomes(length=5000)
    db = mc.Database()
    db.add_targets(g.text, g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    srv = mc.Server(db, slots=2)
    reads = synth.sample_reads(g, 50, 100, seed=2)
    t = srv.submit(reads.text, reads.offsets)
    lab, _, _ = srv.wait(t)
    assert lab.size == 50
    with pytest.raises(mc.MCError) as e:
        srv.wait(t)
    assert e.value.code == mc.MC_ERR_INVALID_ARG
    srv.close()


def test_budget_shared_by_slots(torch):
    """Batches that each fit the budget but not all at once: slots take turns
    (free slots give their buffers back), every batch completes with the
    labels it gets alone."""
    g = synth.tiny_genomes(length=20_000)
    db = mc.Database()
    db.add_targets(g.text, g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    reads = synth.sample_reads(g, 400_000, 100, seed=8)
    cuts = [0, 150_000, 151_000, 300_000, 301_000, 400_000]
    batches = [sub_batch(reads, a, b) for a, b in zip(cuts[:-1], cuts[1:])]
    alone = [plain(torch, db, r, False) for r in batches]
    # a 150k-read batch needs about 17 MB of device buffers; 40 MiB for four
    # slots lets at most two large ones in flight
    srv = mc.Server(db, slots=4, memory_budget=40 << 20, staging_bytes=1 << 20)
    tickets = [srv.submit(r.text, r.offsets, with_top=True) for r in batches]
    for (lab0, top0), t in zip(alone, tickets):
        lab, top, _ = srv.wait(t)
        assert np.array_equal(lab, lab0) and np.array_equal(top, top0)
    srv.close()


def test_long_records_through_the_server(torch):
    """Records whose candidate lists outgrow the fast pass, in a batch of two
    chunks (more than 131,072 records) and in small batches: the server runs
    the large-list and HBM-list passes only for the chunks whose fast pass
    queued records, and every label and top-hit list equals the plain
    launch's; the long records also equal the oracle's. The reference set is
    the tiny set plus 300 identical copies of another genome, whose features
    each hold 254 locations: a 100 bp read of those copies gathers 4,064
    locations (large-list pass), a 600 bp read 24,384 (HBM-list pass)."""
    tiny = synth.tiny_genomes(length=20_000)
    rep = synth.repeated_genome(300, 20_000, seed=21)
    g = synth.Genomes(np.concatenate([tiny.text, rep.text]),
                      np.concatenate([tiny.lengths, rep.lengths]),
                      np.concatenate([tiny.taxa, np.full(rep.lengths.size, 10, np.uint32)]),
                      tiny.parents)
    db = mc.Database()
    db.add_targets(torch.from_numpy(g.text.copy()).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    short = synth.sample_reads(tiny, 140_000, 100, seed=31)
    r0 = rep.genome(0)
    long_at = {7: r0[0:100], 70_001: r0[1000:1600], 131_080: r0[2000:2100],
               139_990: synth.reverse_complement_text(r0[5000:5600])}
    pieces = [long_at.get(i, short.text[int(short.offsets[i]):int(short.offsets[i + 1])])
              for i in range(short.n_records)]
    off = np.zeros(len(pieces) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in pieces])
    big = synth.Reads(np.concatenate(pieces), off, False)
    batches = [big, sub_batch(big, 0, 10), sub_batch(big, 70_000, 70_003),
               sub_batch(big, 131_070, 131_100)]
    alone = [plain(torch, db, r, False, min_hits=1) for r in batches]
    srv = mc.Server(db, slots=3)
    tickets = [srv.submit(r.text, r.offsets, with_top=True, min_hits=1) for r in batches]
    for (lab0, top0), t in zip(alone, tickets):
        lab, top, _ = srv.wait(t)
        assert np.array_equal(lab, lab0) and np.array_equal(top, top0)
    srv.close()
    odb = orc.OracleDB()
    odb.add_targets(g.text, g.lengths, g.taxa)
    odb.set_taxonomy(g.parents)
    lab0, top0 = alone[0]
    for i in sorted(long_at):
        ol, ot = odb.classify(big.text, big.offsets, first=i, count=1, min_hits=1)
        assert ol[0] == lab0[i] and np.array_equal(ot[0], top0[i]), i
        assert lab0[i] != 0xFFFFFFFF
