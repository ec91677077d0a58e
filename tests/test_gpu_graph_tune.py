"""Captured query graphs and the launch-shape autotuner.

Every launch shape, the shape the autotuner keeps and every graph replay must
give the oracle's labels and top hits (with eager work and input changes
between replays), and a graph must be captured again after the database
changes.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2106_08150_amd as mc
from paper_2106_08150_amd import synth

pytestmark = pytest.mark.gpu


def oracle_results(g, recs, n_targets=None):
    """Oracle labels and top hits of the paired-layout records (as int32, the
    dtype of the device tensors) against the first n_targets genomes."""
    odb = orc.OracleDB()
    n = g.lengths.size if n_targets is None else n_targets
    odb.add_targets(g.text[:int(g.offsets[n])], g.lengths[:n], g.taxa[:n], threads=8)
    odb.set_taxonomy(g.parents)
    lab, top = odb.classify(recs.text, recs.offsets, paired=True, insert_size=400, threads=8)
    return lab.view(np.int32), top.view(np.int32)


def assert_oracle(want, lab, top=None):
    assert np.array_equal(lab.cpu().numpy(), want[0])
    if top is not None:
        assert np.array_equal(top.cpu().numpy(), want[1])


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = synth.tiny_genomes(length=60_000)
    db = mc.Database()
    db.add_targets(torch.from_numpy(g.text.copy()).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    recs = synth.mixed_records(g, 6000, seed=3)
    return torch, g, db, recs


@pytest.fixture(scope="module")
def want(setup):
    _, g, _, recs = setup
    return oracle_results(g, recs)


def dev(torch, recs):
    r = torch.from_numpy(recs.text.copy()).cuda()
    o = torch.from_numpy(recs.offsets.view(np.int64).copy()).cuda()
    return r, o


def test_all_launch_shapes_agree(setup, want):
    torch, g, db, recs = setup
    r, o = dev(torch, recs)
    ref = db.classify(r, o, recs.n_records, paired=True, insert_size=400, with_top=True)
    torch.cuda.synchronize()
    assert_oracle(want, *ref)
    for cap in (256, 512, 1024):
        for wpb in (2, 4, 8):
            for blocks in (1, 37, 16384):
                mc.mc_db_set_launch_config(db.h, cap, wpb, blocks)
                lab, top = db.classify(r, o, recs.n_records, paired=True, insert_size=400,
                                       with_top=True)
                torch.cuda.synchronize()
                assert torch.equal(lab, ref[0]) and torch.equal(top, ref[1]), (cap, wpb, blocks)
    with pytest.raises(mc.MCError):
        mc.mc_db_set_launch_config(db.h, 300, 4, 10)
    mc.mc_db_set_launch_config(db.h, 512, 4, 16384)


def test_autotune_keeps_results(setup, want):
    torch, g, db, recs = setup
    r, o = dev(torch, recs)
    ref, _ = db.classify(r, o, recs.n_records, paired=True, insert_size=400)
    torch.cuda.synchronize()
    out = torch.empty(recs.n_records, dtype=torch.int32, device="cuda")
    cfg, ms = mc.mc_db_autotune(db.h, r, o, recs.n_records, mc.QueryOpts(4, 4, 0, 400, 1), out)
    assert ms > 0 and cfg == mc.mc_db_get_launch_config(db.h)
    lab, top = db.classify(r, o, recs.n_records, paired=True, insert_size=400, with_top=True)
    torch.cuda.synchronize()
    assert torch.equal(lab, ref) and torch.equal(out, ref)
    assert_oracle(want, lab, top)     # the tuned shape against the oracle
    mc.mc_db_set_launch_config(db.h, 512, 4, 16384)


def test_graph_replays_match_eager(setup, want):
    torch, g, db, recs = setup
    other = synth.mixed_records(g, recs.n_records, seed=99)
    want2 = oracle_results(g, other)
    r, o = dev(torch, recs)
    r2, o2 = dev(torch, other)
    n = recs.n_records
    opts = mc.QueryOpts(4, 4, 0, 400, 1)
    eager1 = db.classify(r, o, n, paired=True, insert_size=400, with_top=True)
    eager2 = db.classify(r2, o2, n, paired=True, insert_size=400, with_top=True)
    # graph buffers: copies that we overwrite between replays
    gr = torch.empty(max(r.numel(), r2.numel()), dtype=torch.uint8, device="cuda")
    go = torch.empty_like(o)
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    top = torch.empty((n, 4, 3), dtype=torch.int32, device="cuda")
    gr[:r.numel()].copy_(r)
    go.copy_(o)
    graph = mc.ClassifyGraph(db.h, gr, go, n, opts, lab, top)
    for rep in range(4):
        src, so, expect = ((r, o, eager1) if rep % 2 == 0 else (r2, o2, eager2))
        gr[:src.numel()].copy_(src)
        go.copy_(so)
        lab.fill_(-7)
        top.fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(lab, expect[0]) and torch.equal(top, expect[1]), rep
        assert_oracle(want if rep % 2 == 0 else want2, lab, top)
        # eager work between replays
        db.classify(r2, o2, n, paired=True, insert_size=400)
        torch.cuda.synchronize()
    graph.close()


def test_graph_recaptured_after_addition(setup):
    torch, g, _, recs = setup
    off = g.offsets
    db = mc.Database()
    db.add_targets(g.text[:int(off[4])], g.lengths[:4], g.taxa[:4])
    db.set_taxonomy(g.parents)
    r, o = dev(torch, recs)
    n = recs.n_records
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    graph = mc.ClassifyGraph(db.h, r, o, n, mc.QueryOpts(4, 4, 0, 400, 1), lab)
    graph.launch()
    torch.cuda.synchronize()
    before = lab.clone()
    db.add_targets(g.text[int(off[4]):], g.lengths[4:], g.taxa[4:])
    graph.launch()
    torch.cuda.synchronize()
    now, _ = db.classify(r, o, n, paired=True, insert_size=400)
    torch.cuda.synchronize()
    assert torch.equal(lab, now) and not torch.equal(before, now)
    assert_oracle(oracle_results(g, recs, 4), before)
    assert_oracle(oracle_results(g, recs), lab)
    graph.close()


def test_size_class_routing(setup, want):
    """Records routed into size classes (at most 2 windows, at most 4, the
    rest), each classified by its own launch shape: the oracle's results, in
    eager launches, after per-class autotuning and in a captured graph."""
    torch, g, db, recs = setup
    r, o = dev(torch, recs)
    n = recs.n_records
    mc.mc_db_set_routing(db.h, [2, 4], [(256, 8, 16384), (512, 4, 64), (1024, 2, 16384)])
    assert mc.mc_db_get_routing(db.h) == ([2, 4], [(256, 8, 16384), (512, 4, 64),
                                                     (1024, 2, 16384)])
    lab, top = db.classify(r, o, n, paired=True, insert_size=400, with_top=True)
    torch.cuda.synchronize()
    assert_oracle(want, lab, top)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    mc.mc_db_autotune(db.h, r, o, n, mc.QueryOpts(4, 4, 0, 400, 1), out)
    bounds, shapes = mc.mc_db_get_routing(db.h)
    assert bounds == [2, 4] and len(shapes) == 3
    assert_oracle(want, out)
    lab2 = torch.empty(n, dtype=torch.int32, device="cuda")
    graph = mc.ClassifyGraph(db.h, r, o, n, mc.QueryOpts(4, 4, 0, 400, 1), lab2)
    for _ in range(3):
        lab2.fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        assert_oracle(want, lab2)
    graph.close()
    with pytest.raises(mc.MCError):
        mc.mc_db_set_routing(db.h, [4, 2], [(256, 4, 64)] * 3)
    mc.mc_db_set_routing(db.h, [], [(512, 4, 16384)])
    mc.mc_db_set_launch_config(db.h, 512, 4, 16384)
