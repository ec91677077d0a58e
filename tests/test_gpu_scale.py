"""Parity at the benchmark's full size, in the benchmark's launch configurations.

The at-scale reference set (1,000 genomes, about 4 Gbp) is built on the GPU
from HBM-resident text and all 10M reads are classified in one launch, once
with the shape the benchmark times ({256 locations, 4 waves, 16,384
workgroups}) and once with the library's default ({512, 4, 16,384}). The
oracle cannot hold that index, so it checks what it can compute exactly:

* a read sample of 3,000 reads spread over the set: the oracle indexes only
  the features those reads look up (exact for them) and classifies them;
* a slice of the table: every stored pair whose feature is below 2^20, taken
  by the same oracle scan (all locations of those features, cap applied).

Plus properties that hold at any size: stored pairs = inserted pairs (no
feature reaches the cap here), window count closed form, label domain.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2106_08150_amd as mc
from paper_2106_08150_amd import synth

pytestmark = pytest.mark.gpu

UNCL = 0xFFFFFFFF
SLICE_HI = (1 << 20) - 1
SHAPES = [(256, 4, 16384), (512, 4, 16384)]   # the benchmark's, the library default


@pytest.mark.timeout(600)
def test_at_scale_sampled_parity():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = synth.scale_genomes()
    reads = synth.scale_reads(g)
    n = reads.n_records
    print(f"\n[scale] {g.lengths.size} genomes, {int(g.lengths.sum())} bp, {n} reads", flush=True)

    db = mc.Database()
    db.add_targets(torch.from_numpy(g.text).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    r = torch.from_numpy(reads.text).cuda()
    o = torch.from_numpy(reads.offsets.view(np.int64)).cuda()
    results = {}
    for shape in SHAPES:
        print(f"[scale] classify with launch shape {shape}", flush=True)
        mc.mc_db_set_launch_config(db.h, *shape)
        labels, top = db.classify(r, o, n, with_top=True)
        torch.cuda.synchronize()
        results[shape] = (labels.cpu().numpy().view(np.uint32), top.cpu().numpy().view(np.uint32))
        del labels, top
    st = db.stats()
    gf, gloc = db.dump(0, SLICE_HI)
    print(f"[scale] gpu done: {st['n_pairs_stored']} pairs, slice {gf.size}", flush=True)

    # properties at full size
    S = 128 - 16 + 1
    assert st["n_windows"] == int(sum(-(-(int(L) - 15) // S) for L in g.lengths))
    assert st["n_pairs_stored"] == st["n_pairs_inserted"]
    assert st["n_features"] <= st["n_pairs_stored"] and st["n_tombstones"] == 0
    for gl, _ in results.values():
        valid = (gl == UNCL) | (gl < g.parents.size)
        assert valid.all()
    assert mc.mc_db_query_status(db.h) == 0

    # oracle on a sample and a feature slice
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(n, 3000, replace=False))
    feats = [orc.query_features(reads.text, reads.offsets, 16, 128, 16, int(i), 1, False)
             for i in sample]
    odb = orc.OracleDB()
    odb.set_filter(np.unique(np.concatenate(feats)))
    odb.set_filter_range(0, SLICE_HI)
    odb.add_targets(g.text, g.lengths, g.taxa, threads=16)
    odb.set_taxonomy(g.parents)
    of, oloc = odb.dump()
    keep = of <= SLICE_HI
    assert np.array_equal(gf, of[keep]) and np.array_equal(gloc, oloc[keep])
    want = [odb.classify(reads.text, reads.offsets, first=int(i), count=1) for i in sample]
    for shape, (gl, gt) in results.items():
        bad = [int(i) for (ol, ot), i in zip(want, sample)
               if ol[0] != gl[i] or not np.array_equal(ot[0], gt[i])]
        print(f"[scale] shape {shape}, sample of {sample.size}: {len(bad)} mismatches",
              flush=True)
        assert not bad, (shape, bad[:10])
    db.close()
