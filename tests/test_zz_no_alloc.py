"""The classification entry point that allocates nothing (mc_classify_noalloc)
against mc_classify_ex, through the C ABI: labels and top hits bit for bit, on
two calls in a row (the second with a smaller batch, so stale scratch contents
would show), over records that take every pass (fast path, large-list pass,
HBM-list pass) and with size-class routing on; oversized batches are rejected
before anything is launched."""
import numpy as np
import pytest

import paper_2106_08150_amd as mc
from paper_2106_08150_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def records(g, n_short, seed):
    """n_short short single-end reads and pairs, then long pairs and reads
    (paired layout). On 24 identical genomes every feature has 24 locations:
    a 100 bp read gathers 384 (fast path), a 2 x 150 bp pair 1,536 (large-list
    pass), a 5,000 bp read 17,280 and a 10,000 bp read 34,176 (HBM-list
    pass)."""
    rng = np.random.default_rng(seed)
    g0 = g.genome(0)
    pieces = []
    for _ in range(n_short):
        t = int(rng.integers(0, g.lengths.size))
        gt = g.genome(t)
        a = int(rng.integers(0, gt.size - 300))
        if rng.random() < 0.5:
            pieces += [gt[a:a + int(rng.integers(50, 251))], gt[:0]]
        else:
            pieces += [gt[a:a + 150], synth.reverse_complement_text(gt[a + 150:a + 300])]
    pieces += [g0[1000:1600], g0[5000:5600],      # 2 x 600: large-list pass
               g0[2000:3000], g0[4000:5000],      # 2 x 1,000: large-list pass
               g0[7000:12000], g0[:0],            # 5,000 bp single: HBM-list pass
               g0[3000:13000], g0[:0]]            # 10,000 bp single: HBM-list pass
    off = np.zeros(len(pieces) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in pieces])
    return synth.Reads(np.concatenate(pieces), off, paired=True)


def run(torch, db, reads, fn, opts):
    n = reads.offsets.size // 2
    r = torch.from_numpy(reads.text.copy()).cuda()
    o = torch.from_numpy(reads.offsets.view(np.int64).copy()).cuda()
    lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    top = torch.full((n * opts.top_m * 3,), -7, dtype=torch.int32, device="cuda")
    fn(db.h, r, o, n, opts, lab, top)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), top.cpu().numpy()


@pytest.mark.parametrize("routed", [False, True])
def test_noalloc_equals_classify_ex(torch, routed):
    g = synth.repeated_genome(24, 20_000, seed=21)
    db = mc.Database()
    db.add_targets(torch.from_numpy(g.text.copy()).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    if routed:
        cfg = (512, 4, 16384)
        mc.mc_db_set_routing(db.h, [3, 8], [cfg, (256, 4, 16384), (1024, 2, 4096)])
    opts = mc.QueryOpts(4, 1, 0, 400, 1)
    for n_short, seed in ((3000, 1), (700, 2)):      # second call smaller
        reads = records(g, n_short, seed)
        print(f"noalloc routed={routed}: {reads.offsets.size // 2} records", flush=True)
        want = run(torch, db, reads, mc.mc_classify_ex, opts)
        got = run(torch, db, reads, mc.mc_classify_noalloc, opts)
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1], want[1])
        assert (want[0][-4:] != -1).all()       # the long records are classified
    db.close()


def test_noalloc_rejects_oversized_batches(torch):
    g = synth.tiny_genomes(length=20_000)
    db = mc.Database()
    db.add_targets(torch.from_numpy(g.text.copy()).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    n = mc.NOALLOC_MAX_RECORDS + 1
    r = torch.zeros(16, dtype=torch.uint8, device="cuda")
    o = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(mc.MCError) as e:
        mc.mc_classify_noalloc(db.h, r, o, n, mc.QueryOpts(4, 4, 0, 0, 0), lab, None)
    assert e.value.code == -1 and "exceed" in str(e.value)
    torch.cuda.synchronize()
    assert bool((lab == -7).all())                  # nothing was launched
    db.close()
