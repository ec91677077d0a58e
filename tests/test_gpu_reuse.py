"""Rebuilds on device blocks the library kept for reuse.

Blocks released by one handle (the table, build scratch, the query workspace's
record queues and HBM-list scratch) are handed to the next handle's
allocations with the previous contents still in them; every result must be
the same as on freshly mapped memory.
"""
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


@pytest.fixture(scope="module")
def sets():
    a = synth.scale_genomes(seed=611, total_bp=1.5e8)
    b = synth.scale_genomes(seed=612, total_bp=1.5e8)
    reads = synth.scale_reads(a, n=100_000, seed=613)
    return a, b, reads


def run(torch, g, reads, reserve):
    db = mc.Database(16, 128, 16, 254)
    if reserve:
        db.reserve(reserve)
    db.add_targets(torch.from_numpy(g.text.copy()).cuda(), g.lengths, g.taxa)
    db.set_taxonomy(g.parents)
    f, loc = db.dump()
    r = torch.from_numpy(reads.text.copy()).cuda()
    o = torch.from_numpy(reads.offsets.view(np.int64).copy()).cuda()
    labels, top = db.classify(r, o, reads.n_records, with_top=True)
    torch.cuda.synchronize()
    out = (f.copy(), loc.copy(), labels.cpu().numpy().copy(), top.cpu().numpy().copy())
    table_bytes = db.stats()["table_bytes"]
    db.close()
    return out, table_bytes


@pytest.fixture()
def keep_blocks():
    mc.mc_set_cached_memory_limit(64 << 30)
    yield
    mc.mc_set_cached_memory_limit(0)


@pytest.mark.parametrize("reserve", [0, 20_000_000])
def test_rebuild_on_reused_blocks(torch, sets, reserve, keep_blocks):
    a, b, reads = sets
    print(f"reuse case: reserve={reserve}", flush=True)
    first, table_bytes = run(torch, a, reads, reserve)
    assert table_bytes >= 256 << 20          # a block the library keeps for reuse
    assert first[0].size > 10_000_000
    run(torch, b, reads, reserve)             # leaves other entries in the blocks it releases
    again, _ = run(torch, a, reads, reserve)
    for x, y in zip(first, again):
        assert np.array_equal(x, y)
    mc.mc_release_cached_memory()
    fresh, _ = run(torch, a, reads, reserve)
    for x, y in zip(first, fresh):
        assert np.array_equal(x, y)
