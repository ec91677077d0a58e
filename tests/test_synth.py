"""Seeded input generators (shared by the oracle and the HIP path; they hold
none of the method's arithmetic)."""
import numpy as np

from paper_2106_08150_amd import synth


def test_large_genomes_independent_of_workers():
    """The large reference set draws cluster c from its own seed, so the text
    is the same whatever the number of worker processes."""
    a = synth.large_genomes(total_bp=2e7, n_clusters=12, per_cluster=10, level1=3, workers=4)
    b = synth.large_genomes(total_bp=2e7, n_clusters=12, per_cluster=10, level1=3, workers=1)
    assert np.array_equal(a.text, b.text)
    assert np.array_equal(a.lengths, b.lengths) and np.array_equal(a.taxa, b.taxa)


def test_large_genomes_shape_and_taxonomy():
    g = synth.large_genomes(total_bp=2e7, n_clusters=12, per_cluster=10, level1=3, workers=2)
    assert g.lengths.size == 120 and abs(int(g.lengths.sum()) - 2e7) < 1000
    assert g.text.size == int(g.lengths.sum())
    assert set(np.unique(g.text).tolist()) <= set(b"ACGT")
    # five levels: root, level 1, cluster, sub-group, leaf; every taxon reaches the root
    depth = np.zeros(g.parents.size, np.int64)
    for v in range(1, g.parents.size):
        d, u = 0, v
        while u != 0:
            u = int(g.parents[u])
            d += 1
            assert d < 10
        depth[v] = d
    assert sorted(set(depth[g.taxa].tolist())) == [4]
    # members of a cluster are copies of one root: close to each other, far from others
    off = np.concatenate([[0], np.cumsum(g.lengths.astype(np.int64))])
    m = int(g.lengths[:10].min())
    x, y = g.text[off[0]:off[0] + m], g.text[off[1]:off[1] + m]
    far = g.text[off[10]:off[10] + m]
    assert (x != y).mean() < 0.45 and abs((x != far).mean() - 0.75) < 0.05
