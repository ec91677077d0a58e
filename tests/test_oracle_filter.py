"""Pins of the oracle's feature-filtered index and of its threaded paths.

The at-scale parity tests and the CPU baseline classify read samples against an
oracle index that keeps only the features those reads look up (plus a feature
range kept for table parity). That shortcut rests on two facts that hold by
the method's definition (Sec. 4.1, Sec. 4.2): a read's hits come only from the
locations of its own sketch features, and the per-feature cap looks at one
feature's locations only. These tests check the filtered oracle against the
unfiltered one (itself pinned by brute force in test_oracle_pins.py): same
labels and top hits for the sample, and the same pairs for every kept feature.
They also check that the thread count of the oracle's build and classify
changes nothing.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2106_08150_amd import synth


def full_oracle(g, threads=1, cap=254):
    odb = orc.OracleDB(16, 128, 16, cap)
    odb.add_targets(g.text, g.lengths, g.taxa, threads=threads)
    odb.set_taxonomy(g.parents)
    return odb


def sample_features(reads, first, count, paired):
    return np.unique(orc.query_features(reads.text, reads.offsets, 16, 128, 16, first, count,
                                        paired))


def filtered_oracle(g, feats, lo=1, hi=0, cap=254, threads=4):
    odb = orc.OracleDB(16, 128, 16, cap)
    odb.set_filter(feats)
    if lo <= hi:
        odb.set_filter_range(lo, hi)
    odb.add_targets(g.text, g.lengths, g.taxa, threads=threads)
    odb.set_taxonomy(g.parents)
    return odb


CASES = {
    "tiny_single": lambda: (synth.tiny_genomes(length=40_000), False),
    "clustered_paired": lambda: (synth.clustered_genomes(5, 6, 3e6, seed=41, median_bp=1e5,
                                                         clip=(3e3, 4e5)), True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_filtered_index_classifies_sample_exactly(case):
    g, paired = CASES[case]()
    if paired:
        reads = synth.mixed_records(g, 600, seed=71)
        opts = dict(paired=True, insert_size=400)
    else:
        reads = synth.sample_reads(g, 600, 100, seed=71, foreign=0.05)
        opts = {}
    full = full_oracle(g)
    first, count = 100, 300
    want_l, want_t = full.classify(reads.text, reads.offsets, first=first, count=count, **opts)
    feats = sample_features(reads, first, count, paired)
    lo, hi = 0, (1 << 26) - 1          # a feature range kept besides the sample's features
    flt = filtered_oracle(g, feats, lo, hi)
    got_l, got_t = flt.classify(reads.text, reads.offsets, first=first, count=count, **opts)
    assert np.array_equal(got_l, want_l) and np.array_equal(got_t, want_t)
    # the filter is not vacuous: it dropped most pairs, and the sample classifies
    assert flt.num_pairs < full.num_pairs // 2
    assert (want_l != orc.UNCLASSIFIED).sum() > count // 2
    # every kept feature has exactly the full index's locations
    ff, fl = full.dump()
    gf, gl = flt.dump()
    keep = np.isin(ff, feats) | ((ff >= lo) & (ff <= hi))
    assert np.array_equal(gf, ff[keep]) and np.array_equal(gl, fl[keep])
    # its dump restricted to the range equals the full dump's slice
    r = (gf >= lo) & (gf <= hi)
    s = (ff >= lo) & (ff <= hi)
    assert np.array_equal(gf[r], ff[s]) and np.array_equal(gl[r], fl[s])


def test_filtered_index_keeps_the_cap():
    """The cap acts per feature: with every genome identical (300 copies, cap
    254) a kept feature holds exactly the 254 smallest locations, filtered or
    not, and the sample's labels agree."""
    g = synth.repeated_genome(300, 3000, seed=9)
    reads = synth.sample_reads(g, 50, 150, seed=10)
    full = full_oracle(g, threads=4)
    feats = sample_features(reads, 0, 50, False)
    flt = filtered_oracle(g, feats)
    ff, fl = full.dump()
    gf, gl = flt.dump()
    keep = np.isin(ff, feats)
    assert np.array_equal(gf, ff[keep]) and np.array_equal(gl, fl[keep])
    u, c = np.unique(gf, return_counts=True)
    # a read's windows start elsewhere than the reference windows, so only some
    # of its features are reference sketch features
    assert (c == 254).all() and u.size == np.isin(feats, ff).sum() > 100
    a = full.classify(reads.text, reads.offsets)
    b = flt.classify(reads.text, reads.offsets)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_thread_count_changes_nothing():
    g = synth.clustered_genomes(4, 5, 2e6, seed=47, median_bp=1e5, clip=(3e3, 3e5))
    one = full_oracle(g, threads=1)
    eight = full_oracle(g, threads=8)
    f1, l1 = one.dump()
    f8, l8 = eight.dump()
    assert np.array_equal(f1, f8) and np.array_equal(l1, l8)
    for reads, opts in ((synth.sample_reads(g, 700, 150, seed=3, foreign=0.05), {}),
                        (synth.mixed_records(g, 500, seed=4), dict(paired=True,
                                                                   insert_size=400))):
        a = one.classify(reads.text, reads.offsets, threads=1, **opts)
        b = one.classify(reads.text, reads.offsets, threads=8, **opts)
        c = eight.classify(reads.text, reads.offsets, threads=3, **opts)
        for x in (b, c):
            assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1])
