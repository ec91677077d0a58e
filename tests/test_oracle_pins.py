"""Pins of the CPU oracle against the paper and against brute force.

Every check here reaches the oracle's result by a different route than the
oracle itself (string slicing instead of 2-bit arithmetic, enumeration of all
ranges instead of the hit-window shortcut, ancestor sets instead of depth
walks, published hash vectors, closed forms), so that a dropped term, a wrong
index or a transposed operand in the oracle fails one of them.
"""
import itertools

import numpy as np
import pytest

from conftest import read_golden
from paper_2106_08150_amd import synth

COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
UNCL = 0xFFFFFFFF


def brute_canonical(kmer: str):
    """Canonical k-mer by strings: lexicographic min of k-mer and its reverse
    complement (A < C < G < T), then read as a base-4 number (A=0 ... T=3)."""
    up = kmer.upper()
    if any(c not in COMP for c in up):
        return None
    rc = "".join(COMP[c] for c in reversed(up))
    best = min(up, rc)
    v = 0
    for c in best:
        v = v * 4 + "ACGT".index(c)
    return v


def brute_window_sketches(seq: str, k: int, w: int, s: int, h1):
    """Sketch of each window by enumerating the k-mer starts of that window."""
    S = w - k + 1
    n_starts = len(seq) - k + 1
    out, j = [], 0
    while n_starts > 0 and j * S < n_starts:
        vals = set()
        for p in range(j * S, min((j + 1) * S, n_starts)):
            c = brute_canonical(seq[p:p + k])
            if c is not None:
                vals.add(h1(c))
        out.append(sorted(vals)[:s])
        j += 1
    return out


def rand_seq(rng, n, n_rate=0.0, lower_rate=0.0):
    s = rng.choice(list("ACGT"), size=n)
    if n_rate:
        s[rng.random(n) < n_rate] = "N"
    if lower_rate:
        m = rng.random(n) < lower_rate
        s[m] = np.char.lower(s[m])
    return "".join(s)


# ---------------------------------------------------------------- h1 ------
def test_h1_published_murmur3_vectors(orc):
    for seed, expected in read_golden("murmur3_fmix32_vectors.txt"):
        assert orc.h1(int(seed, 16)) == int(expected, 16)


def _unxorshift(y, r):
    x = y
    for _ in range(32 // r + 1):
        x = y ^ (x >> r)
    return x & 0xFFFFFFFF


def test_h1_is_a_bijection(orc):
    """Inverse derived from the algebra (xor-shift inversion, modular inverses
    of the odd multipliers) undoes h1 on random and edge inputs."""
    m1, m2 = 0x85EBCA6B, 0xC2B2AE35
    i1, i2 = pow(m1, -1, 1 << 32), pow(m2, -1, 1 << 32)

    def inv(y):
        x = _unxorshift(y, 16)
        x = (x * i2) & 0xFFFFFFFF
        x = _unxorshift(x, 13)
        x = (x * i1) & 0xFFFFFFFF
        return _unxorshift(x, 16)

    rng = np.random.default_rng(7)
    xs = [0, 1, 2, 0xFFFFFFFF, 0x80000000] + [int(v) for v in rng.integers(0, 1 << 32, 20000)]
    for x in xs:
        assert inv(orc.h1(x)) == x


# ------------------------------------------------------ k-mers, sketch ----
@pytest.mark.parametrize("k", [1, 4, 7, 15, 16])
def test_canonical_kmers_brute_force(orc, k):
    rng = np.random.default_rng(k)
    seq = rand_seq(rng, 400, n_rate=0.02, lower_rate=0.1)
    canon, valid = orc.kmers(seq, k)
    assert canon.size == len(seq) - k + 1
    for p in range(len(seq) - k + 1):
        c = brute_canonical(seq[p:p + k])
        assert valid[p] == (c is not None)
        if c is not None:
            assert canon[p] == c


def test_paper_worked_minhash_example(orc):
    """Sec. 2: with the listed hash values and s = 2 the sketch is {7, 8}."""
    rows = {r[0]: r[1:] for r in read_golden("minhash_worked_example.txt") if r[0] != "kmer"}
    kmers = [r[1:] for r in read_golden("minhash_worked_example.txt") if r[0] == "kmer"]
    seq, k, s = rows["sequence"][0], int(rows["k"][0]), int(rows["s"][0])
    # the 4-mers the paper lists are exactly the consecutive 4-mers of the text
    assert [seq[p:p + k] for p in range(len(seq) - k + 1)] == [m for m, _ in kmers]
    # equal k-mers get equal canonical values in the oracle (ACTG at 0 and 4)
    canon, valid = orc.kmers(seq, k)
    assert valid.all() and canon[0] == canon[4] and len(set(canon.tolist())) == 4
    mock = [int(v) for _, v in kmers]
    assert orc.bottom_s(mock, s) == [int(x) for x in rows["selected"]]
    # s larger than the number of distinct values keeps them all, in order
    assert orc.bottom_s(mock, 10) == [7, 8, 11, 14]


def test_window_counts_closed_form(orc):
    for L, k, w, nw, last in (map(int, r) for r in read_golden("window_counts.txt")):
        assert orc.num_windows(L, k, w) == nw
        if nw:
            S = w - k + 1
            assert (L - k + 1) - (nw - 1) * S == last


@pytest.mark.parametrize("k,w,s", [(16, 128, 16), (4, 20, 3), (5, 5, 1), (16, 40, 25)])
def test_window_sketches_brute_force(orc, k, w, s):
    rng = np.random.default_rng(w)
    for L in [0, k - 1, k, w, w + 1, 3 * w + 7, 700]:
        seq = rand_seq(rng, L, n_rate=0.01, lower_rate=0.05)
        got = orc.sketch_windows(seq, k, w, s)
        want = brute_window_sketches(seq, k, w, s, orc.h1)
        assert got == want
        # every k-mer start lies in exactly one window
        S = w - k + 1
        assert len(got) == (0 if L < k else -(-(L - k + 1) // S))


def test_sketch_reverse_complement_invariance(orc):
    """A single window holds the same canonical k-mers on both strands."""
    rng = np.random.default_rng(3)
    for L in [16, 50, 100, 128]:
        for _ in range(20):
            seq = rand_seq(rng, L, n_rate=0.01)
            rc = "".join(COMP.get(c, "N") for c in reversed(seq))
            a = orc.sketch_windows(seq, 16, 128, 16)
            b = orc.sketch_windows(rc, 16, 128, 16)
            assert a == b


def test_homopolymer_window_has_one_feature(orc):
    sk = orc.sketch_windows("A" * 300, 16, 128, 16)
    assert all(len(x) == 1 for x in sk) and len(sk) == 3
    # the poly-A k-mer is 0 (its reverse complement poly-T is larger); h1(0) = 0
    assert sk[0] == [0]


# --------------------------------------------------------- index + cap ----
def small_db(orc, genomes, k=16, w=128, s=16, cap=254, split=None, stop=False):
    db = orc.OracleDB(k, w, s, cap)
    if split is None:
        db.add_targets(genomes.text, genomes.lengths, genomes.taxa, stop_at_cap=stop)
    else:
        off = genomes.offsets
        for a, b in split:
            db.add_targets(genomes.text[int(off[a]):int(off[b])], genomes.lengths[a:b],
                           genomes.taxa[a:b], stop_at_cap=stop)
    db.set_taxonomy(genomes.parents)
    return db


def test_pairs_before_cap_equal_sum_of_sketch_sizes(orc):
    g = synth.tiny_genomes(length=20_000)
    db = small_db(orc, g, cap=65535)
    total = 0
    for i in range(g.lengths.size):
        total += sum(len(x) for x in orc.sketch_windows(g.genome(i), 16, 128, 16))
    assert db.num_pairs == total


def test_cap_strategies_agree(orc):
    """Trim-after-all-inserts equals in-order insertion that stops at the cap."""
    g = synth.repeated_genome(12, 3000, seed=5)
    g.text = g.text.copy()
    rng = np.random.default_rng(1)
    for i in range(1, 12):  # make the copies slightly different
        pos = rng.integers(0, 3000, 30) + 3000 * i
        g.text[pos] = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, 30)]
    for cap in [1, 3, 5, 11]:
        a = small_db(orc, g, cap=cap).dump()
        b = small_db(orc, g, cap=cap, stop=True).dump()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_cap_stress_repeated_genomes(orc):
    """300 identical genomes: each feature keeps its 254 smallest locations of
    the uncapped set, which brute force builds from genome 0's sketches."""
    n_copies, L = 300, 5000
    g = synth.repeated_genome(n_copies, L, seed=9)
    db = small_db(orc, g, cap=254)
    f, l = db.dump()
    windows_of = {}
    for j, sk in enumerate(orc.sketch_windows(g.genome(0), 16, 128, 16)):
        for x in sk:
            windows_of.setdefault(x, []).append(j)
    want_f, want_l = [], []
    for x in sorted(windows_of):
        locs = sorted((t << 18) | j for t in range(n_copies) for j in windows_of[x])[:254]
        want_f += [x] * len(locs)
        want_l += locs
    assert np.array_equal(f, np.array(want_f, np.uint32))
    assert np.array_equal(l, np.array(want_l, np.uint32))
    # every feature is full
    _, counts = np.unique(f, return_counts=True)
    assert (counts == 254).all()


def test_incremental_build_equals_one_shot(orc):
    g = synth.tiny_genomes(length=30_000)
    for cap in [2, 254]:
        a = small_db(orc, g, cap=cap).dump()
        b = small_db(orc, g, cap=cap, split=[(0, 3), (3, 4), (4, 8)]).dump()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_target_capacity_errors(orc):
    """Target ids use 14 bits (16383 ids, 0 .. 16382) and window ids 18 bits."""
    db = orc.OracleDB()
    n = 16384
    with pytest.raises(ValueError):
        db.add_targets(np.full(n * 20, ord("A"), np.uint8), np.full(n, 20, np.uint64),
                       np.zeros(n, np.uint32))
    assert db.num_pairs == 0
    big = (1 << 18) * 113 + 16          # one window more than 2^18
    with pytest.raises(ValueError):
        db.add_targets(np.full(16, ord("A"), np.uint8), np.array([big], np.uint64),
                       np.zeros(1, np.uint32))


# --------------------------------------------------------- taxonomy ------
def test_lca_hand_cases(orc):
    rows = read_golden("lca_tiny_tree.txt")
    parents = [int(x) for x in rows[0][1:]]
    db = orc.OracleDB()
    db.set_taxonomy(np.array(parents, np.uint32))
    for a, b, want in rows[1:]:
        assert db.lca(int(a), int(b)) == int(want)


def test_lca_against_ancestor_sets(orc):
    g = synth.clustered_genomes(6, 5, 6e5, seed=3, median_bp=2e4, clip=(1e4, 4e4))
    parents = g.parents
    db = orc.OracleDB()
    db.set_taxonomy(parents)

    def chain(x):
        out = [x]
        while parents[x] != x:
            x = int(parents[x])
            out.append(x)
        return out

    rng = np.random.default_rng(0)
    for _ in range(300):
        a, b = (int(v) for v in rng.integers(0, parents.size, 2))
        common = set(chain(a)) & set(chain(b))
        deepest = max(common, key=lambda x: len(chain(x)))
        assert db.lca(a, b) == deepest


def test_decision_rule_hand_cases(orc):
    db = orc.OracleDB()
    db.set_taxonomy(synth.TINY_PARENTS)
    g = synth.tiny_genomes(length=2000)
    db.add_targets(g.text, g.lengths, g.taxa)     # targets 0..7 -> species 3..10
    # no candidate / below threshold
    assert db.decide([], [], 4, 0) == UNCL
    assert db.decide([0], [3], 4, 0) == UNCL
    # clear lead -> taxon of the top target
    assert db.decide([2, 5], [9, 5], 4, 0) == 5
    # tie -> LCA of the tied targets' taxa (targets 0,1 -> species 3,4 -> genus 1)
    assert db.decide([0, 1, 6], [7, 7, 2], 4, 0) == 1
    # tie across genera -> root
    assert db.decide([0, 4], [7, 7], 4, 0) == 0
    # lead 2 with hit_diff 1 -> species; with hit_diff 2 -> LCA of both
    assert db.decide([0, 1], [9, 7], 4, 1) == 3
    assert db.decide([0, 1], [9, 7], 4, 2) == 1
    # "close to maximum" includes lower entries within hit_diff only
    assert db.decide([0, 1, 4], [9, 8, 6], 4, 1) == 1
    assert db.decide([0, 1, 4], [9, 8, 7], 4, 2) == 0
    # single candidate at threshold
    assert db.decide([7], [4], 4, 0) == 10


# ---------------------------------------------------------- scoring ------
def brute_classify(index_f, index_l, feats, F, k, w, top_m):
    """Top list by enumerating every (target, start window) range."""
    from collections import Counter
    S = w - k + 1
    sws = 1 if F < k else -(-(F - k) // S) + 1
    by_f = {}
    for f, l in zip(index_f.tolist(), index_l.tolist()):
        by_f.setdefault(f, []).append(l)
    hits = Counter()
    for f in feats:
        for l in by_f.get(int(f), []):
            hits[l] += 1
    targets = sorted({l >> 18 for l in hits})
    cand = []
    for t in targets:
        wins = {l & 0x3FFFF: c for l, c in hits.items() if l >> 18 == t}
        top_w = max(wins)
        best, start = -1, None
        for w0 in range(0, top_w + 1):        # every start, not only hit windows
            sc = sum(wins.get(x, 0) for x in range(w0, w0 + sws))
            if sc > best:
                best, start = sc, w0
        begin = min(x for x in wins if start <= x < start + sws)
        cand.append((t, best, begin))
    cand.sort(key=lambda c: (-c[1], c[0]))
    return cand[:top_m]


@pytest.mark.parametrize("top_m,min_hits,hit_diff", [(4, 4, 0), (1, 1, 0), (2, 1, 3)])
def test_classify_matches_brute_force(orc, top_m, min_hits, hit_diff):
    g = synth.tiny_genomes(length=6000)
    db = small_db(orc, g, cap=5)
    f_idx, l_idx = db.dump()
    rng = np.random.default_rng(top_m * 10 + hit_diff)
    # single-end reads of several lengths, plus paired records
    se = [synth.sample_reads(g, 40, L, seed=L, error=0.02, foreign=0.1) for L in (20, 100, 150, 260)]
    for r in se:
        labels, top = db.classify(r.text, r.offsets, top_m=top_m, min_hits=min_hits,
                                  hit_diff=hit_diff)
        for i in range(r.n_records):
            a, b = int(r.offsets[i]), int(r.offsets[i + 1])
            feats = orc.query_features(r.text[a:b], np.array([0, b - a], np.uint64), 16, 128,
                                       16, 0, 1, False)
            want = brute_classify(f_idx, l_idx, feats, b - a, 16, 128, top_m)
            got = [tuple(int(x) for x in top[i, j]) for j in range(len(want))]
            assert got == want
            for j in range(len(want), top_m):
                assert tuple(top[i, j]) == (UNCL, 0, 0)
            lab = db.decide([c[0] for c in want], [c[1] for c in want], min_hits, hit_diff)
            assert labels[i] == lab
    # paired layout: mate 2 reverse-complemented from a fragment end
    recs = synth.mixed_records(g, 60, seed=11)
    labels, top = db.classify(recs.text, recs.offsets, paired=True, top_m=top_m,
                              min_hits=min_hits, hit_diff=hit_diff, insert_size=400)
    for i in range(recs.n_records):
        a, b, c = (int(x) for x in recs.offsets[2 * i:2 * i + 3])
        feats = orc.query_features(recs.text, recs.offsets, 16, 128, 16, i, 1, True)
        F = (b - a) + (c - b)
        if b > a and c > b:
            F = max(F, 400)
        want = brute_classify(f_idx, l_idx, feats, F, 16, 128, top_m)
        got = [tuple(int(x) for x in top[i, j]) for j in range(len(want))]
        assert got == want


def test_exact_window_read_hits_its_window(orc):
    """A read equal to reference window (t, j) carries that window's sketch, so
    target t scores at least the sketch size in a range starting at or before j."""
    g = synth.tiny_genomes(length=10_000)
    db = small_db(orc, g)
    S = 113
    for t in [0, 3, 7]:
        sk = orc.sketch_windows(g.genome(t), 16, 128, 16)
        for j in [0, 5, 40]:
            txt = g.genome(t)[j * S:j * S + 128]
            off = np.array([0, txt.size], np.uint64)
            _, top = db.classify(txt, off, top_m=8)
            row = {int(x[0]): (int(x[1]), int(x[2])) for x in top[0] if x[0] != UNCL}
            assert t in row and row[t][0] >= len(sk[j]) and row[t][1] <= j


def test_sws_closed_form_by_enumeration(orc):
    """sws is the most windows the k-mers of a length-F fragment can touch."""
    k, w = 16, 128
    S = w - k + 1
    for F, want in [(100, 2), (150, 3), (250, 4), (400, 5), (16, 1), (15, 1), (129, 2), (130, 3)]:
        if F >= k:
            most = max(len({p // S for p in range(q, q + F - k + 1)}) for q in range(3 * S))
            assert most == want
        assert orc.sws(F, k, w) == want


def test_reads_shorter_than_k_are_unclassified(orc):
    g = synth.tiny_genomes(length=3000)
    db = small_db(orc, g)
    txt = g.genome(0)[100:115]
    labels, top = db.classify(txt, np.array([0, 15, 15], np.uint64), min_hits=1)
    assert labels.tolist() == [UNCL, UNCL]
    assert (top[:, :, 0] == UNCL).all()
