"""Seeded synthetic inputs shaped like the paper's workloads.

This module only produces bytes: reference genomes as ASCII, taxonomies as
parent arrays, and read records as ASCII plus offsets. It holds none of the
classifier's arithmetic (no base codes, k-mers, hashes or sketches), so both
the HIP path and the CPU oracle can take their inputs from it.

Generator rules (numpy ``Generator(PCG64(seed))`` everywhere):

* bases are i.i.d. uniform over ``ACGT``;
* a mutated copy substitutes every base independently with probability ``d``
  by one of the three other letters, chosen uniformly (substitution sites are
  drawn as geometric gaps, which is the same Bernoulli process);
* a read picks a genome uniformly, a start uniformly in ``[0, L - len]`` and
  the reverse strand with probability 1/2 (reverse strand = reverse
  complement of the ASCII text), then gets substitutions at its error rate;
* foreign reads are i.i.d. random text that is not drawn from any genome.

The reference sets of the paper (RefSeq 202, AFS 31) and its read sets (HiSeq,
MiSeq, KAL_D) are not available; these generators stand in for them with the
shapes given in the evaluation section (read lengths around 100 to 250 bp,
paired reads of 2 x 101 to 2 x 150 bp, thousands of bacterial-sized genomes).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_LETTERS = np.frombuffer(b"ACGT", dtype=np.uint8)
# For every letter, the three other letters (substitution targets).
_OTHER = np.zeros((256, 3), dtype=np.uint8)
for _c, _o in ((b"A", b"CGT"), (b"C", b"AGT"), (b"G", b"ACT"), (b"T", b"ACG")):
    _OTHER[_c[0]] = np.frombuffer(_o, dtype=np.uint8)
# ASCII complement table for the reverse strand of generated text.
_COMP = np.arange(256, dtype=np.uint8)
for _a, _b in ((b"A", b"T"), (b"C", b"G"), (b"G", b"C"), (b"T", b"A")):
    _COMP[_a[0]] = _b[0]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_text(rng: np.random.Generator, n: int) -> np.ndarray:
    """``n`` i.i.d. uniform letters from ACGT as uint8 ASCII."""
    return _LETTERS[rng.integers(0, 4, size=int(n), dtype=np.uint8)]


def substitute(rng: np.random.Generator, text: np.ndarray, d: float) -> np.ndarray:
    """Copy of ``text`` with each letter replaced w.p. ``d`` by another letter."""
    out = np.array(text, dtype=np.uint8, copy=True)
    substitute_inplace(rng, out, d)
    return out


def substitute_inplace(rng: np.random.Generator, out: np.ndarray, d: float) -> None:
    """In-place form of :func:`substitute` (same random draws)."""
    n = out.size
    if d <= 0.0 or n == 0:
        return
    # Bernoulli(d) sites as cumulative geometric gaps.
    est = int(n * d + 10 * np.sqrt(n * d + 1) + 16)
    pos = np.cumsum(rng.geometric(d, size=est)) - 1
    while pos.size and pos[-1] < n:  # extend in the (rare) short case
        more = np.cumsum(rng.geometric(d, size=est)) + pos[-1]
        pos = np.concatenate([pos, more])
    pos = pos[pos < n]
    pick = rng.integers(0, 3, size=pos.size)
    out[pos] = _OTHER[out[pos], pick]


def _windows(text: np.ndarray, width: int) -> np.ndarray:
    """Read-only view of every ``width``-long substring of ``text`` (one per row)."""
    t = np.ascontiguousarray(text, dtype=np.uint8)
    return np.lib.stride_tricks.as_strided(t, shape=(max(t.size - width + 1, 0), width),
                                           strides=(1, 1), writeable=False)


def reverse_complement_text(text: np.ndarray) -> np.ndarray:
    return _COMP[np.asarray(text, dtype=np.uint8)[::-1]]


@dataclass
class Genomes:
    """Concatenated reference text plus per-genome lengths and taxa."""
    text: np.ndarray          # uint8 ASCII, all genomes back to back
    lengths: np.ndarray       # uint64 [n]
    taxa: np.ndarray          # uint32 [n]
    parents: np.ndarray       # uint32 [n_nodes], parents[root] == root

    @property
    def offsets(self) -> np.ndarray:
        o = np.zeros(self.lengths.size + 1, dtype=np.uint64)
        np.cumsum(self.lengths, out=o[1:])
        return o

    def genome(self, i: int) -> np.ndarray:
        o = self.offsets
        return self.text[int(o[i]):int(o[i + 1])]


@dataclass
class Reads:
    """Read records: ASCII text plus u64 offsets.

    Single-end (``paired=False``): record i is ``text[off[i]:off[i+1]]``.
    Paired (``paired=True``): record i has mate 1 ``text[off[2i]:off[2i+1]]``
    and mate 2 ``text[off[2i+1]:off[2i+2]]``; an empty mate 2 marks a
    single-end record inside a paired batch.
    """
    text: np.ndarray
    offsets: np.ndarray
    paired: bool = False
    origin: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))

    @property
    def n_records(self) -> int:
        return (self.offsets.size - 1) // (2 if self.paired else 1)


def _pack(chunks: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    lens = np.fromiter((c.size for c in chunks), dtype=np.uint64, count=len(chunks))
    off = np.zeros(len(chunks) + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    text = np.concatenate(chunks) if chunks else np.zeros(0, np.uint8)
    return text.astype(np.uint8, copy=False), off


# --------------------------------------------------------------------------
# Tiny configuration: 8 genomes of 100 kbp, root -> 2 genera -> 4 species each.
# --------------------------------------------------------------------------
TINY_DIVERGENCE = (0.0, 0.01, 0.025, 0.04, 0.055, 0.07, 0.085, 0.10)
TINY_PARENTS = np.array([0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2], dtype=np.uint32)


def tiny_genomes(seed: int = 101, length: int = 100_000) -> Genomes:
    rng = rng_for(seed)
    g0 = random_text(rng, length)
    chunks = [g0] + [substitute(rng, g0, d) for d in TINY_DIVERGENCE[1:]]
    text, off = _pack(chunks)
    lengths = np.diff(off).astype(np.uint64)
    taxa = np.arange(3, 3 + len(chunks), dtype=np.uint32)   # genome i -> species 3+i
    return Genomes(text, lengths, taxa, TINY_PARENTS.copy())


def sample_reads(genomes: Genomes, n: int, length: int, seed: int,
                 error: float = 0.01, foreign: float = 0.0,
                 chunk: int = 200_000, progress=None) -> Reads:
    """``n`` single-end reads of a fixed ``length`` (see the module rules)."""
    rng = rng_for(seed)
    off_g = genomes.offsets
    lens = genomes.lengths.astype(np.int64)
    ok = np.nonzero(lens >= length)[0]
    text = np.empty(n * length, dtype=np.uint8)
    origin = np.empty(n, dtype=np.int64)
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        gi = ok[rng.integers(0, ok.size, size=m)]
        is_foreign = rng.random(m) < foreign
        start = (rng.random(m) * (lens[gi] - length + 1)).astype(np.int64)
        rev = rng.random(m) < 0.5
        block = _windows(genomes.text, length)[off_g[gi].astype(np.int64) + start]
        block[rev] = _COMP[block[rev][:, ::-1]]
        nf = int(is_foreign.sum())
        if nf:
            block[is_foreign] = random_text(rng, nf * length).reshape(nf, length)
        flat = substitute(rng, block.reshape(-1), error)
        text[c0 * length:(c0 + m) * length] = flat
        origin[c0:c0 + m] = np.where(is_foreign, -1, gi)
        if progress is not None and (c0 // chunk) % 10 == 9:
            progress(f"reads {c0 + m}/{n}")
    offsets = np.arange(n + 1, dtype=np.uint64) * np.uint64(length)
    return Reads(text, offsets, False, origin)


def tiny_reads(genomes: Genomes, n: int = 10_000, seed: int = 102) -> Reads:
    return sample_reads(genomes, n, 100, seed, error=0.01)


# --------------------------------------------------------------------------
# Clustered reference sets (the "at scale" shape): clusters of mutated copies.
# --------------------------------------------------------------------------
def clustered_genomes(n_clusters: int, per_cluster: int, total_bp: float,
                      seed: int, div_lo: float = 0.02, div_hi: float = 0.15,
                      median_bp: float = 4e6, sigma: float = 0.4,
                      clip: tuple[float, float] = (1e6, 1e7),
                      level1: int | None = None, progress=None) -> Genomes:
    """Clusters of mutated copies with log-normal lengths.

    Lengths are log-normal around ``median_bp`` (shape ``sigma``), clipped to
    ``clip`` and rescaled together so that they sum to about ``total_bp``.
    Each cluster has a random root as long as its longest member; member ``i``
    is the root's prefix of its own length with divergence ``U[div_lo,
    div_hi]``. Taxonomy: root -> ``level1`` nodes -> one node per cluster ->
    three sub-groups per cluster (members split as evenly as possible) -> one
    leaf per genome.
    """
    rng = rng_for(seed)
    n = n_clusters * per_cluster
    raw = np.exp(rng.normal(np.log(median_bp), sigma, size=n))
    raw = np.clip(raw, clip[0], clip[1])
    lengths = np.maximum(np.round(raw * (total_bp / raw.sum())), 1).astype(np.int64)
    level1 = level1 or max(1, n_clusters // 5)
    # node ids: 0 root | level1 | clusters | 3 per cluster | leaves
    l1_base = 1
    cl_base = l1_base + level1
    sub_base = cl_base + n_clusters
    leaf_base = sub_base + 3 * n_clusters
    n_nodes = leaf_base + n
    parents = np.zeros(n_nodes, dtype=np.uint32)
    parents[l1_base:cl_base] = 0
    for c in range(n_clusters):
        parents[cl_base + c] = l1_base + (c * level1) // n_clusters
        for j in range(3):
            parents[sub_base + 3 * c + j] = cl_base + c
    taxa = np.zeros(n, dtype=np.uint32)
    # genomes are stored in generation order: cluster by cluster, group by group
    order = []
    for c in range(n_clusters):
        ids = np.arange(c * per_cluster, (c + 1) * per_cluster)
        for grp in np.array_split(np.arange(per_cluster), 3):
            order.extend(int(ids[m]) for m in grp)
    out_len = lengths[np.array(order)]
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(out_len, out=off[1:])
    text = np.empty(int(off[-1]), dtype=np.uint8)
    pos = 0
    for c in range(n_clusters):
        ids = np.arange(c * per_cluster, (c + 1) * per_cluster)
        root = random_text(rng, int(lengths[ids].max()))
        divs = rng.uniform(div_lo, div_hi, size=per_cluster)
        groups = np.array_split(np.arange(per_cluster), 3)
        for gidx, grp in enumerate(groups):
            for m in grp:
                gid = int(ids[m])
                L = int(lengths[gid])
                dst = text[int(off[pos]):int(off[pos]) + L]
                dst[:] = root[:L]
                substitute_inplace(rng, dst, float(divs[m]))
                parents[leaf_base + gid] = sub_base + 3 * c + gidx
                taxa[gid] = leaf_base + gid
                pos += 1
        if progress is not None and c % 10 == 9:
            progress(f"clusters {c + 1}/{n_clusters}")
    return Genomes(text, out_len.astype(np.uint64), taxa[np.array(order)], parents)


def scale_genomes(seed: int = 201, total_bp: float = 4.0e9, progress=None) -> Genomes:
    """1,000 genomes = 100 clusters x 10 (about 4 Gbp), 5-level taxonomy."""
    return clustered_genomes(100, 10, total_bp, seed, level1=20, progress=progress)


_LARGE_TEXT = None   # shared text of large_genomes() while its workers run


def _large_cluster(args) -> None:
    """Worker of :func:`large_genomes`: cluster c written into the shared text."""
    seed, c, spans, divs = args
    text = _LARGE_TEXT
    rng = rng_for(seed * 1_000_003 + c)
    root = random_text(rng, max(L for _, L in spans))
    for (o, L), d in zip(spans, divs):
        dst = text[o:o + L]
        dst[:] = root[:L]
        substitute_inplace(rng, dst, d)


def _gpu_runtime_in_use() -> bool:
    """Whether this process has initialised a GPU through torch, or loaded
    libmc.so on a machine with a GPU (its HIP runtime must not be shared with
    forked children). Counting devices does not initialise one."""
    import sys
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return True
    mc = sys.modules.get("paper_2106_08150_amd")
    return (mc is not None and getattr(mc, "_lib", None) is not None and torch is not None
            and torch.cuda.device_count() > 0)


def large_genomes(seed: int = 501, total_bp: float = 3.0e10, n_clusters: int = 750,
                  per_cluster: int = 10, div_lo: float = 0.01, div_hi: float = 0.20,
                  level1: int = 150, workers: int = 16, progress=None) -> Genomes:
    """The large reference set: 7,500 genomes = 750 clusters x 10 (about 30 Gbp),
    divergence U[1%, 20%], lengths and taxonomy as :func:`clustered_genomes`.
    Cluster c is drawn from its own seed, so the text does not depend on the
    number of worker processes. Workers are forked: call this before the
    process touches a GPU."""
    import mmap
    import multiprocessing as mp
    import sys
    global _LARGE_TEXT
    if _gpu_runtime_in_use():
        raise RuntimeError("large_genomes forks worker processes: call it before the process "
                           "touches a GPU or loads the HIP library")
    rng = rng_for(seed)
    n = n_clusters * per_cluster
    raw = np.exp(rng.normal(np.log(4e6), 0.4, size=n))
    raw = np.clip(raw, 1e6, 1e7)
    lengths = np.maximum(np.round(raw * (total_bp / raw.sum())), 1).astype(np.int64)
    divs = rng.uniform(div_lo, div_hi, size=n)
    l1_base = 1
    cl_base = l1_base + level1
    sub_base = cl_base + n_clusters
    leaf_base = sub_base + 3 * n_clusters
    parents = np.zeros(leaf_base + n, dtype=np.uint32)
    taxa = np.zeros(n, dtype=np.uint32)
    order, leaf_parent = [], {}
    for c in range(n_clusters):
        parents[cl_base + c] = l1_base + (c * level1) // n_clusters
        ids = np.arange(c * per_cluster, (c + 1) * per_cluster)
        for j, grp in enumerate(np.array_split(np.arange(per_cluster), 3)):
            parents[sub_base + 3 * c + j] = cl_base + c
            for m in grp:
                gid = int(ids[m])
                order.append(gid)
                parents[leaf_base + gid] = sub_base + 3 * c + j
                taxa[gid] = leaf_base + gid
    order = np.array(order)
    out_len = lengths[order]
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(out_len, out=off[1:])
    size = int(off[-1])
    # anonymous shared mapping: the forked workers write into it in place
    buf = mmap.mmap(-1, max(size, 1), flags=mmap.MAP_SHARED | mmap.MAP_ANONYMOUS)
    text = np.frombuffer(buf, dtype=np.uint8, count=size)
    pos_of = {int(g): i for i, g in enumerate(order)}
    jobs = []
    for c in range(n_clusters):
        ids = range(c * per_cluster, (c + 1) * per_cluster)
        spans = [(int(off[pos_of[g]]), int(lengths[g])) for g in ids]
        jobs.append((seed, c, spans, [float(divs[g]) for g in ids]))
    _LARGE_TEXT = text
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            for i, _ in enumerate(pool.imap_unordered(_large_cluster, jobs, chunksize=4)):
                if progress is not None and i % 50 == 49:
                    progress(f"clusters {i + 1}/{n_clusters}")
    finally:
        _LARGE_TEXT = None
    return Genomes(text, out_len.astype(np.uint64), taxa[order], parents)


def scale_reads(genomes: Genomes, n: int = 10_000_000, seed: int = 202, progress=None) -> Reads:
    """150 bp reads, 1% substitutions, 5% foreign."""
    return sample_reads(genomes, n, 150, seed, error=0.01, foreign=0.05, progress=progress)


_READS_JOB = None   # (genomes, shared output text) while the workers of stream_reads run


def _reads_block(args) -> None:
    """Worker of :func:`stream_reads`: block b of the reads into the shared text."""
    seed, b, first, m, length, error, foreign = args
    genomes, text = _READS_JOB
    blk = sample_reads(genomes, m, length, seed * 1_000_003 + b, error=error, foreign=foreign,
                       chunk=m)
    text[first * length:(first + m) * length] = blk.text


def stream_reads(genomes: Genomes, n: int, seed: int, length: int = 150, error: float = 0.01,
                 foreign: float = 0.05, block: int = 1_000_000, workers: int = 16,
                 progress=None) -> Reads:
    """``n`` fixed-length reads (module rules) for a large read stream, drawn in
    blocks of ``block`` reads by forked workers into one shared mapping. Block
    b is drawn from its own seed, so the reads do not depend on the number of
    workers. Call it before the process touches a GPU."""
    import mmap
    import multiprocessing as mp
    import sys
    global _READS_JOB
    if _gpu_runtime_in_use():
        raise RuntimeError("stream_reads forks worker processes: call it before the process "
                           "touches a GPU or loads the HIP library")
    size = n * length
    buf = mmap.mmap(-1, max(size, 1), flags=mmap.MAP_SHARED | mmap.MAP_ANONYMOUS)
    text = np.frombuffer(buf, dtype=np.uint8, count=size)
    jobs = [(seed, b, f, min(block, n - f), length, error, foreign)
            for b, f in enumerate(range(0, n, block))]
    _READS_JOB = (genomes, text)
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            for i, _ in enumerate(pool.imap_unordered(_reads_block, jobs)):
                if progress is not None and i % 10 == 9:
                    progress(f"reads {min(n, (i + 1) * block)}/{n}")
    finally:
        _READS_JOB = None
    offsets = np.arange(n + 1, dtype=np.uint64) * np.uint64(length)
    return Reads(text, offsets, False)


def mixed_records(genomes: Genomes, n: int, seed: int = 301, error: float = 0.01,
                  foreign: float = 0.05, chunk: int = 100_000, progress=None) -> Reads:
    """Uneven batch in the paired layout.

    Half the records are single-end with length U{50..250} (empty mate 2);
    half are pairs 2 x 150 from a fragment of length round(N(400, 50))
    clipped to [150, 700] on a random strand: mate 1 reads the fragment's
    first 150 bases, mate 2 the reverse complement of its last 150.
    """
    rng = rng_for(seed)
    off_g = genomes.offsets.astype(np.int64)
    lens = genomes.lengths.astype(np.int64)
    ok = np.nonzero(lens >= 1500)[0]
    w150 = _windows(genomes.text, 150)
    w250 = _windows(genomes.text, 250)
    cols = np.arange(250, dtype=np.int32)
    texts, mlens = [], []
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        is_pair = rng.random(m) < 0.5
        is_foreign = rng.random(m) < foreign
        se_len = rng.integers(50, 251, size=m)
        frag = np.clip(np.round(rng.normal(400, 50, size=m)), 150, 700).astype(np.int64)
        span = np.where(is_pair, frag, se_len)
        gi = ok[rng.integers(0, ok.size, size=m)]
        start = off_g[gi] + 250 + (rng.random(m) * (lens[gi] - 1000)).astype(np.int64)
        rev = rng.random(m) < 0.5
        # genome segment [start, start + span); on the reverse strand the
        # fragment is its reverse complement
        head = w150[start]                       # segment's first 150 bases
        rc_tail = _COMP[w150[start + span - 150][:, ::-1]]
        m1 = head.copy()                         # fragment's first 150
        m1[rev] = rc_tail[rev]
        m2 = rc_tail                             # revcomp of fragment's last 150
        m2[rev] = head[rev]
        # single-end reads: first se_len bases of the fragment
        seg = w250[np.where(rev, start + span - 250, start)]
        seg[rev] = _COMP[seg[rev][:, ::-1]]
        nf = int(is_foreign.sum())
        if nf:
            m1[is_foreign] = random_text(rng, nf * 150).reshape(nf, 150)
            m2[is_foreign] = random_text(rng, nf * 150).reshape(nf, 150)
            seg[is_foreign] = random_text(rng, nf * 250).reshape(nf, 250)
        l1 = np.where(is_pair, 150, se_len)
        l2 = np.where(is_pair, 150, 0)
        first = np.where(is_pair[:, None], np.concatenate([m1, np.zeros((m, 100), np.uint8)], 1),
                         seg)
        keep1 = cols[None, :] < l1[:, None]
        keep2 = cols[None, :150] < l2[:, None]
        # interleave mate 1 and mate 2 per record
        both = np.concatenate([first, m2], axis=1)
        keep = np.concatenate([keep1, keep2], axis=1)
        texts.append(substitute(rng, both[keep], error))
        ml = np.empty(2 * m, dtype=np.int64)
        ml[0::2] = l1
        ml[1::2] = l2
        mlens.append(ml)
        if progress is not None and (c0 // chunk) % 20 == 19:
            progress(f"records {c0 + m}/{n}")
    ml = np.concatenate(mlens) if mlens else np.zeros(0, np.int64)
    off = np.zeros(ml.size + 1, dtype=np.uint64)
    np.cumsum(ml, out=off[1:])
    text = np.concatenate(texts) if texts else np.zeros(0, np.uint8)
    return Reads(text, off, True)


def repeated_genome(n_copies: int, length: int, seed: int) -> Genomes:
    """``n_copies`` identical genomes (stress input for the per-feature cap)."""
    rng = rng_for(seed)
    g = random_text(rng, length)
    text = np.tile(g, n_copies)
    lengths = np.full(n_copies, length, dtype=np.uint64)
    parents = np.zeros(1 + n_copies, dtype=np.uint32)
    taxa = np.arange(1, 1 + n_copies, dtype=np.uint32)
    return Genomes(text, lengths, taxa, parents)


def arrival_trace(n_batches: int, seed: int, lo: float = 1e3, hi: float = 1e6,
                  rate_hz: float = 100.0) -> tuple[np.ndarray, np.ndarray]:
    """Poisson arrival times (s) and log-uniform batch sizes (reads)."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_batches)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_batches)).astype(np.int64)
    return np.cumsum(gaps), sizes


def sample_reads_varlen(genomes: Genomes, n: int, lo: int, hi: int, seed: int,
                        error: float = 0.01, foreign: float = 0.0,
                        chunk: int = 100_000) -> Reads:
    """``n`` single-end reads with lengths uniform in {lo..hi} (module rules)."""
    rng = rng_for(seed)
    off_g = genomes.offsets.astype(np.int64)
    lens = genomes.lengths.astype(np.int64)
    ok = np.nonzero(lens >= 3 * hi)[0]
    rows = _windows(genomes.text, hi)
    pieces, all_len = [], []
    cols = np.arange(hi, dtype=np.int32)
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        L = rng.integers(lo, hi + 1, size=m)
        gi = ok[rng.integers(0, ok.size, size=m)]
        is_foreign = rng.random(m) < foreign
        # fragment [start, start + L) with start uniform in [hi, len - 2 hi]
        start = hi + (rng.random(m) * (lens[gi] - 3 * hi + 1)).astype(np.int64)
        rev = rng.random(m) < 0.5
        first = off_g[gi] + start
        # reverse strand: the hi-window ending at the fragment end, reversed
        block = rows[np.where(rev, first + L - hi, first)]
        block[rev] = _COMP[block[rev][:, ::-1]]
        nf = int(is_foreign.sum())
        if nf:
            block[is_foreign] = random_text(rng, nf * hi).reshape(nf, hi)
        keep = cols[None, :] < L[:, None]
        flat = substitute(rng, block[keep], error)
        pieces.append(flat)
        all_len.append(L)
    lengths = np.concatenate(all_len) if all_len else np.zeros(0, np.int64)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    text = np.concatenate(pieces) if pieces else np.zeros(0, np.uint8)
    return Reads(text, offsets, False)


def addition_genomes(base: Genomes, n_clusters: int, per_cluster: int, total_bp: float,
                     seed: int, first_taxon_node: int | None = None) -> tuple[Genomes, np.ndarray]:
    """New genomes for an on-demand addition and the extended parent array.

    The new clusters hang under existing level-1 nodes of ``base``'s taxonomy
    (children of its root); their cluster, group and leaf nodes get new ids
    after the existing ones. Returns the new genomes (taxa in the extended
    numbering) and the extended parents.
    """
    add = clustered_genomes(n_clusters, per_cluster, total_bp, seed, level1=1)
    root = int(np.nonzero(base.parents == np.arange(base.parents.size))[0][0])
    level1 = np.nonzero((base.parents == root) & (np.arange(base.parents.size) != root))[0]
    start = base.parents.size if first_taxon_node is None else first_taxon_node
    n_new = add.parents.size - 2            # drop the small set's root and level-1 node
    mapping = np.zeros(add.parents.size, dtype=np.int64)
    mapping[0] = root
    rng = rng_for(seed + 1)
    mapping[1] = int(level1[rng.integers(0, level1.size)]) if level1.size else root
    mapping[2:] = np.arange(start, start + n_new)
    parents = np.concatenate([base.parents, np.zeros(n_new, dtype=np.uint32)])
    parents[start:start + n_new] = mapping[add.parents[2:]].astype(np.uint32)
    taxa = mapping[add.taxa].astype(np.uint32)
    return Genomes(add.text, add.lengths, taxa, parents), parents
