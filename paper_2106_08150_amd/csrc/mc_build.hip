// Database build kernels (Sec. 4.1, Sec. 5.1-5.3): encode + canonical k-mers +
// h1 + bottom-s sketch per window + insertion into the bucketed multi-value
// table, the deterministic per-feature cap, table growth and test exports.
#include <algorithm>

#include "mc_device.hpp"
#include "mc_internal.hpp"

namespace mc {

namespace {

constexpr int kWavesPerBuild = kBuildThreads / kWave;
constexpr int kMaxSketch = 64;
// words of one tile: (kTileWindows-1) strides of at most 256 bases plus one
// window of at most 271 bases, 16 bases per word, plus alignment and one
// look-ahead word.
constexpr int kTileWordsMax = ((kTileWindows - 1) * 256 + 271 + 15) / 16 + 3;

struct SketchLds {
    Word words[kTileWordsMax];
    uint32_t scratch[kWavesPerBuild][kWave];
    uint32_t feats[kWavesPerBuild][2 * kMaxSketch];   // sketches of a window pair
    uint32_t hist[kScatGroups * kMaxParts];
};

// Partition of a feature: its home bucket >> part_shift, so partition p holds
// the features whose home buckets form the p-th contiguous range of the table.
__device__ __forceinline__ uint32_t part_of(uint32_t f, uint64_t nb, uint32_t shift) {
    return (uint32_t)(home_bucket(f, nb) >> shift);
}

// Sketch every window of the call (B1-B4). One workgroup stages a tile of 32
// consecutive windows of one target as 2-bit words in LDS; each wave sketches
// every fourth window of the tile.
//   kPairs = false: out_counts[w] and out_feats[w*s ..] per window (export).
//   kPairs = true:  pairs[w*s + i] = feature << 32 | location for i < n and
//                   empty for n <= i < s, plus a histogram of the pairs' table
//                   partitions per scatter group (the group of a tile's pairs
//                   is that of the level-1 scatter chunk holding the tile).
//
// Eight waves a SIMD: left unbounded, the kernel takes 106 scalar registers
// and fewer waves fit; the scalar spills that the 8-wave budget costs are
// cheaper than the lost latency hiding (10.6 -> 9.9 ms on a 4 Gbp build).
template <int KPL, bool kPairs>
__global__ __launch_bounds__(kBuildThreads) __attribute__((amdgpu_waves_per_eu(8)))
void k_sketch(BuildArgs a) {
    __shared__ SketchLds L;
    const int tid = threadIdx.x;
    // the wave index in a scalar register: the window loop and its bounds
    // are then wave-uniform
    const int wave = (int)uniform((uint32_t)tid >> 6), lane = tid & 63;
    const Threshold th(a.S, a.s);
    if (kPairs) {
        for (uint32_t p = tid; p < kScatGroups * kMaxParts; p += kBuildThreads) L.hist[p] = 0;
    }
    for (uint64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        // target of this tile: last t with tile_first[t] <= tile
        uint32_t lo = 0, hi = a.n_targets;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (a.tile_first[mid] <= tile) lo = mid; else hi = mid;
        }
        const TargetDesc td = a.targets[lo];
        const uint32_t hbase = (uint32_t)((tile / a.chunk_tiles) % kScatGroups) * kMaxParts;
        const uint32_t j0 = (uint32_t)(tile - a.tile_first[lo]) * kTileWindows;
        const uint32_t nwin = min((uint32_t)kTileWindows, td.nw - j0);
        if (kPairs && tid == 0) {   // slot bounds of the level-1 scatter chunks
            if (tile % a.chunk_tiles == 0) a.chunk_slot[tile / a.chunk_tiles] = (td.win_base + j0) * a.s;
            if (tile + 1 == a.n_tiles)
                a.chunk_slot[(a.n_tiles + a.chunk_tiles - 1) / a.chunk_tiles] =
                    (td.win_base + j0 + nwin) * a.s;
        }
        const uintptr_t tstart = (uintptr_t)(a.text + td.off);
        const uintptr_t tend = tstart + td.len;
        const uintptr_t blo = tstart + (uint64_t)j0 * a.S;
        uintptr_t bhi = tstart + (uint64_t)(j0 + nwin - 1) * a.S + a.w;
        if (bhi > tend) bhi = tend;
        __syncthreads();
        // a tile without a non-base byte (the common case) skips the
        // per-k-mer validity test
        const bool dirty =
            __syncthreads_or(stage_words(L.words, blo, bhi, tstart, tend, tid, kBuildThreads));
        const uintptr_t A0 = blo & ~(uintptr_t)15;
        const uint64_t n_starts = td.len - a.k + 1;
        // each wave sketches pairs of windows (2i, 2i+1) of the tile
        for (uint32_t wv = 2u * (uint32_t)wave; wv < nwin; wv += 2u * kWavesPerBuild) {
            uint32_t nk[2], x0[2];
            for (int h = 0; h < 2; ++h) {
                const uint32_t j = j0 + wv + (uint32_t)h;
                const uint64_t first = (uint64_t)j * a.S;
                nk[h] = wv + h < nwin ? (uint32_t)min((uint64_t)a.S, n_starts - first) : 0u;
                x0[h] = wv + h < nwin ? (uint32_t)(tstart + first - A0) : 0u;
            }
            uint32_t* sk = L.feats[wave];
            uint32_t n[2];
            sketch_pair<KPL, true>(L.words, x0[0], nk[0], L.words, x0[1], nk[1], a.k, a.s, th, sk,
                             sk + kMaxSketch, L.scratch[wave], n[0], n[1], dirty, dirty);
            wave_lds_sync();
            // entry e of the pair: window e / s, sketch slot e % s
            const uint32_t npair = wv + 1 < nwin ? 2u : 1u;
            for (uint32_t e = (uint32_t)lane; e < npair * a.s; e += kWave) {
                const uint32_t h = e >= a.s ? 1u : 0u, i = e - h * a.s;
                const uint32_t j = j0 + wv + h;
                const uint64_t gw = td.win_base + j;
                const uint32_t nh = h ? n[1] : n[0];
                if (kPairs) {
                    uint64_t pe = kEmpty;
                    if (i < nh) {
                        const uint32_t f = sk[h * kMaxSketch + i];
                        pe = ((uint64_t)f << 32) | ((td.id << kWindowBits) | j);
                        atomicAdd(&L.hist[hbase + part_of(f, a.nb, a.part_shift)], 1u);
                    }
                    a.pairs[gw * a.s + i] = pe;
                } else {
                    if (i == 0) a.out_counts[gw] = nh;
                    if (i < nh) a.out_feats[gw * a.s + i] = sk[h * kMaxSketch + i];
                }
            }
            wave_lds_sync();
        }
    }
    if (kPairs) {
        __syncthreads();
        for (uint32_t i = tid; i < kScatGroups * kMaxParts; i += kBuildThreads)
            if (L.hist[i]) atomicAdd(&a.hist[i], L.hist[i]);
    }
}

// Exclusive scan of one value per thread over a 256-thread workgroup; returns
// the thread's exclusive prefix and sets total.
__device__ __forceinline__ unsigned long long block_scan256(unsigned long long v,
                                                            unsigned long long* wsum,
                                                            unsigned long long& total) {
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    unsigned long long x = v;      // inclusive wave scan
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t lo = shfl_idx((uint32_t)x, lane >= (uint32_t)d ? lane - d : lane);
        uint32_t hi = shfl_idx((uint32_t)(x >> 32), lane >= (uint32_t)d ? lane - d : lane);
        if (lane >= (uint32_t)d) x += ((unsigned long long)hi << 32) | lo;
    }
    __syncthreads();
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    unsigned long long base = 0;
    for (uint32_t i = 0; i < w; ++i) base += wsum[i];
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    return base + x - v;
}

constexpr uint32_t kHistChunk = 65536;   // pairs per histogram chunk (slice mode)
constexpr uint32_t kNoKey = 0xFFFFFFFFu;  // register-held entry without a key

// Exclusive scan of the partition histogram (one workgroup of 256 threads):
// part_start[p], and the cursor of each scatter group within partition p
// (groups in order). In slice mode also the prefix of histogram and scatter
// chunks per partition (chunks never straddle two partitions) and the most
// scatter chunks of any partition.
__global__ __launch_bounds__(kMaxParts) void k_scan_parts(BuildArgs a) {
    __shared__ unsigned long long wsum[kMaxParts / kWave];
    __shared__ unsigned long long cmax;
    const uint32_t t = threadIdx.x, P = a.n_parts;
    unsigned long long v = 0;
    if (t < P)
        for (uint32_t g = 0; g < kScatGroups; ++g) v += a.hist[g * kMaxParts + t];
    unsigned long long total;
    const unsigned long long excl = block_scan256(v, wsum, total);
    if (t < P) {
        a.part_start[t] = excl;
        unsigned long long run = excl;
        for (uint32_t g = 0; g < kScatGroups; ++g) {
            a.cursor[g * kMaxParts + t] = run;
            run += a.hist[g * kMaxParts + t];
        }
    }
    if (t == 0) a.part_start[P] = total;
    if (!a.slice_mode) return;
    const unsigned long long ch = t < P ? (v + kHistChunk - 1) / kHistChunk : 0ull;
    const unsigned long long cs = t < P ? (v + kScatChunk - 1) / kScatChunk : 0ull;
    unsigned long long th, ts;
    const unsigned long long eh = block_scan256(ch, wsum, th);
    const unsigned long long es = block_scan256(cs, wsum, ts);
    if (t == 0) cmax = 0;
    __syncthreads();
    if (cs) atomicMax(&cmax, cs);
    __syncthreads();
    if (t < P) {
        a.chunk_first[t] = eh;
        a.chunk_first[kMaxParts + 1 + t] = es;
    }
    if (t == 0) {
        a.chunk_first[P] = th;
        a.chunk_first[kMaxParts + 1 + P] = ts;
        a.chunk_first[kChunkMaxAt] = cmax;
    }
}

// Exclusive prefix sums of one u32 per thread over a kScatThreads workgroup.
__device__ __forceinline__ uint32_t block_scan1024(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = shfl_idx(x, lane >= (uint32_t)d ? (int)lane - d : (int)lane);
        if (lane >= (uint32_t)d) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t base = 0;
    total = 0;
    for (uint32_t i = 0; i < (uint32_t)(kScatThreads / kWave); ++i) {
        const uint32_t y = wsum[i];
        if (i < w) base += y;
        total += y;
    }
    return base + x - v;
}

constexpr uint32_t kMaxBins = 1u << kMaxFineBits;   // bins of one scatter (>= kMaxParts)
static_assert(kMaxBins >= kMaxParts && kMaxBins <= (uint32_t)kScatThreads, "one thread a bin");

struct ScatLds {
    unsigned long long buf[kScatChunk];   // the chunk's pairs, sorted by bin
    uint32_t hist[kMaxBins], lstart[kMaxBins];
    unsigned long long gbase[kMaxBins];
    uint32_t wsum[kScatThreads / kWave];
};

// One chunk of a scatter: entries in[c0, c1) (1 <= c1 - c0 <= kScatChunk) and
// the cursors of its bins.
struct ScatChunk {
    uint64_t c0, c1;
    unsigned long long* cursor;
};

// A chunk's entries into registers, kScatPer a thread (past the end: a repeat
// of the last entry).
__device__ __forceinline__ void scat_load(const unsigned long long* in, const ScatChunk& c,
                                          uint32_t t, unsigned long long (&e)[kScatPer]) {
    const uint32_t n = (uint32_t)(c.c1 - c.c0);
#pragma unroll
    for (int j = 0; j < kScatPer; ++j) e[j] = in[c.c0 + min((uint32_t)j * kScatThreads + t, n - 1)];
}

// Scatter the chunks that next() yields (kEmpty entries are skipped) into
// nbins <= kMaxBins bins: each thread holds kScatPer entries in registers and
// ranks them within their bin with an LDS counter; the workgroup reserves one
// run per bin with an atomic on that bin's cursor, sorts the entries by bin in
// LDS and writes the runs out contiguously (counting sort). The cursor atomics
// are in flight while the chunk is sorted into LDS, and the next chunk's loads
// while this one is written out. bin_of is evaluated again for the write
// instead of being stored.
template <typename NextFn, typename BinOf>
__device__ __forceinline__ void scatter_chunks(const unsigned long long* in, NextFn next,
                                               BinOf bin_of, uint32_t nbins,
                                               unsigned long long* out, ScatLds& S) {
    const uint32_t t = threadIdx.x;
    ScatChunk cur;
    bool have = next(cur);
    unsigned long long e[kScatPer];
    if (have) scat_load(in, cur, t, e);
    while (have) {
        ScatChunk nxt;
        const bool have_next = next(nxt);
        const uint32_t n = (uint32_t)(cur.c1 - cur.c0);
        if (t < nbins) S.hist[t] = 0;
        __syncthreads();                   // also: the previous chunk's write-out is done
        uint32_t key[kScatPer];            // bin << 16 | rank within the bin, or kNoKey
#pragma unroll
        for (int j = 0; j < kScatPer; ++j)
            key[j] = (uint32_t)j * kScatThreads + t < n && e[j] != kEmpty ? 0u : kNoKey;
#pragma unroll
        for (int j = 0; j < kScatPer; ++j) {
            if (key[j] == 0u) {
                const uint32_t b = bin_of(e[j]);
                key[j] = (b << 16) | atomicAdd(&S.hist[b], 1u);
            }
        }
        __syncthreads();
        const uint32_t v = t < nbins ? S.hist[t] : 0u;
        uint32_t total;
        const uint32_t excl = block_scan1024(v, S.wsum, total);
        unsigned long long g = 0ull;
        if (t < nbins) {
            S.lstart[t] = excl;
            if (v) g = atomicAdd(&cur.cursor[t], (unsigned long long)v);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScatPer; ++j)
            if (key[j] != kNoKey) S.buf[S.lstart[key[j] >> 16] + (key[j] & 0xFFFFu)] = e[j];
        if (t < nbins) S.gbase[t] = g;
        __syncthreads();
        if (have_next) scat_load(in, nxt, t, e);
        for (uint32_t i = t; i < total; i += kScatThreads) {
            const unsigned long long x = S.buf[i];
            const uint32_t b = bin_of(x);
            out[S.gbase[b] + (i - S.lstart[b])] = x;
        }
        cur = nxt;
        have = have_next;
    }
}

// Level 1: the per-window pairs into partition order (parted). Chunk m is
// the slots of sketch tiles [m * chunk_tiles, (m + 1) * chunk_tiles) and
// takes its runs from cursor set m % kScatGroups.
__global__ __launch_bounds__(kScatThreads) void k_scatter(BuildArgs a) {
    __shared__ ScatLds S;
    const uint64_t nb = a.nb;
    const uint32_t sh = a.part_shift;
    const uint64_t n_chunks = (a.n_tiles + a.chunk_tiles - 1) / a.chunk_tiles;
    uint64_t m = blockIdx.x;
    auto next = [&](ScatChunk& c) -> bool {
        for (; m < n_chunks; m += gridDim.x) {
            const uint64_t c0 = a.chunk_slot[m], c1 = a.chunk_slot[m + 1];
            if (c1 > c0) {
                c = ScatChunk{c0, c1, a.cursor + (m % kScatGroups) * kMaxParts};
                m += gridDim.x;
                return true;
            }
        }
        return false;
    };
    scatter_chunks(a.pairs, next,
                   [=](unsigned long long e) { return part_of((uint32_t)(e >> 32), nb, sh); },
                   a.n_parts, a.parted, S);
}

// Partition of chunk ci of the prefix first[0..P] (first[P] = number of chunks).
__device__ __forceinline__ uint32_t chunk_part(const unsigned long long* first, uint32_t P,
                                               uint64_t ci) {
    uint32_t lo = 0, hi = P;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (first[mid] <= ci) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t fine_of(unsigned long long e, uint64_t nb, uint32_t shift,
                                            uint32_t mask) {
    return (uint32_t)(home_bucket((uint32_t)(e >> 32), nb) >> shift) & mask;
}

// Slice mode, level 2 histogram: pairs per slice within each partition.
__global__ __launch_bounds__(kBuildThreads) void k_hist2(BuildArgs a) {
    __shared__ uint32_t h[kMaxBins];
    const uint32_t t = threadIdx.x, P = a.n_parts;
    const uint32_t mask = (1u << a.fine_bits) - 1u;
    const uint64_t n_chunks = a.chunk_first[P];
    for (uint64_t ci = blockIdx.x; ci < n_chunks; ci += gridDim.x) {
        const uint32_t p = chunk_part(a.chunk_first, P, ci);
        const uint64_t c0 = a.part_start[p] + (ci - a.chunk_first[p]) * kHistChunk;
        const uint64_t end = a.part_start[p + 1];
        const uint64_t c1 = c0 + kHistChunk < end ? c0 + kHistChunk : end;
        for (uint32_t b = t; b <= mask; b += kBuildThreads) h[b] = 0;
        __syncthreads();
        constexpr int U = 8;   // independent loads in flight a thread
        for (uint64_t i0 = c0 + t; i0 < c1; i0 += U * kBuildThreads) {
            unsigned long long x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i = i0 + (uint64_t)u * kBuildThreads;
                x[u] = a.parted[i < c1 ? i : c1 - 1];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + (uint64_t)u * kBuildThreads < c1)
                    atomicAdd(&h[fine_of(x[u], a.nb, a.slice_shift, mask)], 1u);
        }
        __syncthreads();
        for (uint32_t b = t; b <= mask; b += kBuildThreads)
            if (h[b]) atomicAdd(&a.hist2[(p << a.fine_bits) + b], h[b]);
        __syncthreads();
    }
}

// Slice mode: exclusive scan of the n_parts << fine_bits slice counts (one
// workgroup, 256 consecutive slices per thread).
__global__ __launch_bounds__(kBuildThreads) void k_scan2(BuildArgs a) {
    __shared__ unsigned long long wsum[kBuildThreads / kWave];
    const uint32_t t = threadIdx.x;
    const uint32_t n = a.n_parts << a.fine_bits;
    const uint32_t per = (n + kBuildThreads - 1) / kBuildThreads;
    const uint32_t i0 = min(n, t * per), i1 = min(n, i0 + per);
    unsigned long long sum = 0;
    for (uint32_t i = i0; i < i1; ++i) sum += a.hist2[i];
    unsigned long long total;
    unsigned long long run = block_scan256(sum, wsum, total);
    for (uint32_t i = i0; i < i1; ++i) {
        a.slice_start[i] = run;
        a.cursor2[i] = run;
        run += a.hist2[i];
    }
    if (t == 0) a.slice_start[n] = total;
}

// Slice mode, level 2: parted (partition order) into slice order (pairs).
// Work item q is chunk q / P of partition q % P, so the chunks in flight
// belong to different partitions and reserve their runs on different cursors.
__global__ __launch_bounds__(kScatThreads) void k_scatter2(BuildArgs a) {
    __shared__ ScatLds S;
    const uint32_t P = a.n_parts;
    const unsigned long long* first = a.chunk_first + kMaxParts + 1;
    const uint64_t n_items = a.chunk_first[kChunkMaxAt] * P;
    const uint64_t nb = a.nb;
    const uint32_t sh = a.slice_shift, mask = (1u << a.fine_bits) - 1u;
    uint64_t q = blockIdx.x;
    auto next = [&](ScatChunk& c) -> bool {
        for (; q < n_items; q += gridDim.x) {
            const uint32_t p = (uint32_t)(q % P);
            const uint64_t r = q / P;
            if (r >= first[p + 1] - first[p]) continue;
            const uint64_t c0 = a.part_start[p] + r * kScatChunk;
            const uint64_t end = a.part_start[p + 1];
            const uint64_t c1 = c0 + kScatChunk < end ? c0 + kScatChunk : end;
            if (c1 > c0) {
                c = ScatChunk{c0, c1, a.cursor2 + ((uint64_t)p << a.fine_bits)};
                q += gridDim.x;
                return true;
            }
        }
        return false;
    };
    scatter_chunks(a.parted, next,
                   [=](unsigned long long e) { return fine_of(e, nb, sh, mask); }, mask + 1u,
                   a.pairs, S);
}

// Insert one entry (B5). Every bucket has a fill counter; an insert claims
// slot `pos` of its bucket with one atomic increment and stores the entry
// there. A counter at 16 or more means the bucket is full and the entry moves
// on to the next bucket, so every entry of a feature lies between its home
// bucket and the first bucket that still has an empty slot (counters only
// grow, so a stale read of a full counter is still a full bucket).
// Returns the number of buckets moved past, or nb + 1 if none had room.
__device__ __forceinline__ uint64_t insert_one(unsigned long long* table, uint32_t* bcount,
                                               uint64_t nb, uint64_t b, unsigned long long e) {
    for (uint64_t d = 0; d <= nb; ++d) {
        if (bcount[b] < (uint32_t)kSlots) {
            uint32_t pos = atomicAdd(&bcount[b], 1u);
            if (pos < (uint32_t)kSlots) {
                table[b * kSlots + pos] = e;
                return d;
            }
        }
        b = next_bucket(b, nb);
    }
    return nb + 1;
}

// Adds a workgroup's insert statistics to the build counters.
__device__ __forceinline__ void add_insert_stats(BuildArgs& a, uint32_t ins, uint32_t probe,
                                                 uint32_t full, uint32_t* red) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        ins += shfl_xor(ins, m);
        probe += shfl_xor(probe, m);
        full += shfl_xor(full, m);
    }
    __syncthreads();
    if (lane == 0) {
        red[0 * kWavesPerBuild + wave] = ins;
        red[1 * kWavesPerBuild + wave] = probe;
        red[2 * kWavesPerBuild + wave] = full;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t v = 0;
        for (int w = 0; w < kWavesPerBuild; ++w) v += red[threadIdx.x * kWavesPerBuild + w];
        const int idx[3] = {kCntInserted, kCntProbe, kCntFull};
        if (v) atomicAdd(&a.counters[idx[threadIdx.x]], (unsigned long long)v);
    }
}

__device__ __forceinline__ void push_candidate(BuildArgs& a, uint32_t f) {
    unsigned long long c = atomicAdd(&a.counters[kCntCand], 1ull);
    if (c < a.cand_cap) a.cand[c] = f;
}

// B5: insert src[0, *n) with the global bucket counters, one entry per lane.
// A persistent grid of resident workgroups takes the entries in order (entry
// = thread slot + i * threads in the grid); with partition-ordered entries
// the threads in flight all work in one range of the table, whose counters
// stay in L2 and lines in the Infinity Cache.
__global__ __launch_bounds__(kBuildThreads) void k_insert(BuildArgs a,
                                                          const unsigned long long* src,
                                                          const unsigned long long* n_ptr) {
    __shared__ uint32_t red[3 * kWavesPerBuild];
    const uint64_t n = *n_ptr;
    uint32_t ins = 0, probe = 0, full = 0;
    const uint64_t step = (uint64_t)gridDim.x * kBuildThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kBuildThreads + threadIdx.x; i < n; i += step) {
        const unsigned long long e = src[i];
        const uint32_t f = (uint32_t)(e >> 32);
        const uint64_t d = insert_one(a.table, a.bcount, a.nb, home_bucket(f, a.nb), e);
        if (d > a.nb) {
            full += 1;
            continue;
        }
        ins += 1;
        probe += (uint32_t)d;
        if (d >= a.cap_dist) push_candidate(a, f);
    }
    add_insert_stats(a, ins, probe, full, red);
}

// B5, slice mode: workgroup z inserts the pairs of slice z (buckets
// [z << slice_shift, (z + 1) << slice_shift), the pairs in slice order); no
// other workgroup touches those buckets meanwhile. The workgroup reads the
// slice's pairs once into registers, ranks each within its home bucket with
// an LDS counter, and places them as the global-counter insert would (each
// pair in the first bucket from its home with a free slot, the slots of a
// bucket filled in order): with d(r) = pairs homed at r minus free slots of
// r, the pairs carried past bucket r are carry(r) = max(0, carry(r-1) + d(r)),
// a max-plus scan across the slice, and buckets <= r hold the first
// N(r) - carry(r) pairs in home order (N = inclusive count). The placed pairs
// are staged in LDS in home order. In a new table every bucket is written as
// one whole 128-byte line (its new pairs, then empty slots), so the table
// sees full-line writes only; in a table that holds entries only the slots
// that gain pairs are written. Pairs carried past the slice end are
// deferred to the global pass (k_insert). A slice with more pairs than the
// registers hold takes the direct path: LDS fill counters, one store a pair.
constexpr int kLineThreads = 1024;
constexpr int kLineWaves = kLineThreads / kWave;
constexpr int kLinePer = 24;                        // pairs per thread held in registers
constexpr uint32_t kLineCap = (uint32_t)kLineThreads * kLinePer;
static_assert(kLineCap < 0x10000, "sorted positions are kept in 16 bits");

__device__ __forceinline__ void defer_pair(BuildArgs& a, unsigned long long e) {
    const unsigned long long q = atomicAdd(&a.counters[kCntDefer], 1ull);
    a.parted[q] = e;
}

__device__ __forceinline__ uint32_t free_slots(uint8_t c) { return (uint32_t)kSlots - c; }

// Direct path of one slice: LDS fill counters, each pair claims a slot.
__device__ __forceinline__ void insert_slice_direct(BuildArgs& a, uint32_t* cnt, uint64_t b0,
                                                    uint32_t nbk, uint64_t p0, uint64_t p1,
                                                    uint32_t& ins, uint32_t& probe) {
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < nbk; i += kLineThreads) cnt[i] = a.fresh ? 0u : a.bcount[b0 + i];
    __syncthreads();
    for (uint64_t i = p0 + tid; i < p1; i += kLineThreads) {
        const unsigned long long e = a.pairs[i];
        const uint32_t f = (uint32_t)(e >> 32);
        const uint32_t h = (uint32_t)(home_bucket(f, a.nb) - b0);
        uint32_t r = h;
        bool done = false;
        for (; r < nbk && !done; ++r) {
            if (cnt[r] < (uint32_t)kSlots) {
                const uint32_t pos = atomicAdd(&cnt[r], 1u);
                if (pos < (uint32_t)kSlots) {
                    a.table[(b0 + r) * kSlots + pos] = e;
                    done = true;
                }
            }
        }
        if (done) {
            const uint32_t dist = r - 1 - h;
            ins += 1;
            probe += dist;
            if (dist >= a.cap_dist) push_candidate(a, f);
        } else {
            defer_pair(a, e);
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < nbk; i += kLineThreads) a.bcount[b0 + i] = cnt[i];
    if (a.fresh) {   // slots no pair claimed (disjoint from the stores above)
        for (uint32_t i = tid; i < nbk * kSlots; i += kLineThreads)
            if (i % kSlots >= min(cnt[i / kSlots], (uint32_t)kSlots))
                a.table[b0 * kSlots + i] = kEmpty;
    }
}

// A fresh slice without pairs: empty lines, zero counters.
__device__ __forceinline__ void clear_slice(BuildArgs& a, uint64_t b0, uint32_t nbk) {
    for (uint32_t i = threadIdx.x; i < nbk * kSlots; i += kLineThreads) a.table[b0 * kSlots + i] = kEmpty;
    for (uint32_t i = threadIdx.x; i < nbk; i += kLineThreads) a.bcount[b0 + i] = 0u;
}

__global__ __launch_bounds__(kLineThreads) void k_insert_slices(BuildArgs a, uint32_t buf_cap,
                                                                uint32_t line_cap) {
    // dynamic LDS: buf[buf_cap] u64 (counters while counting, staged pairs
    // while writing), then per bucket: Te u16, Tp u16, c8 u8
    extern __shared__ unsigned long long buf[];
    __shared__ uint32_t wsum[kLineWaves];
    __shared__ int wA[kLineWaves], wD[kLineWaves];
    __shared__ uint32_t red[2 * kLineWaves];
    const uint32_t SB = 1u << a.slice_shift;
    uint32_t* const cnt = reinterpret_cast<uint32_t*>(buf);
    uint16_t* const Te = reinterpret_cast<uint16_t*>(buf + buf_cap);   // first position homed at r
    uint16_t* const Tp = Te + SB;                                      // pairs placed in buckets <= r
    uint8_t* const c8 = reinterpret_cast<uint8_t*>(Tp + SB);           // slots in use before
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t n_slices = a.n_parts << a.fine_bits;
    const int kNone = -(1 << 30);
    uint32_t ins = 0, probe = 0;
    for (uint32_t z = blockIdx.x; z < n_slices; z += gridDim.x) {
        const uint64_t b0 = (uint64_t)z << a.slice_shift;
        if (b0 >= a.nb) break;            // slices past the table are empty
        const uint32_t nbk = (uint32_t)(b0 + SB <= a.nb ? SB : a.nb - b0);
        const uint64_t p0 = a.slice_start[z], p1 = a.slice_start[z + 1];
        const uint32_t np = (uint32_t)(p1 - p0);
        if (np == 0) {
            if (a.fresh) clear_slice(a, b0, nbk);
            continue;
        }
        __syncthreads();                  // LDS of the previous slice is free
        if (np > line_cap) {
            insert_slice_direct(a, cnt, b0, nbk, p0, p1, ins, probe);
            continue;
        }
        // per-thread indices recomputed each slice (not held across the loop)
        uint32_t t = tid;
        asm volatile("" : "+v"(t));
        const uint32_t ln = t & 63;
        for (uint32_t i = tid; i < nbk; i += kLineThreads) {
            cnt[i] = 0u;
            c8[i] = a.fresh ? (uint8_t)0 : (uint8_t)min(a.bcount[b0 + i], (uint32_t)kSlots);
        }
        __syncthreads();
        // the slice's pairs, each ranked within its home bucket
        unsigned long long e[kLinePer];
        uint32_t key[kLinePer];
#pragma unroll
        for (int k = 0; k < kLinePer; ++k) {   // past the end: a repeat of the last pair, no key
            const uint32_t i = t + (uint32_t)k * kLineThreads;
            e[k] = a.pairs[p0 + min(i, np - 1)];
            key[k] = i < np ? 0u : kNoKey;
        }
#pragma unroll
        for (int k = 0; k < kLinePer; ++k) {
            if (key[k] == 0u) {
                const uint32_t r = (uint32_t)(home_bucket((uint32_t)(e[k] >> 32), a.nb) - b0);
                if (r < nbk) {
                    key[k] = (r << 16) | atomicAdd(&cnt[r], 1u);
                } else {
                    key[k] = kNoKey;
                    defer_pair(a, e[k]);    // not homed in this slice (does not occur)
                }
            }
        }
        __syncthreads();
        // per-thread run of buckets: count sum and carry function max(A, x + D)
        const uint32_t per = (nbk + kLineThreads - 1) / kLineThreads;
        const uint32_t r0 = min(nbk, t * per), r1 = min(nbk, r0 + per);
        uint32_t S = 0;
        int A = kNone, D = 0;
        for (uint32_t r = r0; r < r1; ++r) {
            const int d = (int)cnt[r] - (int)free_slots(c8[r]);
            S += cnt[r];
            A = max(0, A + d);
            D += d;
        }
        // inclusive scan within the wave (a later run composed after an earlier one)
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int src = ln >= (uint32_t)d ? (int)ln - d : (int)ln;
            const uint32_t pS = shfl_idx(S, src);
            const int pA = (int)shfl_idx((uint32_t)A, src), pD = (int)shfl_idx((uint32_t)D, src);
            if (ln >= (uint32_t)d) {
                S += pS;
                A = max(A, pA + D);
                D += pD;
            }
        }
        const int up = ln ? (int)ln - 1 : 0;
        uint32_t eS = shfl_idx(S, up);
        int eA = (int)shfl_idx((uint32_t)A, up), eD = (int)shfl_idx((uint32_t)D, up);
        if (ln == 0) {
            eS = 0;
            eA = kNone;
            eD = 0;
        }
        if (ln == kWave - 1) {
            wsum[w] = S;
            wA[w] = A;
            wD[w] = D;
        }
        __syncthreads();
        uint32_t PS = 0;
        int PA = kNone, PD = 0;
        for (uint32_t i = 0; i < w; ++i) {
            PS += wsum[i];
            PA = max(wA[i], PA + wD[i]);
            PD += wD[i];
        }
        uint32_t run = PS + eS;                          // pairs homed before r0
        int carry = max(0, max(max(eA, PA + eD), PD + eD));   // carried into r0
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t n = cnt[r];
            Te[r] = (uint16_t)run;
            run += n;
            carry = max(0, carry + (int)n - (int)free_slots(c8[r]));
            Tp[r] = (uint16_t)(run - (uint32_t)carry);
        }
        __syncthreads();
        const uint32_t placed_all = Tp[nbk - 1];
        // home-order positions; pairs beyond the placed ones leave the slice
#pragma unroll
        for (int k = 0; k < kLinePer; ++k) {
            if (key[k] != kNoKey) {
                const uint32_t j = Te[key[k] >> 16] + (key[k] & 0xFFFFu);
                key[k] = j;
                if (j >= placed_all) {
                    defer_pair(a, e[k]);
                    key[k] = kNoKey;
                }
            }
        }
        const uint32_t sl = tid & (kSlots - 1);
        unsigned long long* const tab = a.table + b0 * kSlots;   // the slice's lines
        uint32_t* const cnt_out = a.bcount + b0;
        if (a.fresh) {   // buckets that gain no pair: empty lines, zero counters
            for (uint32_t r = tid / kSlots; r < nbk; r += kLineThreads / kSlots) {
                if (Tp[r] != (r ? Tp[r - 1] : 0u)) continue;
                tab[r * kSlots + sl] = kEmpty;
                if (sl == 0) cnt_out[r] = 0u;
            }
        }
        // rounds: positions [W, W + buf_cap) staged; buckets starting in [W, W + step)
        const uint32_t step = buf_cap - kSlots;
        for (uint32_t W = 0; W < placed_all; W += step) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kLinePer; ++k)
                if (key[k] - W < buf_cap) buf[key[k] - W] = e[k];   // kNoKey never
            __syncthreads();
            for (uint32_t r = tid / kSlots; r < nbk; r += kLineThreads / kSlots) {
                const uint32_t st = r ? Tp[r - 1] : 0u, placed = Tp[r] - st;
                if (placed == 0 || st - W >= step) continue;
                // a new table's line is written whole (new pairs, then empty
                // slots); in a table that holds entries only the new pairs'
                // slots are written (old slots stay, empty ones are empty)
                const uint32_t c = c8[r];
                if (sl < c) continue;
                unsigned long long v = kEmpty;
                if (sl - c < placed) {
                    v = buf[st - W + sl - c];
                    ins += 1;
                    // nothing carried into r (the first pair placed there is the
                    // first homed there): its pairs are all homed at r, distance 0
                    if (st != (uint32_t)Te[r]) {
                        const uint32_t f = (uint32_t)(v >> 32);
                        const uint32_t dist = r - (uint32_t)(home_bucket(f, a.nb) - b0);
                        probe += dist;
                        if (dist >= a.cap_dist) push_candidate(a, f);
                    } else if (a.cap_dist == 0) {   // caps of 1..15: every insert is a candidate
                        push_candidate(a, (uint32_t)(v >> 32));
                    }
                } else if (!a.fresh) {
                    continue;
                }
                tab[r * kSlots + sl] = v;
                if (sl == c) cnt_out[r] = c + placed;
            }
        }
    }
    // statistics
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        ins += shfl_xor(ins, m);
        probe += shfl_xor(probe, m);
    }
    __syncthreads();
    if (lane == 0) {
        red[w] = ins;
        red[kLineWaves + w] = probe;
    }
    __syncthreads();
    if (tid < 2) {
        uint32_t v = 0;
        for (int i = 0; i < kLineWaves; ++i) v += red[tid * kLineWaves + i];
        if (v) atomicAdd(&a.counters[tid == 0 ? kCntInserted : kCntProbe], (unsigned long long)v);
    }
}

// ---------------------------------------------------------------- cap -----
// Walk the chain of feature f (home bucket to the first bucket holding an
// empty slot), four buckets per step. Counts f's valid entries with location
// <= thr; with kMark, replaces f's entries with location > thr by tombstones
// (feature kept, location invalid) instead.
template <bool kMark>
__device__ uint32_t chain_pass(unsigned long long* table, uint64_t nb, uint32_t f, uint32_t thr) {
    const int lane = lane_id();
    const int g = lane >> 4, gl = lane & 15;
    uint64_t b = home_bucket(f, nb);
    uint32_t total = 0;
    for (uint64_t walked = 0; walked <= nb; walked += 4) {
        uint64_t bi = b + (uint64_t)g;
        while (bi >= nb) bi -= nb;
        unsigned long long* p = &table[bi * kSlots + gl];
        uint64_t sl = *p;
        uint64_t emp = ballot(sl == kEmpty);
        int gend = 4;
#pragma unroll
        for (int x = 3; x >= 0; --x)
            if ((emp >> (16 * x)) & 0xFFFFull) gend = x;
        uint32_t loc = (uint32_t)sl;
        bool mine = g <= gend && (uint32_t)(sl >> 32) == f && live_entry(sl);
        if (kMark) {
            if (mine && loc > thr) *p = ((unsigned long long)f << 32) | kTombLoc;
        } else {
            total += popc64(ballot(mine && loc <= thr));
        }
        if (gend < 4) break;
        b += 4;
        while (b >= nb) b -= nb;
    }
    return total;
}

// Per-feature cap (Sec. 4.1): keep the `cap` smallest locations. Idempotent,
// so duplicate candidates or concurrent waves on one feature are harmless.
__device__ void finalize_feature(unsigned long long* table, uint64_t nb, uint32_t cap, uint32_t f) {
    uint32_t n = chain_pass<false>(table, nb, f, 0xFFFFFFFEu);
    if (n <= cap) return;
    uint32_t lo = 0, hi = 0xFFFFFFFEu;       // smallest thr with count(<= thr) >= cap
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (chain_pass<false>(table, nb, f, mid) >= cap) hi = mid; else lo = mid + 1;
    }
    chain_pass<true>(table, nb, f, lo);
}

__global__ __launch_bounds__(256) void k_cap_finalize(unsigned long long* table, uint64_t nb,
                                                      uint32_t cap, const uint32_t* cand,
                                                      uint64_t n_cand) {
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
    const uint64_t step = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t c = wave; c < n_cand; c += step) finalize_feature(table, nb, cap, cand[c]);
}

// Fallback when the candidate list overflowed: every entry stored at probe
// distance >= cap_dist triggers the finalisation of its feature.
__global__ __launch_bounds__(256) void k_cap_scan(unsigned long long* table, uint64_t nb,
                                                  uint32_t cap, uint32_t cap_dist) {
    const uint64_t n = nb * kSlots;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < n;
         i0 += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i = i0 + threadIdx.x;
        uint64_t sl = i < n ? (uint64_t)table[i] : kEmpty;
        bool hit = false;
        uint32_t f = (uint32_t)(sl >> 32);
        if (live_entry(sl)) {
            uint64_t hb = home_bucket(f, nb), bb = i / kSlots;
            uint64_t dist = bb >= hb ? bb - hb : bb + nb - hb;
            hit = dist >= cap_dist;
        }
        uint64_t m = ballot(hit);
        while (m) {   // the whole wave finalises each flagged feature in turn
            int src = __builtin_ctzll(m);
            m &= m - 1;
            uint32_t ff = shfl_idx(f, src);
            finalize_feature(table, nb, cap, ff);
        }
    }
}

// ------------------------------------------------------------- growth -----
// Re-insert every valid entry of the old table (tombstones are dropped).
__global__ __launch_bounds__(256) void k_rehash(const unsigned long long* old_table, uint64_t old_nb,
                                                unsigned long long* table, uint32_t* bcount,
                                                uint64_t nb, unsigned long long* counters) {
    const uint64_t n = old_nb * kSlots;
    uint32_t moved = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long e = old_table[i];
        if (!live_entry(e)) continue;
        const uint64_t d = insert_one(table, bcount, nb, home_bucket((uint32_t)(e >> 32), nb), e);
        if (d <= nb) moved += 1;
        else atomicAdd(&counters[kCntFull], 1ull);
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) moved += shfl_xor(moved, m);
    if (lane_id() == 0 && moved) atomicAdd(&counters[kCntMoved], (unsigned long long)moved);
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------- exports ----
__global__ __launch_bounds__(256) void k_dump(const unsigned long long* table, uint64_t nb,
                                              uint32_t lo, uint32_t hi, unsigned long long* out,
                                              uint64_t cap, unsigned long long* count) {
    const uint64_t n = nb * kSlots;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < n;
         i0 += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i = i0 + threadIdx.x;
        uint64_t e = i < n ? (uint64_t)table[i] : kEmpty;
        uint32_t f = (uint32_t)(e >> 32);
        bool keep = live_entry(e) && f >= lo && f <= hi;
        uint64_t m = ballot(keep);
        if (m == 0) continue;
        uint64_t base = 0;
        if (lane_id() == 0) base = atomicAdd(count, (unsigned long long)popc64(m));
        base = uniform64(((uint64_t)shfl_idx((uint32_t)(base >> 32), 0) << 32) |
                         shfl_idx((uint32_t)base, 0));
        uint64_t pos = base + rank_below(m);
        if (keep && pos < cap) out[pos] = e;
    }
}

// Census of the table: live entries, tombstones, and distinct features of the
// live entries. A live entry counts as its feature's first when no live entry
// of that feature lies before it on the feature's chain (buckets from the
// home bucket on, and the lower slots of its own bucket); chains are short
// (about one bucket) so the backwards walk is cheap.
__global__ __launch_bounds__(256) void k_census(const unsigned long long* table, uint64_t nb,
                                                unsigned long long* count) {
    const uint64_t n = nb * kSlots;
    uint32_t live = 0, tomb = 0, first = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = table[i];
        if (e == kEmpty) continue;
        if (!live_entry(e)) { tomb += 1; continue; }
        live += 1;
        const uint32_t f = (uint32_t)(e >> 32);
        const uint64_t bb = i / kSlots;
        uint64_t b = home_bucket(f, nb);
        bool seen = false;
        for (;; b = next_bucket(b, nb)) {
            const uint32_t end = b == bb ? (uint32_t)(i % kSlots) : (uint32_t)kSlots;
            for (uint32_t j = 0; j < end && !seen; ++j) {
                const uint64_t x = table[b * kSlots + j];
                seen = live_entry(x) && (uint32_t)(x >> 32) == f;
            }
            if (seen || b == bb) break;
        }
        first += seen ? 0u : 1u;
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        live += shfl_xor(live, m);
        tomb += shfl_xor(tomb, m);
        first += shfl_xor(first, m);
    }
    if (lane_id() == 0) {
        if (live) atomicAdd(&count[0], (unsigned long long)live);
        if (tomb) atomicAdd(&count[1], (unsigned long long)tomb);
        if (first) atomicAdd(&count[2], (unsigned long long)first);
    }
}

// Undo of a failed add: live entries of targets >= first_target become
// tombstones (their slots stay occupied, so every chain stays intact).
__global__ __launch_bounds__(256) void k_rollback(unsigned long long* table, uint64_t nb,
                                                  uint32_t first_target) {
    const uint64_t n = nb * kSlots;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = table[i];
        if (live_entry(e) && ((uint32_t)e >> kWindowBits) >= first_target)
            table[i] = (e & 0xFFFFFFFF00000000ull) | kTombLoc;
    }
}

inline unsigned grid_for(uint64_t items, unsigned per_block, unsigned max_blocks) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_sketch(const BuildArgs& a, bool pairs, hipStream_t st) {
    if (a.n_tiles == 0) return hipSuccess;
    unsigned grid = grid_for(a.n_tiles, 1, 16384);
    dim3 blk(kBuildThreads);
    if (a.S <= 64) {
        if (pairs) hipLaunchKernelGGL((k_sketch<1, true>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_sketch<1, false>), dim3(grid), blk, 0, st, a);
    } else if (a.S <= 128) {
        if (pairs) hipLaunchKernelGGL((k_sketch<2, true>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_sketch<2, false>), dim3(grid), blk, 0, st, a);
    } else {
        if (pairs) hipLaunchKernelGGL((k_sketch<4, true>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_sketch<4, false>), dim3(grid), blk, 0, st, a);
    }
    return hipGetLastError();
}

// Staging entries of the slice insert for 2^slice_shift buckets: the dynamic
// LDS left (at most 160 KiB a workgroup, less its static arrays) after 5 bytes
// a bucket; 0 if that is too few for the direct path's counters or a round.
uint32_t slice_buf_cap(uint32_t slice_shift) {
    static int max_lds = -1;
    if (max_lds < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 0;
        max_lds = v;
    }
    const int64_t avail = (int64_t)std::min(max_lds, 160 * 1024) - 1024 - ((int64_t)5 << slice_shift);
    if (avail <= 0) return 0;
    const uint32_t cap = (uint32_t)std::min<int64_t>(avail / 8, kLineCap) & ~7u;
    if ((uint64_t)cap * 8 < ((uint64_t)4 << slice_shift) || cap < 4 * kSlots) return 0;
    return cap;
}

bool slice_mode_fits(uint32_t slice_shift) {
    return slice_shift <= kMaxSliceShift && slice_buf_cap(slice_shift) != 0;
}

hipError_t launch_partition(const BuildArgs& a, uint64_t n_slots, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kMaxParts), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_slots == 0) return e;
    const uint64_t n_chunks = (a.n_tiles + a.chunk_tiles - 1) / a.chunk_tiles;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n_chunks, 1, 8192)), dim3(kScatThreads), 0, st,
                       a);
    e = hipGetLastError();
    if (e != hipSuccess || !a.slice_mode) return e;
    const uint64_t pairs_bound = n_slots;   // chunks: at most one partial per partition
    hipLaunchKernelGGL(k_hist2, dim3(grid_for(pairs_bound, kHistChunk, 4096) + a.n_parts),
                       dim3(kBuildThreads), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kBuildThreads), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter2, dim3(grid_for(pairs_bound, kScatChunk, 8192)),
                       dim3(kScatThreads), 0, st, a);
    return hipGetLastError();
}

namespace {
int resident_blocks(const void* kernel, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBuildThreads, lds) !=
            hipSuccess || cus * per_cu <= 0)
        return 2048;
    return cus * per_cu;
}
}  // namespace

hipError_t launch_insert(const BuildArgs& a, uint64_t max_items, hipStream_t st) {
    if (max_items == 0) return hipSuccess;
    static int resident = 0;   // workgroups of k_insert resident on the device at once
    if (resident == 0) resident = resident_blocks((const void*)k_insert, 0);
    if (!a.slice_mode) {
        uint64_t need = (max_items + kBuildThreads - 1) / kBuildThreads;
        unsigned grid = (unsigned)std::min<uint64_t>(need, (uint64_t)resident);
        hipLaunchKernelGGL(k_insert, dim3(grid), dim3(kBuildThreads), 0, st, a,
                           (const unsigned long long*)a.parted,
                           (const unsigned long long*)(a.part_start + a.n_parts));
        return hipGetLastError();
    }
    const uint32_t n_slices = a.n_parts << a.fine_bits;
    uint32_t buf_cap = slice_buf_cap(a.slice_shift), line_cap = kLineCap;
    if (buf_cap == 0) return hipErrorInvalidConfiguration;
    // forced (tests): a smaller staging buffer (more rounds a slice), or the
    // direct path for every slice
    if (a.stage_entries) {
        const uint64_t lo = std::max<uint64_t>(4 * kSlots, (uint64_t)1 << (a.slice_shift - 1));
        const uint64_t v = std::max<uint64_t>(lo, (uint64_t)a.stage_entries);
        buf_cap = (uint32_t)std::min<uint64_t>(buf_cap, (v + 7) & ~7ull);
    }
    if (a.force_direct) line_cap = 0;
    const size_t lds = (size_t)buf_cap * 8 + ((size_t)5 << a.slice_shift);
    hipLaunchKernelGGL(k_insert_slices, dim3(n_slices), dim3(kLineThreads), lds, st, a, buf_cap,
                       line_cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // deferred entries (count known on the device only): a small persistent grid
    hipLaunchKernelGGL(k_insert, dim3(std::min(resident, 1024)), dim3(kBuildThreads), 0, st, a,
                       (const unsigned long long*)a.parted,
                       (const unsigned long long*)(a.counters + kCntDefer));
    return hipGetLastError();
}

hipError_t launch_cap_finalize(unsigned long long* table, uint64_t nb, uint32_t cap,
                               const uint32_t* cand, uint64_t n_cand, hipStream_t st) {
    if (n_cand == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cap_finalize, dim3(grid_for(n_cand, 4, 8192)), dim3(256), 0, st, table,
                       nb, cap, cand, n_cand);
    return hipGetLastError();
}

hipError_t launch_cap_scan(unsigned long long* table, uint64_t nb, uint32_t cap,
                           uint32_t cap_dist, hipStream_t st) {
    hipLaunchKernelGGL(k_cap_scan, dim3(grid_for(nb * kSlots, 256, 8192)), dim3(256), 0, st,
                       table, nb, cap, cap_dist);
    return hipGetLastError();
}

hipError_t launch_rehash(const unsigned long long* old_table, uint64_t old_nb,
                         unsigned long long* table, uint32_t* bcount, uint64_t nb,
                         unsigned long long* counters, hipStream_t st) {
    if (old_nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rehash, dim3(grid_for(old_nb * kSlots, 256, 16384)), dim3(256), 0, st,
                       old_table, old_nb, table, bcount, nb, counters);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v,
                           hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_dump(const unsigned long long* table, uint64_t nb, uint32_t lo, uint32_t hi,
                       unsigned long long* out, uint64_t cap, unsigned long long* count,
                       hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dump, dim3(grid_for(nb * kSlots, 256, 16384)), dim3(256), 0, st, table,
                       nb, lo, hi, out, cap, count);
    return hipGetLastError();
}

hipError_t launch_census(const unsigned long long* table, uint64_t nb,
                         unsigned long long* count, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_census, dim3(grid_for(nb * kSlots, 256, 16384)), dim3(256), 0, st,
                       table, nb, count);
    return hipGetLastError();
}

hipError_t launch_rollback(unsigned long long* table, uint64_t nb, uint32_t first_target,
                           hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rollback, dim3(grid_for(nb * kSlots, 256, 16384)), dim3(256), 0, st,
                       table, nb, first_target);
    return hipGetLastError();
}

}  // namespace mc
