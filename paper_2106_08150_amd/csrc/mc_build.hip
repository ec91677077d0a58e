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
constexpr uint32_t kMaxParts = 256;   // table partitions (8 bits)

struct SketchLds {
    Word words[kTileWordsMax];
    uint32_t scratch[kWavesPerBuild][kWave];
    uint32_t feats[kWavesPerBuild][kMaxSketch];
    uint32_t hist[kMaxParts];
};

// Bucket-range partition of a feature: the top bits of h2, so partition p
// holds the features whose home buckets form the p-th contiguous slice of the
// table (home = floor(h2 * nb / 2^64) is monotone in h2).
__device__ __forceinline__ uint32_t part_of(uint32_t f, uint32_t bits) {
    return bits ? (uint32_t)(h2(f) >> (64 - bits)) : 0u;
}

// Sketch every window of the call (B1-B4). One workgroup stages a tile of 32
// consecutive windows of one target as 2-bit words in LDS; each wave sketches
// every fourth window of the tile.
//   kPairs = false: out_counts[w] and out_feats[w*s ..] per window (export).
//   kPairs = true:  pairs[w*s + i] = feature << 32 | location for i < n and
//                   empty for n <= i < s, plus a histogram of the pairs' table
//                   partitions.
template <int KPL, bool kPairs>
__global__ __launch_bounds__(kBuildThreads) void k_sketch(BuildArgs a) {
    __shared__ SketchLds L;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t P = 1u << a.part_bits;
    if (kPairs) {
        for (uint32_t p = tid; p < P; p += kBuildThreads) L.hist[p] = 0;
    }
    for (uint64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        // target of this tile: last t with tile_first[t] <= tile
        uint32_t lo = 0, hi = a.n_targets;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (a.tile_first[mid] <= tile) lo = mid; else hi = mid;
        }
        const TargetDesc td = a.targets[lo];
        const uint32_t j0 = (uint32_t)(tile - a.tile_first[lo]) * kTileWindows;
        const uint32_t nwin = min((uint32_t)kTileWindows, td.nw - j0);
        const uintptr_t tstart = (uintptr_t)(a.text + td.off);
        const uintptr_t tend = tstart + td.len;
        const uintptr_t blo = tstart + (uint64_t)j0 * a.S;
        uintptr_t bhi = tstart + (uint64_t)(j0 + nwin - 1) * a.S + a.w;
        if (bhi > tend) bhi = tend;
        __syncthreads();
        stage_words(L.words, blo, bhi, tstart, tend, tid, kBuildThreads);
        __syncthreads();
        const uintptr_t A0 = blo & ~(uintptr_t)15;
        const uint64_t n_starts = td.len - a.k + 1;
        for (uint32_t wv = (uint32_t)wave; wv < nwin; wv += kWavesPerBuild) {
            const uint32_t j = j0 + wv;
            const uint64_t first = (uint64_t)j * a.S;
            const uint32_t nk = (uint32_t)min((uint64_t)a.S, n_starts - first);
            const uint32_t x0 = (uint32_t)(tstart + first - A0);
            uint32_t* sk = L.feats[wave];
            uint32_t n = sketch_window<KPL>(L.words, x0, nk, a.k, a.s, sk, L.scratch[wave]);
            wave_lds_sync();
            const uint64_t gw = td.win_base + j;
            if (kPairs) {
                if ((uint32_t)lane < a.s) {
                    uint64_t e = kEmpty;
                    if ((uint32_t)lane < n) {
                        uint32_t f = sk[lane];
                        e = ((uint64_t)f << 32) | ((td.id << kWindowBits) | j);
                        atomicAdd(&L.hist[part_of(f, a.part_bits)], 1u);
                    }
                    a.pairs[gw * a.s + lane] = e;
                }
            } else {
                if (lane == 0) a.out_counts[gw] = n;
                if ((uint32_t)lane < n) a.out_feats[gw * a.s + lane] = sk[lane];
            }
            wave_lds_sync();
        }
    }
    if (kPairs) {
        __syncthreads();
        for (uint32_t p = tid; p < P; p += kBuildThreads)
            if (L.hist[p]) atomicAdd(&a.hist[p], L.hist[p]);
    }
}

// Exclusive scan of the partition histogram (one workgroup, P <= 256):
// part_start[p] and the scatter cursors; part_start[P] = number of pairs.
__global__ __launch_bounds__(kMaxParts) void k_scan_parts(const uint32_t* hist, uint32_t P,
                                                          unsigned long long* part_start,
                                                          unsigned long long* cursor) {
    __shared__ unsigned long long wsum[kMaxParts / kWave];
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    unsigned long long v = t < P ? hist[t] : 0ull;
    unsigned long long x = v;      // inclusive wave scan
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t lo = shfl_idx((uint32_t)x, lane >= (uint32_t)d ? lane - d : lane);
        uint32_t hi = shfl_idx((uint32_t)(x >> 32), lane >= (uint32_t)d ? lane - d : lane);
        if (lane >= (uint32_t)d) x += ((unsigned long long)hi << 32) | lo;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    unsigned long long base = 0;
    for (uint32_t i = 0; i < w; ++i) base += wsum[i];
    unsigned long long excl = base + x - v;
    if (t < P) {
        part_start[t] = excl;
        cursor[t] = excl;
    }
    if (t == kMaxParts - 1) part_start[P] = base + x;
}

// Scatter the pairs into partition order (counting sort). A workgroup takes a
// chunk of 4096 slots, sorts its pairs by partition in LDS, reserves one run
// per partition with an atomic on that partition's cursor, and writes the
// runs out contiguously.
constexpr int kScatPer = 16;
constexpr int kScatChunk = kBuildThreads * kScatPer;

__global__ __launch_bounds__(kBuildThreads) void k_scatter(const unsigned long long* pairs,
                                                           uint64_t n_slots, uint32_t bits,
                                                           unsigned long long* cursor,
                                                           unsigned long long* out) {
    __shared__ unsigned long long buf[kScatChunk];
    __shared__ uint8_t bpart[kScatChunk];
    __shared__ uint32_t hist[kMaxParts], lstart[kMaxParts];
    __shared__ unsigned long long gbase[kMaxParts];
    __shared__ uint32_t wsum[kBuildThreads / kWave];
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t P = 1u << bits;
    for (uint64_t c0 = (uint64_t)blockIdx.x * kScatChunk; c0 < n_slots;
         c0 += (uint64_t)gridDim.x * kScatChunk) {
        hist[t] = 0;
        __syncthreads();
        unsigned long long e[kScatPer];
        uint32_t pos[kScatPer], pp[kScatPer];
#pragma unroll
        for (int j = 0; j < kScatPer; ++j) {
            uint64_t i = c0 + (uint64_t)j * kBuildThreads + t;
            e[j] = i < n_slots ? pairs[i] : kEmpty;
            pp[j] = 0;
            pos[j] = 0;
            if (e[j] != kEmpty) {
                pp[j] = part_of((uint32_t)(e[j] >> 32), bits);
                pos[j] = atomicAdd(&hist[pp[j]], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of hist (thread t owns partition t)
        uint32_t v = t < P ? hist[t] : 0u, x = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            uint32_t y = shfl_idx(x, lane >= (uint32_t)d ? lane - d : lane);
            if (lane >= (uint32_t)d) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        uint32_t base = 0;
        for (uint32_t i = 0; i < w; ++i) base += wsum[i];
        const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (t < P) {
            lstart[t] = base + x - v;
            gbase[t] = v ? atomicAdd(&cursor[t], (unsigned long long)v) : 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScatPer; ++j) {
            if (e[j] != kEmpty) {
                uint32_t d = lstart[pp[j]] + pos[j];
                buf[d] = e[j];
                bpart[d] = (uint8_t)pp[j];
            }
        }
        __syncthreads();
        for (uint32_t i = t; i < total; i += kBuildThreads) {
            uint32_t p = bpart[i];
            out[gbase[p] + (i - lstart[p])] = buf[i];
        }
        __syncthreads();
    }
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

// B5: insert the partition-ordered pairs, one entry per lane. A persistent
// grid of resident workgroups takes the entries in order (entry = thread slot
// + i * threads in the grid), so the threads in flight all work in one slice
// of the table: its counters stay in L2 and its lines in the Infinity Cache.
__global__ __launch_bounds__(kBuildThreads) void k_insert(BuildArgs a) {
    __shared__ uint32_t red[3][kWavesPerBuild];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t n = a.part_start[1u << a.part_bits];
    uint32_t ins = 0, probe = 0, full = 0;
    const uint64_t step = (uint64_t)gridDim.x * kBuildThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kBuildThreads + threadIdx.x; i < n; i += step) {
        const unsigned long long e = a.parted[i];
        const uint32_t f = (uint32_t)(e >> 32);
        const uint64_t d = insert_one(a.table, a.bcount, a.nb, home_bucket(f, a.nb), e);
        if (d > a.nb) {
            full += 1;
            continue;
        }
        ins += 1;
        probe += (uint32_t)d;
        if (d >= a.cap_dist) {
            unsigned long long c = atomicAdd(&a.counters[kCntCand], 1ull);
            if (c < a.cand_cap) a.cand[c] = f;
        }
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        ins += shfl_xor(ins, m);
        probe += shfl_xor(probe, m);
        full += shfl_xor(full, m);
    }
    if (lane == 0) {
        red[0][wave] = ins;
        red[1][wave] = probe;
        red[2][wave] = full;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t v = 0;
        for (int w = 0; w < kWavesPerBuild; ++w) v += red[threadIdx.x][w];
        const int idx[3] = {kCntInserted, kCntProbe, kCntFull};
        if (v) atomicAdd(&a.counters[idx[threadIdx.x]], (unsigned long long)v);
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

__global__ __launch_bounds__(256) void k_count_valid(const unsigned long long* table, uint64_t nb,
                                                     unsigned long long* count) {
    const uint64_t n = nb * kSlots;
    uint32_t c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t e = table[i];
        c += live_entry(e) ? 1u : 0u;
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) c += shfl_xor(c, m);
    if (lane_id() == 0 && c) atomicAdd(count, (unsigned long long)c);
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

hipError_t launch_partition(const BuildArgs& a, uint64_t n_slots, hipStream_t st) {
    const uint32_t P = 1u << a.part_bits;
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kMaxParts), 0, st, a.hist, P, a.part_start,
                       a.cursor);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_slots == 0) return e;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n_slots, kScatChunk, 8192)), dim3(kBuildThreads),
                       0, st, (const unsigned long long*)a.pairs, n_slots, a.part_bits, a.cursor,
                       a.parted);
    return hipGetLastError();
}

hipError_t launch_insert(const BuildArgs& a, uint64_t max_items, hipStream_t st) {
    if (max_items == 0) return hipSuccess;
    static int resident = 0;   // workgroups of k_insert resident on the device at once
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_insert, kBuildThreads, 0) !=
                hipSuccess || cus * per_cu <= 0)
            resident = 2048;
        else
            resident = cus * per_cu;
    }
    uint64_t need = (max_items + kBuildThreads - 1) / kBuildThreads;
    unsigned grid = (unsigned)std::min<uint64_t>(need, (uint64_t)resident);
    hipLaunchKernelGGL(k_insert, dim3(grid), dim3(kBuildThreads), 0, st, a);
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

hipError_t launch_count_valid(const unsigned long long* table, uint64_t nb,
                              unsigned long long* count, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_valid, dim3(grid_for(nb * kSlots, 256, 16384)), dim3(256), 0, st,
                       table, nb, count);
    return hipGetLastError();
}

}  // namespace mc
