// Database build kernels (Sec. 4.1, Sec. 5.1-5.3): encode + canonical k-mers +
// h1 + bottom-s sketch per window + insertion into the bucketed multi-value
// table, the deterministic per-feature cap, table growth and test exports.
#include "mc_device.hpp"
#include "mc_internal.hpp"

namespace mc {

namespace {

constexpr int kWavesPerBuild = kBuildThreads / kWave;
constexpr int kWinPerWave = kTileWindows / kWavesPerBuild;     // 8
constexpr int kMaxSketch = 64;
// words of one tile: (kTileWindows-1) strides of at most 256 bases plus one
// window of at most 271 bases, 16 bases per word, plus alignment and one
// look-ahead word.
constexpr int kTileWordsMax = ((kTileWindows - 1) * 256 + 271 + 15) / 16 + 3;

struct BuildLds {
    Word words[kTileWordsMax];
    uint32_t feats[kWavesPerBuild][kWinPerWave * kMaxSketch];
    uint8_t wix[kWavesPerBuild][kWinPerWave * kMaxSketch];
};

// Insert the wave's pending (feature, location) items. Each 16-lane group
// owns one item at a time and reads its bucket as one 128-byte line; the
// group's first empty slot is claimed with a 64-bit compare-and-swap. A full
// bucket sends the item on to the next bucket, so every entry of a feature
// lies between its home bucket and the first bucket that still has an empty
// slot. Up to 8 items per group are in flight together.
__device__ void insert_items(const BuildArgs& a, const uint32_t* F, const uint8_t* WX,
                             uint32_t nf, uint32_t tid, uint32_t j0, uint64_t& ins,
                             uint64_t& probe, uint64_t& full) {
    constexpr int NB = 8;
    const int lane = lane_id();
    const int g = lane >> 4, gl = lane & 15;
    for (uint32_t base = 0; base < nf; base += 4 * NB) {
        uint64_t b[NB], ent[NB];
        uint32_t d[NB];
        bool pend[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            uint32_t i = base + (uint32_t)g + 4u * (uint32_t)q;
            pend[q] = i < nf;
            uint32_t f = pend[q] ? F[i] : 0u;
            uint32_t loc = (tid << kWindowBits) | (j0 + (pend[q] ? WX[i] : 0u));
            ent[q] = ((uint64_t)f << 32) | loc;
            b[q] = home_bucket(f, a.nb);
            d[q] = 0;
        }
        while (true) {
            bool any = false;
#pragma unroll
            for (int q = 0; q < NB; ++q) any |= pend[q];
            if (ballot(any) == 0) break;
            uint64_t sl[NB], old[NB];
            bool tried[NB];
            uint32_t gm[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                sl[q] = pend[q] ? (uint64_t)a.table[b[q] * kSlots + gl] : 0ull;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                uint64_t emp = ballot(pend[q] && sl[q] == kEmpty);
                gm[q] = (uint32_t)(emp >> (16 * g)) & 0xFFFFu;
                tried[q] = pend[q] && gm[q] != 0 && gl == __builtin_ctz(gm[q] | 0x10000u);
                old[q] = 0;
                if (tried[q])
                    old[q] = atomicCAS(&a.table[b[q] * kSlots + gl], (unsigned long long)kEmpty,
                                       (unsigned long long)ent[q]);
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                uint64_t wb = ballot(tried[q] && old[q] == kEmpty);
                bool won = ((wb >> (16 * g)) & 0xFFFFull) != 0;
                if (pend[q]) {
                    if (won) {
                        pend[q] = false;
                        if (gl == 0) {
                            ins += 1;
                            probe += d[q];
                            if (d[q] >= a.cap_dist) {
                                unsigned long long c = atomicAdd(&a.counters[kCntCand], 1ull);
                                if (c < a.cand_cap) a.cand[c] = (uint32_t)(ent[q] >> 32);
                            }
                        }
                    } else if (gm[q] == 0) {
                        b[q] = next_bucket(b[q], a.nb);
                        d[q] += 1;
                        if ((uint64_t)d[q] > a.nb) {
                            pend[q] = false;
                            if (gl == 0) full += 1;
                        }
                    }
                }
            }
        }
    }
}

template <int KPL, bool kInsert>
__global__ __launch_bounds__(kBuildThreads) void k_build(BuildArgs a) {
    __shared__ BuildLds L;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    uint64_t ins = 0, probe = 0, full = 0;
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
        uint32_t nf = 0;
        for (uint32_t wv = (uint32_t)wave; wv < nwin; wv += kWavesPerBuild) {
            const uint32_t j = j0 + wv;
            const uint64_t first = (uint64_t)j * a.S;
            const uint32_t nk = (uint32_t)min((uint64_t)a.S, n_starts - first);
            const uint32_t x0 = (uint32_t)(tstart + first - A0);
            uint32_t* sk = &L.feats[wave][nf];
            uint32_t n = sketch_window<KPL>(L.words, x0, nk, a.k, a.s, sk);
            wave_lds_sync();
            if (kInsert) {
                if ((uint32_t)lane < n) L.wix[wave][nf + lane] = (uint8_t)wv;
            } else {
                const uint64_t gw = td.win_base + j;
                if (lane == 0) a.out_counts[gw] = n;
                if ((uint32_t)lane < n) a.out_feats[gw * a.s + lane] = sk[lane];
            }
            nf += n;
        }
        if (kInsert) {
            wave_lds_sync();
            insert_items(a, L.feats[wave], L.wix[wave], nf, td.id, j0, ins, probe, full);
        }
    }
    if (kInsert) {
        // one atomic per wave for the counters
        uint32_t i32 = (uint32_t)ins, p32 = (uint32_t)probe, f32 = (uint32_t)full;
#pragma unroll
        for (int m = 1; m < kWave; m <<= 1) {
            i32 += shfl_xor(i32, m);
            p32 += shfl_xor(p32, m);
            f32 += shfl_xor(f32, m);
        }
        if (lane == 0) {
            if (i32) atomicAdd(&a.counters[kCntInserted], (unsigned long long)i32);
            if (p32) atomicAdd(&a.counters[kCntProbe], (unsigned long long)p32);
            if (f32) atomicAdd(&a.counters[kCntFull], (unsigned long long)f32);
        }
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
        bool mine = g <= gend && sl != kEmpty && (uint32_t)(sl >> 32) == f && loc != kBadLoc;
        if (kMark) {
            if (mine && loc > thr) *p = ((unsigned long long)f << 32) | kBadLoc;
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
        if (sl != kEmpty && (uint32_t)sl != kBadLoc) {
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
                                                unsigned long long* table, uint64_t nb,
                                                unsigned long long* counters) {
    const uint64_t n = old_nb * kSlots;
    uint32_t moved = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t e = old_table[i];
        if (e == kEmpty || (uint32_t)e == kBadLoc) continue;
        uint64_t b = home_bucket((uint32_t)(e >> 32), nb);
        bool done = false;
        for (uint64_t d = 0; d <= nb && !done; ++d) {
            for (int s = 0; s < kSlots && !done; ++s) {
                unsigned long long* p = &table[b * kSlots + s];
                if (*p == kEmpty && atomicCAS(p, (unsigned long long)kEmpty,
                                              (unsigned long long)e) == kEmpty)
                    done = true;
            }
            b = next_bucket(b, nb);
        }
        moved += done ? 1u : 0u;
        if (!done) atomicAdd(&counters[kCntFull], 1ull);
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
        bool keep = e != kEmpty && (uint32_t)e != kBadLoc && f >= lo && f <= hi;
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
        c += (e != kEmpty && (uint32_t)e != kBadLoc) ? 1u : 0u;
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

hipError_t launch_build(const BuildArgs& a, bool insert, hipStream_t st) {
    if (a.n_tiles == 0) return hipSuccess;
    unsigned grid = grid_for(a.n_tiles, 1, 16384);
    dim3 blk(kBuildThreads);
    if (a.S <= 64) {
        if (insert) hipLaunchKernelGGL((k_build<1, true>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_build<1, false>), dim3(grid), blk, 0, st, a);
    } else if (a.S <= 128) {
        if (insert) hipLaunchKernelGGL((k_build<2, true>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_build<2, false>), dim3(grid), blk, 0, st, a);
    } else {
        if (insert) hipLaunchKernelGGL((k_build<4, true>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_build<4, false>), dim3(grid), blk, 0, st, a);
    }
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
                         unsigned long long* table, uint64_t nb, unsigned long long* counters,
                         hipStream_t st) {
    if (old_nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rehash, dim3(grid_for(old_nb * kSlots, 256, 16384)), dim3(256), 0, st,
                       old_table, old_nb, table, nb, counters);
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
