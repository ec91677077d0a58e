// Classification kernels (Sec. 4.2, Sec. 5.2-5.6). One wave classifies one
// record: it sketches every window of both mates (same code as the build),
// gathers the location lists of all sketch elements into LDS, sorts them,
// counts equal locations (window count statistic), scores the best range of
// `sws` consecutive windows per target, keeps the top m targets and labels the
// record, by LCA when the top scores are close. Records whose list does not
// fit the fast path's LDS are queued for a second pass with a larger list.
#include <algorithm>
#include <cstddef>

#include "mc_device.hpp"
#include "mc_internal.hpp"

namespace mc {

namespace {

// Kernel arguments used once per record or on rare paths are read where they
// are used (a scalar load from the argument segment at an offset the compiler
// treats as unknown), so they do not occupy scalar registers across the record
// loop; the hot loop needs every scalar register it can get.
template <typename T>
__device__ __forceinline__ T arg_at_use(uint32_t off) {
    asm volatile("" : "+s"(off));
    const __attribute__((address_space(4))) char* base =
        (const __attribute__((address_space(4))) char*)__builtin_amdgcn_kernarg_segment_ptr();
    return *(const __attribute__((address_space(4))) T*)(base + off);
}
#define MC_COLD(field) arg_at_use<decltype(QueryArgs::field)>((uint32_t)offsetof(QueryArgs, field))

constexpr int kStageWords = 20;    // one window of at most 271 bases (19 words)
constexpr uint32_t kMaxFeat = 128; // sketch elements buffered before lookups

constexpr uint32_t kRing = kMaxFeat;   // lookup work items: at most one per feature
// Entries [kRing, kRing + kRingMirror) repeat entries [0, kRingMirror), so that
// the 32 items of a batch are read without wrapping (immediate LDS offsets).
constexpr uint32_t kRingMirror = 32;

// LDS of one wave. The sketch area serves a record's sketches and lookups, the
// rank area its run-length and scoring after the last lookup; they overlap.
template <uint32_t LCAP>
struct QueryLds {
    uint2 ring[kRing + kRingMirror];  // (feature, bucket) lookup work items
    uint32_t list[LCAP + kWave];      // one item batch may overshoot LCAP by < 64
    union {
        struct {
            Word stage[2 * kStageWords];
            uint32_t scratch[kWave];
            uint32_t feats[kMaxFeat];
        } sk;
        struct {
            uint16_t uidx[LCAP + 2];
            uint16_t score[LCAP];
        } rk;
    };
    uint32_t sel_t[kMaxTopM], sel_s[kMaxTopM], sel_b[kMaxTopM];   // top-m list
};

// Lanes below m (any m), computed in scalar registers.
__device__ __forceinline__ uint64_t lanes_below(uint32_t m) {
    return m >= 64u ? ~0ull : (1ull << m) - 1ull;
}

// s_waitcnt immediate for vmcnt(0) with the other counters left alone (gfx9
// encoding: vmcnt bits 3..0 and 15..14, expcnt 6..4, lgkmcnt 11..8).
constexpr int kWaitVmem0 = 0x0F70;

// Lanes 7, 15, ..., 63: the lanes holding the last slot of the bucket each
// 8-lane group reads.
constexpr uint64_t kLastSlots = 0x8080808080808080ull;

// Append the locations of features F[0..nf) to list (LDS). A work item is a
// (feature, bucket) pair; the wave takes up to 8 * NB items at a time, item
// 8q + g read by 8-lane group g as one 128-byte bucket line (16 bytes, two
// slots, a lane), so that NB lines per group are in flight. Slots of a bucket
// fill in order, so a bucket is full exactly when its last slot is occupied:
// a full bucket queues the feature's next bucket as a new item, and a
// feature's chain ends at its first bucket that is not full (inserts never
// pass such a bucket). Items wait in a ring in LDS, at most one per feature;
// every ring entry always holds some item of the launch (the ring is cleared
// to bucket 0 when a wave starts), so groups past a batch's last item may read
// any entry and their lines are simply ignored. Returns false once the list
// outgrew LCAP (locations past LCAP + 64 are then not stored: the record goes
// to the large-list pass). junk holds one word per lane that lanes without a
// hit store into.
template <uint32_t LCAP>
__device__ bool lookup(const QueryArgs& a, const uint32_t* F, uint32_t nf, uint2* ring,
                       uint32_t* list, uint32_t* junk, uint32_t& nlist, uint32_t& probes) {
    constexpr int NB = 4;
    constexpr uint32_t G = 8;            // groups of 8 lanes, one bucket line each
    const uint32_t lane = (uint32_t)lane_id();
    const uint32_t g = lane >> 3;
    for (uint32_t i = lane; i < nf; i += kWave) {
        const uint2 it = make_uint2(F[i], (uint32_t)home_bucket(F[i], a.nb));
        ring[i] = it;
        if (i < kRingMirror) ring[i + kRing] = it;
    }
    wave_lds_sync();
    // slots 2 (lane & 7) and 2 (lane & 7) + 1 of a bucket, as one 16-byte load
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2* slot2 = reinterpret_cast<const u64x2*>(a.table) + (lane & 7u);
    uint32_t head = 0, tail = nf;
    while (head < tail) {
        // every line issued so far has been used; saying so here lets this
        // batch's loads go out back to back (the compiler cannot tell which
        // of the previous batch's loads were issued)
        __builtin_amdgcn_s_waitcnt(kWaitVmem0);
        const uint32_t c = min(tail - head, G * NB);
        uint32_t f[NB], b[NB];
        u64x2 sl[NB];
        const uint2* batch = ring + ((head & (kRing - 1u)) + g);   // item 8q + g at batch[8q]
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const uint2 it = batch[G * q];
            f[q] = it.x;
            b[q] = it.y;
        }
        // groups past the batch's last item load nothing (their lines would
        // be fetched only to be ignored); the mask of the groups holding an
        // item keeps their unloaded values out of every result
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (G * q + g < c) sl[q] = slot2[(uint64_t)b[q] * (kSlots / 2)];
        head += c;
        probes += c;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (G * q >= c) break;
            const uint32_t nv = min(c - G * q, G);   // groups holding an item
            // lanes of the groups holding an item: one vector compare (scalar
            // issue, not vector issue, limits this kernel)
            const uint64_t held = ballot(g < nv);
            const unsigned long long s0 = sl[q].x, s1 = sl[q].y;
            // a slot is the item's if it holds the item's feature and a
            // stored location (not a tombstone); the last slot of a bucket is
            // occupied unless its location word is all ones (empty)
            const uint64_t hit0 = held & ballot((uint32_t)(s0 >> 32) == f[q]) &
                                  ballot((uint32_t)s0 < kTombLoc);
            const uint64_t hit1 = held & ballot((uint32_t)(s1 >> 32) == f[q]) &
                                  ballot((uint32_t)s1 < kTombLoc);
            if (hit0 | hit1) {
                // every lane stores both slots, those without a hit into a
                // word of their own (no branch around the stores); nlist <=
                // LCAP here, so hit0's entries stay below LCAP + 64
                const uint32_t n0 = popc64(hit0);
                const uint32_t i1 = rank_below(hit1, nlist + n0);
                uint32_t* const d0 = lane_in(hit0) ? list + rank_below(hit0, nlist) : junk + lane;
                uint32_t* const d1 = lane_in(hit1) && i1 < LCAP + kWave ? list + i1 : junk + lane;
                *d0 = (uint32_t)s0;
                *d1 = (uint32_t)s1;
                nlist += n0 + popc64(hit1);
                if (nlist > LCAP) return false;
            }
            const uint64_t full = held & kLastSlots & ballot((uint32_t)s1 != 0xFFFFFFFFu);
            if (full) {
                if (lane_in(full)) {
                    // the bucket count is read here, not held across the loop
                    const uint32_t nxt = b[q] + 1u == (uint32_t)MC_COLD(nb) ? 0u : b[q] + 1u;
                    const uint32_t pos = (tail + rank_below(full)) & (kRing - 1u);
                    ring[pos] = make_uint2(f[q], nxt);
                    if (pos < kRingMirror) ring[pos + kRing] = make_uint2(f[q], nxt);
                }
                tail += popc64(full);
            }
        }
        wave_lds_sync();
    }
    return true;
}

// Condensed layout: a work item is a (feature, index bucket) pair; 8-lane
// group g reads item 8q + g's index line, one 16-byte entry a lane. A feature
// has exactly one entry: found, its locations are appended (inline ones at
// once; a run is noted in `runs` and copied after the batch, all runs of the
// batch by the whole wave with one flat index, so that their loads are in
// flight together); not found in a full bucket, the feature's next bucket is
// queued. runs: 96 words of LDS owned by the wave. Returns false once the
// list outgrew LCAP.
template <uint32_t LCAP>
__device__ bool lookup_cond(const QueryArgs& a, const uint32_t* F, uint32_t nf, uint2* ring,
                            uint32_t* list, uint32_t* runs, uint32_t& nlist, uint32_t& probes) {
    constexpr int NB = 4;
    constexpr uint32_t G = 8;
    const uint32_t lane = (uint32_t)lane_id();
    const uint32_t g = lane >> 3;
    for (uint32_t i = lane; i < nf; i += kWave) {
        const uint2 it = make_uint2(F[i], (uint32_t)home_bucket(F[i], a.nb));
        ring[i] = it;
        if (i < kRingMirror) ring[i + kRing] = it;
    }
    wave_lds_sync();
    const uint4* ent = reinterpret_cast<const uint4*>(a.table) + (lane & 7u);
    uint32_t head = 0, tail = nf;
    while (head < tail) {
        __builtin_amdgcn_s_waitcnt(kWaitVmem0);
        const uint32_t c = min(tail - head, G * NB);
        uint32_t f[NB], b[NB];
        uint4 e[NB];
        const uint2* batch = ring + ((head & (kRing - 1u)) + g);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const uint2 it = batch[G * q];
            f[q] = it.x;
            b[q] = it.y;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)   // idle groups load nothing (see lookup)
            if (G * q + g < c) e[q] = ent[(uint64_t)b[q] * kCondEntries];
        head += c;
        uint32_t nrun = 0;   // runs of this batch (at most one a group and q: 32)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (G * q >= c) break;
            const uint32_t nv = min(c - G * q, G);
            probes += nv;
            const uint64_t used = ballot(g < nv) & ballot(e[q].y != 0u);   // occupied entries
            const uint64_t mine = used & ballot(e[q].x == f[q]);
            const uint64_t small = ballot(e[q].y <= kCondInline);
            const uint64_t hitA = mine & small, hitR = mine & ~small;
            const uint64_t hitB = hitA & ballot(e[q].y == 2u);
            if (hitA | hitR) {
                const uint32_t nA = popc64(hitA);
                if (nlist + nA + popc64(hitB) > LCAP) return false;
                if (lane_in(hitA)) list[rank_below(hitA, nlist)] = e[q].z;
                if (lane_in(hitB)) list[rank_below(hitB, nlist + nA)] = e[q].w;
                nlist += nA + popc64(hitB);
                if (lane_in(hitR)) {
                    const uint32_t r = nrun + rank_below(hitR);
                    runs[3 * r + 0] = e[q].y;
                    runs[3 * r + 1] = e[q].z;
                    runs[3 * r + 2] = e[q].w;
                }
                nrun += popc64(hitR);
            }
            // a group that did not find its feature in a full line goes on:
            // spread each group's found bits to its lowest lane, move that to
            // its last lane, and keep the full lines' last lanes without one
            uint64_t gf = mine;
            gf |= gf >> 1;
            gf |= gf >> 2;
            gf |= gf >> 4;
            const uint64_t full = used & kLastSlots & ~((gf & 0x0101010101010101ull) << 7);
            if (full) {
                if (lane_in(full)) {
                    // the bucket count is read here, not held across the loop
                    const uint32_t nxt = b[q] + 1u == (uint32_t)MC_COLD(nb) ? 0u : b[q] + 1u;
                    const uint32_t pos = (tail + rank_below(full)) & (kRing - 1u);
                    ring[pos] = make_uint2(f[q], nxt);
                    if (pos < kRingMirror) ring[pos + kRing] = make_uint2(f[q], nxt);
                }
                tail += popc64(full);
            }
        }
        if (nrun) {
            // lane r holds run r; an inclusive scan of the counts gives every
            // run's first list position
            wave_lds_sync();
            const uint32_t cnt = lane < nrun ? runs[3 * lane + 0] : 0u;
            uint32_t incl = cnt;
#pragma unroll
            for (int d = 1; d < 32; d <<= 1) {
                const uint32_t y = shfl_idx(incl, lane >= (uint32_t)d ? (int)lane - d : (int)lane);
                if (lane >= (uint32_t)d) incl += y;
            }
            const uint32_t total = uniform(shfl_idx(incl, (int)nrun - 1));
            if (nlist + total > LCAP) return false;
            wave_lds_sync();
            // runs[3r] = first position of run r (past the runs: above every
            // position), runs[3r + 1..2] = its offset in the value array
            if (lane < 32u) runs[3 * lane] = lane < nrun ? incl - cnt : 0xFFFFFFFFu;
            wave_lds_sync();
            for (uint32_t i = lane; i < total; i += kWave) {
                uint32_t r = 0;   // the last run whose first position is <= i
#pragma unroll
                for (uint32_t step = 16; step > 0; step >>= 1)
                    if (runs[3 * (r + step)] <= i) r += step;
                const uint64_t off = ((uint64_t)runs[3 * r + 2] << 32) | runs[3 * r + 1];
                list[nlist + i] = a.cval[off + (i - runs[3 * r])];
            }
            nlist += total;
        }
        wave_lds_sync();
    }
    return true;
}

template <int K>
__device__ __forceinline__ void sort_regs(uint32_t* list, uint32_t n) {
    const int lane = lane_id();
    uint32_t v[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        uint32_t e = (uint32_t)(r * kWave + lane);
        v[r] = e < n ? list[e] : 0xFFFFFFFFu;
    }
    wave_sort<K>(v);
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < K; ++r) {
        uint32_t e = (uint32_t)(r * kWave + lane);
        if (e < n) list[e] = v[r];
    }
    wave_lds_sync();
}

// Bitonic sort of list[0..P) in LDS by one wave (P a power of two, entries
// n..P-1 padded with the largest key).
__device__ void sort_lds(uint32_t* list, uint32_t n, uint32_t P) {
    const uint32_t lane = (uint32_t)lane_id();
    for (uint32_t e = n + lane; e < P; e += kWave) list[e] = 0xFFFFFFFFu;
    wave_lds_sync();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t idx = lane; idx < P / 2; idx += kWave) {
                uint32_t i = (idx / stride) * 2 * stride + (idx % stride);
                uint32_t j = i + stride;
                bool asc = (i & size) == 0;
                uint32_t x = list[i], y = list[j];
                if ((x > y) == asc) {
                    list[i] = y;
                    list[j] = x;
                }
            }
            wave_lds_sync();
        }
    }
}

// Lists of more than 128 locations.
template <uint32_t LCAP>
__device__ __forceinline__ void sort_list_long_body(uint32_t* list, uint32_t n) {
    uint32_t P = 256;
    while (P < n) P <<= 1;
    switch (P) {
        case 256: sort_regs<4>(list, n); break;
        case 512: sort_regs<8>(list, n); break;
        case 1024: if (LCAP >= 1024) sort_regs<16>(list, n); break;
        default: sort_lds(list, n, P); break;
    }
}

// The fast paths' copy is out of line (the hot loop stays small in the
// instruction cache), with an LDS pointer so that the out-of-line code keeps
// LDS instructions. The large-list pass, which every classification launches,
// inlines it: there the out-of-line call needed a stack frame in scratch
// memory.
template <uint32_t LCAP>
__device__ __attribute__((noinline)) void sort_list_long(MC_LDS uint32_t* lds_list, uint32_t n) {
    sort_list_long_body<LCAP>((uint32_t*)lds_list, n);
}

// Ascending sort of list[0..n) in LDS.
template <uint32_t LCAP>
__device__ __forceinline__ void sort_list(uint32_t* list, uint32_t n) {
    if (n <= 64) sort_regs<1>(list, n);
    else if (n <= 128) sort_regs<2>(list, n);
    else if constexpr (LCAP <= 1024) sort_list_long<LCAP>((MC_LDS uint32_t*)list, n);
    else sort_list_long_body<LCAP>(list, n);
}

// Label and top-m list of a record (lane x writes the x-th top hit).
template <typename Lds>
__device__ __forceinline__ void write_result(const QueryArgs& a, uint32_t rec, uint32_t label,
                                             const Lds& L, uint32_t nsel) {
    const uint32_t lane = (uint32_t)lane_id();
    if (lane == 0) a.out_labels[rec] = label;
    uint32_t* const out_top = MC_COLD(out_top);
    const uint32_t top_m = MC_COLD(top_m);
    if (out_top && lane < top_m) {
        const bool h = lane < nsel;
        uint32_t* o = out_top + ((uint64_t)rec * top_m + lane) * 3;
        o[0] = h ? L.sel_t[lane] : kNone;
        o[1] = h ? L.sel_s[lane] : 0u;
        o[2] = h ? L.sel_b[lane] : 0u;
    }
}

// floor(n / S): a multiply-high for the counts of any real record, a 64-bit
// division only past 2^32.
__device__ __forceinline__ uint64_t div_by_S(const QueryArgs& a, uint64_t n) {
    if ((n >> 32) == 0) {
        const uint32_t x = (uint32_t)n, t = __umulhi(a.divS.m, x);
        return (t + ((x - t) >> a.divS.sh1)) >> a.divS.sh2;
    }
    return n / a.S;
}

// Windows of a mate of len bases, and the windows of reference a fragment of
// F bases can touch (sws).
__device__ __forceinline__ uint64_t mate_windows(const QueryArgs& a, uint64_t len) {
    return len < a.k ? 0 : div_by_S(a, len - a.k + a.S);
}
// The same for a mate of a record shorter than 2^31 bytes: len - k + S then
// fits 32 bits, so the division needs no 64-bit fallback.
__device__ __forceinline__ uint32_t mate_windows32(const QueryArgs& a, uint32_t len) {
    if (len < a.k) return 0u;
    const uint32_t x = len - a.k + a.S, t = __umulhi(a.divS.m, x);
    return (t + ((x - t) >> a.divS.sh1)) >> a.divS.sh2;
}
__device__ __forceinline__ uint32_t fragment_sws(const QueryArgs& a, uint64_t F) {
    return F < a.k ? 1u : (uint32_t)(div_by_S(a, F - a.k + a.S - 1) + 1);
}
// The same for a fragment below 2^32 bases: F - k + S - 1 fits 32 bits unless
// F lies within 512 of 2^32 (S is at most 256).
__device__ __forceinline__ uint32_t fragment_sws32(const QueryArgs& a, uint32_t F) {
    if (F < a.k) return 1u;
    if (F > 0xFFFFFE00u) return fragment_sws(a, F);
    const uint32_t x = F - a.k + a.S - 1u, t = __umulhi(a.divS.m, x);
    return ((t + ((x - t) >> a.divS.sh1)) >> a.divS.sh2) + 1u;
}

// One window of a record: its bytes [lo, hi) inside the mate [vlo, vhi), as
// 32-bit offsets from the record's first byte rounded down to 16 bytes (the
// staging base; records are shorter than 2^31 bytes), its number of k-mer
// starts and the offset of its first base in the staged words.
struct WinRef {
    uint32_t lo, hi, vlo, vhi, nk, x0;
};

// Window i of the record (mate 1's windows first; mate 2 follows mate 1);
// i >= nwt gives an empty one. r0: the record's first byte from the base.
__device__ __forceinline__ WinRef window_ref(const QueryArgs& a, uint32_t i, uint32_t nwt,
                                             uint32_t nw0, uint32_t r0, const uint32_t (&len)[2]) {
    WinRef r{0u, 0u, 0u, 0u, 0u, 0u};
    if (i >= nwt) return r;
    const int sg = i < nw0 ? 0 : 1;
    const uint32_t j = sg ? i - nw0 : i;
    r.vlo = r0 + (sg ? len[0] : 0u);
    r.vhi = r.vlo + len[sg];
    r.lo = r.vlo + j * a.S;
    r.hi = min(r.lo + a.w, r.vhi);
    r.nk = min(a.S, len[sg] - a.k + 1u - j * a.S);
    r.x0 = r.lo & 15u;
    return r;
}

// Words staged for a window: its bytes from the 16-byte boundary below it, plus
// one look-ahead word.
__device__ __forceinline__ uint32_t staged_words(const WinRef& r) {
    return r.nk ? (r.hi - (r.lo & ~15u) + 15u) / 16u + 1u : 0u;
}

// Stage two windows at once, A's words into W[0..) and B's into
// W[kStageWords..), one dword (4 bases) per lane: a 150-base read's two
// windows take a single pass of the wave. dirtyA / dirtyB (wave-uniform): a
// staged byte of that window's mate is not a base.
__device__ __forceinline__ void stage_pair(Word* W, uintptr_t base, const WinRef& A,
                                           const WinRef& B, int lane, bool& dirtyA,
                                           bool& dirtyB) {
    const uint32_t ndA = 4u * staged_words(A), nd = ndA + 4u * staged_words(B);
    // the flags are vector words, not lane masks: merging lane masks across
    // the loop took scalar instructions (scalar issue limits this kernel)
    uint32_t badA = 0u, badB = 0u;
    for (uint32_t q = (uint32_t)lane; q < nd; q += kWave) {
        const bool second = q >= ndA;
        const uint32_t bad = stage_dword(W + (second ? kStageWords : 0), base,
                                         (second ? B.lo : A.lo) & ~15u, second ? q - ndA : q,
                                         second ? B.vlo : A.vlo, second ? B.vhi : A.vhi);
        badA |= second ? 0u : bad;
        badB |= second ? bad : 0u;
    }
    dirtyA = ballot(badA != 0u) != 0;
    dirtyB = ballot(badB != 0u) != 0;
}

// A record's staging base and lengths, or false for a record of 2^31 bytes or
// more (beyond every pass: left unclassified and counted as too long).
struct RecordSpan {
    uintptr_t base;
    uint32_t r0;
    uint32_t len[2];
};
__device__ __forceinline__ bool record_span(const QueryArgs& a, uint64_t o0, uint64_t o1,
                                            uint64_t o2, RecordSpan& rs) {
    if (o2 - o0 >= (1ull << 31)) return false;
    const uintptr_t first = (uintptr_t)(a.reads + o0);
    rs.base = first & ~(uintptr_t)15;
    rs.r0 = (uint32_t)(first - rs.base);
    rs.len[0] = (uint32_t)(o1 - o0);
    rs.len[1] = (uint32_t)(o2 - o1);
    return true;
}

struct WaveStats {
    uint32_t features = 0, locations = 0, probes = 0, passed_on = 0;
};

// Label of a record from its top-m list (sel_* in LDS, nsel entries): the
// best target's taxon on a clear lead, else the LCA of the taxa of the listed
// targets within hit_diff of the best score.
// The taxonomy arrays are read by scalar loads (every index is wave-uniform;
// the arrays are small and do not change during a launch).
typedef const __attribute__((address_space(4))) uint32_t ConstU32;
__device__ __forceinline__ ConstU32* scalar_ptr(const uint32_t* p) {
    return (ConstU32*)(uintptr_t)p;
}

__device__ __forceinline__ uint32_t lca_uniform(uint32_t a, uint32_t b, ConstU32* parent,
                                                ConstU32* depth) {
    uint32_t da = depth[a], db = depth[b];
    while (da > db) { a = parent[a]; --da; }
    while (db > da) { b = parent[b]; --db; }
    while (a != b) { a = parent[a]; b = parent[b]; }
    return a;
}

template <typename Lds>
__device__ __forceinline__ uint32_t label_of(const QueryArgs& a, const Lds& L, uint32_t nsel) {
    const uint32_t min_hits = MC_COLD(min_hits), hit_diff = MC_COLD(hit_diff);
    uint32_t label = kNone;
    const uint32_t c1 = uniform(L.sel_s[0]);
    if (nsel > 0 && c1 >= min_hits) {
        const uint32_t c2 = nsel > 1 ? uniform(L.sel_s[1]) : 0u;
        ConstU32* const taxon = scalar_ptr(MC_COLD(target_taxon));
        label = taxon[uniform(L.sel_t[0])];
        if (c1 - c2 <= hit_diff) {
            ConstU32* const parents = scalar_ptr(MC_COLD(parents));
            ConstU32* const depth = scalar_ptr(MC_COLD(depth));
            for (uint32_t x = 1; x < nsel; ++x)
                if ((uint64_t)uniform(L.sel_s[x]) + hit_diff >= c1)
                    label = lca_uniform(label, taxon[uniform(L.sel_t[x])], parents, depth);
        }
    }
    return label;
}

// Whether the top-m rounds can stop after round m (score: its score): only
// when no top-hit list is written; then after the first round if the best
// score is below min_hits (unclassified), else at the first score more than
// hit_diff below the best (later, lower entries take no part in the label).
struct TopStop {
    bool whole_list;
    uint32_t min_hits, hit_diff, c_best = 0;
    __device__ __forceinline__ bool operator()(uint32_t m, uint32_t score) {
        if (whole_list) return false;
        if (m == 0) {
            c_best = score;
            return score < min_hits;
        }
        return (uint64_t)score + hit_diff < c_best;
    }
};

// Steps Q5-Q8 for a list of at most 64 locations (most records), held one a
// lane: sorted in registers; the runs of equal locations (window counts) are
// found with one ballot; distinct location u moves to lane u with its first
// list index P(u) (the number of smaller locations), so that a range's score
// is P(end) - P(u), end being the first distinct location past the range
// (at most sws windows of one target); top-m by wave maxima as below.
template <typename Lds>
__device__ __forceinline__ void label_short_list(const QueryArgs& a, uint32_t rec, Lds& L,
                                                 uint32_t n, uint32_t sws) {
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t v[1] = {lane < n ? L.list[lane] : 0xFFFFFFFFu};
    wave_sort<1>(v);
    const uint32_t prev = (uint32_t)__builtin_amdgcn_mov_dpp((int)v[0], 0x138, 0xF, 0xF, false);
    const uint64_t firsts = lanes_below(n) & (ballot(v[0] != prev) | 1ull);
    const uint32_t U = popc64(firsts);
    uint32_t* const first_of = L.sk.scratch;          // lane of distinct location u
    if (lane_in(firsts)) first_of[rank_below(firsts)] = lane;
    wave_lds_sync();
    const uint32_t P = lane < U ? first_of[lane] : n;    // P(U) = n
    const uint32_t loc = shfl_idx(v[0], (int)(P & 63u));
    wave_lds_sync();
    // end of the range of sws windows starting at loc (not past its target)
    const uint32_t w = loc & kWindowMask, base = loc - w;
    const uint32_t lim = base + min(w + sws, 1u << kWindowBits);
    uint32_t end = lane + 1u;
    const uint32_t steps = min(sws, U);
    for (uint32_t j = 1; j < steps; ++j) {
        const uint32_t l2 = shfl_idx(loc, (int)min(lane + j, 63u));
        end += (lane + j < U && l2 < lim) ? 1u : 0u;
    }
    const uint32_t Pend = shfl_idx(P, (int)min(end, 63u));
    const uint32_t score = (end >= U ? n : Pend) - P;
    uint32_t key = lane < U ? (score << 16) | (0xFFFFu - lane) : 0u;
    const uint32_t t = loc >> kWindowBits;
    TopStop stop{MC_COLD(out_top) != nullptr, MC_COLD(min_hits), MC_COLD(hit_diff)};
    const uint32_t top_m = MC_COLD(top_m);
    uint32_t nsel = 0;
    for (uint32_t m = 0; m < top_m; ++m) {
        const uint32_t k = wave_max_u32(key);
        if (k == 0) break;
        const uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)loc, (int)(0xFFFFu - (k & 0xFFFFu)));
        if (lane == 0) {
            L.sel_t[m] = sl >> kWindowBits;
            L.sel_s[m] = k >> 16;
            L.sel_b[m] = sl & kWindowMask;
        }
        nsel = m + 1;
        if (stop(m, k >> 16)) break;
        if (t == sl >> kWindowBits) key = 0;
    }
    wave_lds_sync();
    write_result(a, rec, label_of(a, L, nsel), L, nsel);
}

template <uint32_t LCAP, int KPL, bool C>
__device__ void classify_record(const QueryArgs& a, uint32_t rec, QueryLds<LCAP>& L, bool big,
                                const Threshold& th, WaveStats& ws) {
    const int lane = lane_id();
    // the record's offsets by scalar loads (rec is wave-uniform; the array
    // does not change during the launch)
    typedef const __attribute__((address_space(4))) uint64_t ConstU64;
    ConstU64* const off = (ConstU64*)(uintptr_t)a.offsets;
    uint64_t o0, o1, o2;
    if (a.paired) {
        o0 = off[2ull * rec]; o1 = off[2ull * rec + 1]; o2 = off[2ull * rec + 2];
    } else {
        o0 = off[rec]; o1 = off[rec + 1ull]; o2 = o1;
    }
    if (o1 < o0 || o2 < o1) {           // malformed record: nothing to classify
        write_result(a, rec, kNone, L, 0);
        return;
    }
    RecordSpan rs;
    if (!record_span(a, o0, o1, o2, rs)) {
        if (lane == 0) atomicAdd(&MC_COLD(counters)[kQTooLong], 1u);
        write_result(a, rec, kNone, L, 0);
        return;
    }
    // the fragment: the record's length (below 2^31), or the insert size
    // when that is longer and both mates are present
    const uint32_t len = rs.len[0] + rs.len[1];
    const uint32_t F = rs.len[0] > 0 && rs.len[1] > 0 && a.insert_size > len ? a.insert_size : len;
    const uint32_t sws = fragment_sws32(a, F);

    // windows of the record, mate 1's then mate 2's, sketched two at a time
    uint32_t nws[2];
    for (int sg = 0; sg < 2; ++sg)
        nws[sg] = mate_windows32(a, rs.len[sg]);
    const uint32_t nwt = nws[0] + nws[1];
    uint32_t nlist = 0, nf = 0;
    bool fits = true;
    for (uint32_t p = 0; p < nwt && fits; p += 2) {
        WinRef wr[2];
        for (int h = 0; h < 2; ++h) wr[h] = window_ref(a, p + h, nwt, nws[0], rs.r0, rs.len);
        wave_lds_sync();
        bool dirtyA, dirtyB;
        stage_pair(L.sk.stage, rs.base, wr[0], wr[1], lane, dirtyA, dirtyB);
        wave_lds_sync();
        uint32_t nA, nB;
        sketch_pair<KPL>(L.sk.stage, wr[0].x0, wr[0].nk, L.sk.stage + kStageWords, wr[1].x0, wr[1].nk,
                         a.k, a.s, th, L.sk.feats + nf, L.sk.feats + nf + a.s, L.sk.scratch, nA,
                         nB, dirtyA, dirtyB);
        wave_lds_sync();
        if (nA < a.s && nB) {      // close the gap after A's features
            const uint32_t f = (uint32_t)lane < nB ? L.sk.feats[nf + a.s + lane] : 0u;
            wave_lds_sync();
            if ((uint32_t)lane < nB) L.sk.feats[nf + nA + lane] = f;
            wave_lds_sync();
        }
        nf += nA + nB;
        // look up the buffered features after the last pair or before the
        // buffer could overflow (one call site keeps the loop compact)
        if (nf && (p + 2 >= nwt || nf + 2 * a.s > kMaxFeat)) {
            ws.features += nf;
            if constexpr (C)   // the stage and scratch areas hold the runs meanwhile
                fits = lookup_cond<LCAP>(a, L.sk.feats, nf, L.ring, L.list,
                                         reinterpret_cast<uint32_t*>(L.sk.stage), nlist,
                                         ws.probes);
            else
                fits = lookup<LCAP>(a, L.sk.feats, nf, L.ring, L.list, L.sk.scratch, nlist,
                                    ws.probes);
            nf = 0;
        }
    }
    if (!fits) {
        // the fast path queues the record for the large-list pass, that pass
        // for the HBM-list pass (ids from n_records on)
        if (lane == 0) {
            uint32_t* const counters = MC_COLD(counters);
            const uint32_t qi = atomicAdd(&counters[big ? kQHuge : kQOverflow], 1u);
            MC_COLD(queue)[(big ? MC_COLD(n_records) : 0u) + qi] = rec;
        }
        ws.passed_on += 1;
        return;
    }
    wave_lds_sync();
    const uint32_t n = nlist;
    ws.locations += n;
    if (n <= (uint32_t)kWave) {
        label_short_list(a, rec, L, n, sws);
        return;
    }
    sort_list<LCAP>(L.list, n);

    // run-length encoding: uidx[u] = first index of the u-th distinct location
    uint32_t U = 0;
    for (uint32_t c = 0; c < n; c += kWave) {
        // i < n + 63 < LCAP + 64: every lane reads inside the list
        const uint32_t i = c + (uint32_t)lane;
        const uint32_t cur = L.list[i], prev = L.list[i ? i - 1u : 0u];
        const uint64_t mb = lanes_below(n - c) & (ballot(cur != prev) | (c == 0 ? 1ull : 0ull));
        if (lane_in(mb)) L.rk.uidx[U + rank_below(mb)] = (uint16_t)i;
        U += popc64(mb);
    }
    if (lane == 0) L.rk.uidx[U] = (uint16_t)n;
    wave_lds_sync();

    // score of the range of sws windows starting at each distinct location
    for (uint32_t u = (uint32_t)lane; u < U; u += kWave) {
        const uint32_t loc = L.list[L.rk.uidx[u]];
        const uint32_t t = loc >> kWindowBits, w_end = (loc & kWindowMask) + sws;
        uint32_t score = 0;
        for (uint32_t v = u; v < U; ++v) {
            const uint32_t l2 = L.list[L.rk.uidx[v]];
            if ((l2 >> kWindowBits) != t || (l2 & kWindowMask) >= w_end) break;
            score += (uint32_t)L.rk.uidx[v + 1] - (uint32_t)L.rk.uidx[v];
        }
        L.rk.score[u] = (uint16_t)score;
    }
    wave_lds_sync();

    // top-m targets by (score desc, target asc); per target the range with the
    // highest score, ties to the smallest start window. The key of distinct
    // location u is score << 16 | (0xFFFF - u): distinct locations ascend with
    // u, so the wave maximum of the keys is the highest score and, among equal
    // scores, the smallest location (smallest target, then window). Each of
    // the m rounds takes one wave maximum and then drops the chosen target.
    //
    // Without a top-hit output only the label needs the list, and the rounds
    // stop once it is decided: after the first round if its score is below
    // min_hits (unclassified), else at the first score more than hit_diff
    // below the best (a clear lead after the second round; later entries
    // with lower scores take no part in the LCA).
    uint32_t nsel = 0;
    const uint32_t top_m = MC_COLD(top_m);
    TopStop decided{MC_COLD(out_top) != nullptr, MC_COLD(min_hits), MC_COLD(hit_diff)};
    if (U <= (uint32_t)kWave) {          // one distinct location per lane
        uint32_t key = 0, t = kNone;
        if ((uint32_t)lane < U) {
            t = L.list[L.rk.uidx[lane]] >> kWindowBits;
            key = ((uint32_t)L.rk.score[lane] << 16) | (0xFFFFu - (uint32_t)lane);
        }
        for (uint32_t m = 0; m < top_m; ++m) {
            const uint32_t k = wave_max_u32(key);
            if (k == 0) break;
            const uint32_t loc = L.list[L.rk.uidx[0xFFFFu - (k & 0xFFFFu)]];
            if (lane == 0) {
                L.sel_t[m] = loc >> kWindowBits;
                L.sel_s[m] = k >> 16;
                L.sel_b[m] = loc & kWindowMask;
            }
            nsel = m + 1;
            if (decided(m, k >> 16)) break;
            if (t == loc >> kWindowBits) key = 0;
        }
        wave_lds_sync();
    } else {
        for (uint32_t m = 0; m < top_m; ++m) {
            uint32_t key = 0;
            for (uint32_t u = (uint32_t)lane; u < U; u += kWave) {
                const uint32_t t = L.list[L.rk.uidx[u]] >> kWindowBits;
                bool excluded = false;
                for (uint32_t x = 0; x < m; ++x) excluded |= (L.sel_t[x] == t);
                const uint32_t ku = ((uint32_t)L.rk.score[u] << 16) | (0xFFFFu - u);
                if (!excluded && ku > key) key = ku;
            }
            const uint32_t k = wave_max_u32(key);
            if (k == 0) break;
            const uint32_t loc = L.list[L.rk.uidx[0xFFFFu - (k & 0xFFFFu)]];
            if (lane == 0) {
                L.sel_t[m] = loc >> kWindowBits;
                L.sel_s[m] = k >> 16;
                L.sel_b[m] = loc & kWindowMask;
            }
            wave_lds_sync();
            nsel = m + 1;
            if (decided(m, k >> 16)) break;
        }
    }

    write_result(a, rec, label_of(a, L, nsel), L, nsel);
}

// Occupancy: the lookups' memory latency is hidden by other waves' work, so
// occupancy pays for a few spilled scalar registers. A 512-entry list takes
// about 5.7 KB of LDS a wave, which holds a CU to 28 waves: seven a SIMD (at
// most 72 VGPRs). A 256-entry list takes about 3.7 KB, so eight waves a SIMD
// fit (64 VGPRs). A 1,024-entry list (9.7 KB) allows four waves a SIMD and
// the large-list pass (about 130 KB) one workgroup a CU: their register
// budgets follow, so that no variant spills vector registers to scratch
// memory (a kernel with scratch makes the runtime set up scratch for the
// hardware queue it runs on, milliseconds on a queue's first such launch).
// The condensed layout's lookups also fit eight waves at a 256-entry list
// (63 VGPRs, more scalar spills than at seven, and 4% faster).
template <uint32_t LCAP, bool C>
constexpr int classify_waves_per_simd() {
    return LCAP <= 256 ? 8 : LCAP <= 512 ? 7 : LCAP <= 1024 ? 4 : 1;
}

template <uint32_t LCAP, int WPB, int KPL, bool C>
__global__ __launch_bounds__(WPB * 64)
__attribute__((amdgpu_waves_per_eu(classify_waves_per_simd<LCAP, C>())))
void k_classify(QueryArgs a, int big, int cls) {
    __shared__ QueryLds<LCAP> L[WPB];
    const int wave = (int)uniform(threadIdx.x >> 6);
    for (uint32_t i = (uint32_t)lane_id(); i < kRing + kRingMirror; i += kWave)
        L[wave].ring[i] = make_uint2(0u, 0u);   // any item must name a bucket of the table
    wave_lds_sync();
    // the records of this launch: all of them, those queued for the large-list
    // pass (big), or those of size class cls >= 0 (routed); the id arrays are
    // read where they are used (no registers held across the record loop)
    const uint32_t n_iter = big ? uniform(a.counters[kQOverflow])
                                : cls >= 0 ? uniform(a.route_meta[cls]) : a.n_records;
    WaveStats ws;
    const Threshold th(a.S, a.s);
    for (uint32_t it = blockIdx.x * WPB + wave; it < n_iter; it += gridDim.x * WPB) {
        uint32_t rec = it;
        if (big) {
            rec = uniform(MC_COLD(queue)[it]);
        } else if (cls >= 0) {
            const uint32_t* const meta = MC_COLD(route_meta);
            rec = uniform(MC_COLD(route_queue)[meta[kMaxRoutes + cls] + it]);
        }
        classify_record<LCAP, KPL, C>(a, rec, L[wave], big != 0, th, ws);
    }
    // work of records that go on to the large-list pass counts in both passes
    if (lane_id() == 0 && a.qstats) {
        unsigned long long* q = a.qstats + ((blockIdx.x * WPB + wave) % kQsCopies) * kQsStride;
        if (ws.features) atomicAdd(&q[kQsFeatures], (unsigned long long)ws.features);
        if (ws.locations) atomicAdd(&q[kQsLocations], (unsigned long long)ws.locations);
        if (ws.probes) atomicAdd(&q[kQsProbes], (unsigned long long)ws.probes);
        if (ws.passed_on)
            atomicAdd(&q[big ? kQsHuge : kQsLarge], (unsigned long long)ws.passed_on);
    }
}

// ------------------------------------------------------ HBM-list pass -----
// Records whose candidate list outgrew the large-list pass: one workgroup a
// record, the lists in its region of the workspace's huge scratch. The steps
// are those of the other passes (Sec. 4.2, Sec. 5.3-5.6) without a sort: the
// window count of each distinct location is accumulated in a hash table in
// HBM (Q4-Q6), the score of the range of `sws` windows starting at each
// distinct location sums the counts of its windows looked up in that table,
// and each target keeps its best range with a 64-bit atomic maximum of
// score << 32 | ~location (highest score, then smallest start window, as the
// sorted passes' keys). Top-m and the label follow as in the other passes.
struct HugeRegion {
    uint32_t* feats;                 // kHugeFeats
    uint32_t* locs;                  // kHugeLocs
    uint32_t* keys;                  // kHugeSlots, kNone = empty
    uint32_t* cnt;                   // kHugeSlots
    unsigned long long* best;        // kHugeTargets, zero between records
    uint32_t* tlist;                 // kHugeTargets
};

__device__ __forceinline__ HugeRegion huge_region(unsigned char* base, uint32_t r) {
    unsigned char* p = base + (uint64_t)r * kHugeRegionBytes;
    HugeRegion h;
    h.best = reinterpret_cast<unsigned long long*>(p);
    p += 8ull * kHugeTargets;
    h.feats = reinterpret_cast<uint32_t*>(p);
    h.locs = h.feats + kHugeFeats;
    h.keys = h.locs + kHugeLocs;
    h.cnt = h.keys + kHugeSlots;
    h.tlist = h.cnt + kHugeSlots;
    return h;
}

// Values written by atomics of this workgroup are read at device scope (not
// from a possibly stale vector L1 line).
__device__ __forceinline__ uint32_t ld_dev(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_dev64(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t loc_slot(uint32_t loc, uint32_t mask) {
    return (loc * 0x9E3779B1u >> 7) & mask;
}

// Window count of `loc` (0 if absent).
__device__ __forceinline__ uint32_t huge_count(const HugeRegion& h, uint32_t mask, uint32_t loc) {
    for (uint32_t i = loc_slot(loc, mask);; i = (i + 1) & mask) {
        const uint32_t k = ld_dev(&h.keys[i]);
        if (k == loc) return ld_dev(&h.cnt[i]);
        if (k == kNone) return 0u;
    }
}

constexpr int kHugeWaves = kHugeThreads / kWave;

struct HugeLds {
    Word stage[kHugeWaves][2 * kStageWords];
    uint32_t scratch[kHugeWaves][kWave];
    uint32_t sk[kHugeWaves][2 * 64];
    unsigned long long red[kHugeWaves];
    uint32_t nfeat, nloc, ntarget, overflow;
    uint32_t sel_t[kMaxTopM], sel_s[kMaxTopM], sel_b[kMaxTopM];
};

// Workgroup maximum of one u64 per thread.
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v,
                                                            unsigned long long* red) {
    v = wave_max_u64(v);
    const uint32_t w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    unsigned long long m = red[0];
    for (int i = 1; i < kHugeWaves; ++i) m = red[i] > m ? red[i] : m;
    return m;
}

template <int KPL, bool C>
__device__ void classify_huge_record(const QueryArgs& a, uint32_t rec, const HugeRegion& h,
                                     HugeLds& L, const Threshold& th) {
    const uint32_t tid = threadIdx.x, lane = (uint32_t)lane_id(), wave = tid >> 6;
    uint64_t o0, o1, o2;
    if (a.paired) {
        o0 = a.offsets[2ull * rec]; o1 = a.offsets[2ull * rec + 1]; o2 = a.offsets[2ull * rec + 2];
    } else {
        o0 = a.offsets[rec]; o1 = a.offsets[rec + 1ull]; o2 = o1;
    }
    // a record of 2^31 bytes or more never comes here (the fast pass counts
    // it as too long); were it to, it is counted the same way (overflow)
    RecordSpan rs;
    const bool spans = record_span(a, o0, o1, o2, rs);
    if (!spans) rs = RecordSpan{0, 0u, {0u, 0u}};
    uint64_t F = (uint64_t)rs.len[0] + rs.len[1];
    if (rs.len[0] > 0 && rs.len[1] > 0 && a.insert_size > F) F = a.insert_size;
    const uint32_t sws = fragment_sws(a, F);
    uint32_t nws[2];
    for (int sg = 0; sg < 2; ++sg)
        nws[sg] = mate_windows32(a, rs.len[sg]);
    const uint32_t nwt = nws[0] + nws[1];
    if (tid == 0) {
        L.nfeat = 0;
        L.nloc = 0;
        L.ntarget = 0;
        L.overflow = spans ? 0u : 1u;
    }
    __syncthreads();

    // sketches of all windows: each wave takes pairs of windows
    for (uint32_t p = 2u * wave; p < nwt; p += 2u * kHugeWaves) {
        WinRef wr[2];
        for (int x = 0; x < 2; ++x) wr[x] = window_ref(a, p + x, nwt, nws[0], rs.r0, rs.len);
        wave_lds_sync();
        bool dirtyA, dirtyB;
        stage_pair(L.stage[wave], rs.base, wr[0], wr[1], (int)lane, dirtyA, dirtyB);
        wave_lds_sync();
        uint32_t nA, nB;
        sketch_pair<KPL>(L.stage[wave], wr[0].x0, wr[0].nk, L.stage[wave] + kStageWords, wr[1].x0,
                         wr[1].nk, a.k, a.s, th, L.sk[wave], L.sk[wave] + 64, L.scratch[wave], nA,
                         nB, dirtyA, dirtyB);
        wave_lds_sync();
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&L.nfeat, nA + nB);
        base = uniform(shfl_idx(base, 0));
        if (base + nA + nB > kHugeFeats) {
            if (lane == 0) L.overflow = 1;
        } else {
            if (lane < nA) h.feats[base + lane] = L.sk[wave][lane];
            if (lane < nB) h.feats[base + nA + lane] = L.sk[wave][64 + lane];
        }
        wave_lds_sync();
    }
    __syncthreads();
    const uint32_t nf = min(L.nfeat, kHugeFeats);

    // lookups: 8-lane groups walk one feature's chain each, appending its
    // locations with an LDS counter
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2* slot2 = reinterpret_cast<const u64x2*>(a.table) + (lane & 7u);
    const uint32_t nb = (uint32_t)a.nb;
    uint32_t probes = 0;
    if constexpr (C) {   // condensed layout: one entry a feature
        const uint4* ent = reinterpret_cast<const uint4*>(a.table) + (lane & 7u);
        for (uint32_t fi = tid >> 3; fi < nf && !L.overflow; fi += kHugeThreads / 8) {
            const uint32_t f = h.feats[fi];
            uint32_t b = (uint32_t)home_bucket(f, a.nb);
            for (;;) {
                const uint4 e = ent[(uint64_t)b * kCondEntries];
                probes += (lane & 7u) == 0 ? 1u : 0u;
                const bool mine = e.x == f && e.y != 0u;
                if (mine) {
                    const uint32_t pos = atomicAdd(&L.nloc, e.y);
                    if (pos + e.y > kHugeLocs) {
                        L.overflow = 1;
                    } else if (e.y <= kCondInline) {
                        h.locs[pos] = e.z;
                        if (e.y == 2u) h.locs[pos + 1] = e.w;
                    } else {
                        const uint64_t off = ((uint64_t)e.w << 32) | e.z;
                        for (uint32_t k = 0; k < e.y; ++k) h.locs[pos + k] = a.cval[off + k];
                    }
                }
                const uint64_t found = ballot(mine);
                const uint32_t last = (lane & ~7u) | 7u;
                const bool full = shfl_idx(e.y != 0u ? 1u : 0u, (int)last) != 0u;
                if (((found >> (lane & ~7u)) & 0xFFull) != 0 || !full) break;
                b = b + 1u == nb ? 0u : b + 1u;
            }
        }
    } else
    for (uint32_t fi = tid >> 3; fi < nf && !L.overflow; fi += kHugeThreads / 8) {
        const uint32_t f = h.feats[fi];
        uint32_t b = (uint32_t)home_bucket(f, a.nb);
        for (;;) {
            const u64x2 sl = slot2[(uint64_t)b * (kSlots / 2)];
            probes += (lane & 7u) == 0 ? 1u : 0u;
            const unsigned long long e[2] = {sl.x, sl.y};
            for (int x = 0; x < 2; ++x) {
                if ((uint32_t)(e[x] >> 32) == f && (uint32_t)e[x] < kTombLoc) {
                    const uint32_t pos = atomicAdd(&L.nloc, 1u);
                    if (pos < kHugeLocs) h.locs[pos] = (uint32_t)e[x];
                    else L.overflow = 1;
                }
            }
            // the group's last lane holds the bucket's last slot: full bucket
            // -> the chain goes on
            const uint32_t last = (lane & ~7u) | 7u;
            const bool full = shfl_idx(sl.y != kEmpty ? 1u : 0u, (int)last) != 0u;
            if (!full) break;
            b = b + 1u == nb ? 0u : b + 1u;
        }
    }
    __syncthreads();
    const uint32_t n = L.nloc;
    if (L.overflow) {
        if (tid == 0) {
            atomicAdd(&a.counters[kQTooLong], 1u);
            a.out_labels[rec] = kNone;
        }
        if (a.out_top && tid < a.top_m) {
            uint32_t* o = a.out_top + ((uint64_t)rec * a.top_m + tid) * 3;
            o[0] = kNone; o[1] = 0u; o[2] = 0u;
        }
        __syncthreads();
        return;
    }

    // window counts: hash table of 2^m >= 2n slots, cleared first
    uint32_t P = 64;
    while (P < 2 * n) P <<= 1;
    const uint32_t mask = P - 1;
    for (uint32_t i = tid; i < P; i += kHugeThreads) {
        h.keys[i] = kNone;
        h.cnt[i] = 0u;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kHugeThreads) {
        const uint32_t loc = h.locs[i];
        for (uint32_t j = loc_slot(loc, mask);; j = (j + 1) & mask) {
            const uint32_t old = atomicCAS(&h.keys[j], kNone, loc);
            if (old == kNone || old == loc) {
                atomicAdd(&h.cnt[j], 1u);
                break;
            }
        }
    }
    __syncthreads();
    // score of the range starting at each distinct location; best per target
    for (uint32_t i = tid; i < P; i += kHugeThreads) {
        const uint32_t loc = ld_dev(&h.keys[i]);
        if (loc == kNone) continue;
        const uint32_t t = loc >> kWindowBits, w = loc & kWindowMask;
        uint32_t score = ld_dev(&h.cnt[i]);
        for (uint32_t d = 1; d < sws && w + d <= kWindowMask; ++d)
            score += huge_count(h, mask, (t << kWindowBits) | (w + d));
        const unsigned long long key = ((unsigned long long)score << 32) | (uint32_t)~loc;
        const unsigned long long old = atomicMax(&h.best[t], key);
        if (old == 0ull) h.tlist[atomicAdd(&L.ntarget, 1u)] = t;
    }
    __syncthreads();

    // top m targets by (score desc, target asc), one workgroup maximum a round
    const uint32_t nt = L.ntarget, top_m = a.top_m;
    uint32_t nsel = 0;
    for (uint32_t m = 0; m < top_m; ++m) {
        unsigned long long key = 0;
        for (uint32_t i = tid; i < nt; i += kHugeThreads) {
            const uint32_t t = h.tlist[i];
            bool excluded = false;
            for (uint32_t x = 0; x < m; ++x) excluded |= L.sel_t[x] == t;
            const unsigned long long ku = ((ld_dev64(&h.best[t]) >> 32) << 32) | (0xFFFFFFFFu - t);
            if (!excluded && ku > key) key = ku;
        }
        key = block_max_u64(key, L.red);
        if (key == 0ull) break;
        if (tid == 0) {
            const uint32_t t = 0xFFFFFFFFu - (uint32_t)key;
            const unsigned long long b = ld_dev64(&h.best[t]);
            L.sel_t[m] = t;
            L.sel_s[m] = (uint32_t)(key >> 32);
            L.sel_b[m] = (~(uint32_t)b) & kWindowMask;
        }
        __syncthreads();
        nsel = m + 1;
    }
    // the bests go back to zero for the next record
    for (uint32_t i = tid; i < nt; i += kHugeThreads) h.best[h.tlist[i]] = 0ull;

    if (tid == 0) {
        uint32_t label = kNone;
        if (nsel > 0 && L.sel_s[0] >= a.min_hits) {
            const uint32_t c1 = L.sel_s[0], c2 = nsel > 1 ? L.sel_s[1] : 0u;
            label = a.target_taxon[L.sel_t[0]];
            if (c1 - c2 <= a.hit_diff)
                for (uint32_t x = 1; x < nsel; ++x)
                    if ((uint64_t)L.sel_s[x] + a.hit_diff >= c1)
                        label = lca(label, a.target_taxon[L.sel_t[x]], a.parents, a.depth);
        }
        a.out_labels[rec] = label;
    }
    if (a.out_top && tid < top_m) {
        const bool hit = tid < nsel;
        uint32_t* o = a.out_top + ((uint64_t)rec * top_m + tid) * 3;
        o[0] = hit ? L.sel_t[tid] : kNone;
        o[1] = hit ? L.sel_s[tid] : 0u;
        o[2] = hit ? L.sel_b[tid] : 0u;
    }
    if (a.qstats) {
        unsigned long long* q = a.qstats + ((blockIdx.x * kHugeWaves + wave) % kQsCopies) * kQsStride;
        for (int m = 1; m < kWave; m <<= 1) probes += shfl_xor(probes, m);
        if (lane == 0 && probes) atomicAdd(&q[kQsProbes], (unsigned long long)probes);
        if (tid == 0) {
            atomicAdd(&q[kQsFeatures], (unsigned long long)nf);
            atomicAdd(&q[kQsLocations], (unsigned long long)n);
        }
    }
    __syncthreads();
}

// Workgroup r uses region r of the huge scratch and takes records r,
// r + kHugeGroups, ... of the HBM-list queue (its ids start at n_records).
template <int KPL, bool C>
__global__ __launch_bounds__(kHugeThreads) void k_classify_huge(QueryArgs a) {
    __shared__ HugeLds L;
    const uint32_t n_iter = uniform(a.counters[kQHuge]);
    const HugeRegion h = huge_region(a.huge, blockIdx.x);
    const Threshold th(a.S, a.s);
    for (uint32_t it = blockIdx.x; it < n_iter; it += gridDim.x)
        classify_huge_record<KPL, C>(a, uniform(a.queue[a.n_records + it]), h, L, th);
}

template <uint32_t LCAP, int WPB, int KPL, bool C>
hipError_t launch_fast_t(const QueryArgs& a, uint32_t max_blocks, int cls, hipStream_t st) {
    uint64_t blocks = ((uint64_t)a.n_records + WPB - 1) / WPB;
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_classify<LCAP, WPB, KPL, C>), dim3((unsigned)blocks), dim3(WPB * 64), 0,
                       st, a, 0, cls);
    return hipGetLastError();
}

// Tuned variants exist for windows of at most 128 k-mers (two per lane); other
// window sizes use the default list capacity and workgroup shape.
template <int KPL, bool C>
hipError_t launch_fast_k(const QueryArgs& a, const ClassifyConfig& c, int cls, hipStream_t st) {
    if constexpr (KPL == 2) {
        const uint32_t key = c.list_cap * 16 + c.waves_per_block;
        switch (key) {
            case 256 * 16 + 2: return launch_fast_t<256, 2, KPL, C>(a, c.max_blocks, cls, st);
            case 256 * 16 + 4: return launch_fast_t<256, 4, KPL, C>(a, c.max_blocks, cls, st);
            case 256 * 16 + 8: return launch_fast_t<256, 8, KPL, C>(a, c.max_blocks, cls, st);
            case 512 * 16 + 2: return launch_fast_t<512, 2, KPL, C>(a, c.max_blocks, cls, st);
            case 512 * 16 + 8: return launch_fast_t<512, 8, KPL, C>(a, c.max_blocks, cls, st);
            case 1024 * 16 + 2: return launch_fast_t<1024, 2, KPL, C>(a, c.max_blocks, cls, st);
            case 1024 * 16 + 4: return launch_fast_t<1024, 4, KPL, C>(a, c.max_blocks, cls, st);
            case 1024 * 16 + 8: return launch_fast_t<1024, 8, KPL, C>(a, c.max_blocks, cls, st);
            default: break;
        }
    }
    return launch_fast_t<kListSmall, 4, KPL, C>(a, c.max_blocks, cls, st);
}

template <int KPL>
hipError_t launch_fast_c(const QueryArgs& a, const ClassifyConfig& c, int cls, hipStream_t st) {
    return a.cval ? launch_fast_k<KPL, true>(a, c, cls, st)
                  : launch_fast_k<KPL, false>(a, c, cls, st);
}

hipError_t launch_fast_any(const QueryArgs& a, const ClassifyConfig& c, int cls, hipStream_t st) {
    if (a.n_records == 0) return hipSuccess;
    if (a.S <= 64) return launch_fast_c<1>(a, c, cls, st);
    if (a.S <= 128) return launch_fast_c<2>(a, c, cls, st);
    return launch_fast_c<4>(a, c, cls, st);
}

// Windows of record rec (both mates), as the classification counts them.
__device__ __forceinline__ uint64_t record_windows(const QueryArgs& a, uint32_t rec) {
    uint64_t o0, o1, o2;
    if (a.paired) {
        o0 = a.offsets[2ull * rec]; o1 = a.offsets[2ull * rec + 1]; o2 = a.offsets[2ull * rec + 2];
    } else {
        o0 = a.offsets[rec]; o1 = a.offsets[rec + 1ull]; o2 = o1;
    }
    if (o1 < o0 || o2 < o1) return 0;
    uint64_t nw = 0;
    const uint64_t len[2] = {o1 - o0, o2 - o1};
    for (int sg = 0; sg < 2; ++sg)
        nw += mate_windows(a, len[sg]);
    return nw;
}

__device__ __forceinline__ uint32_t size_class(uint64_t nw, const RouteConfig& r) {
    for (uint32_t c = 0; c + 1 < r.n; ++c)
        if (nw <= r.max_windows[c]) return c;
    return r.n - 1;
}

// Routing, pass 1: records per size class (wave-aggregated counters).
__global__ __launch_bounds__(256) void k_route_count(QueryArgs a, RouteConfig r) {
    uint32_t cnt[kMaxRoutes] = {0, 0, 0, 0};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_records;
         i += (uint64_t)gridDim.x * blockDim.x)
        cnt[size_class(record_windows(a, (uint32_t)i), r)] += 1;
    for (uint32_t c = 0; c < r.n; ++c) {
        uint32_t v = cnt[c];
#pragma unroll
        for (int m = 1; m < kWave; m <<= 1) v += shfl_xor(v, m);
        if (lane_id() == 0 && v) atomicAdd(&a.route_meta[c], v);
    }
}

// Routing, pass 2: first ids of the classes (their counts' prefix), cursors.
__global__ void k_route_scan(QueryArgs a, RouteConfig r) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (uint32_t c = 0; c < r.n; ++c) {
        a.route_meta[kMaxRoutes + c] = run;
        a.route_meta[2 * kMaxRoutes + c] = run;
        run += a.route_meta[c];
    }
}

// Routing, pass 3: every record's id at its class's cursor.
__global__ __launch_bounds__(256) void k_route_scatter(QueryArgs a, RouteConfig r) {
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < a.n_records; i0 += step) {
        const uint64_t i = i0 + threadIdx.x;
        const bool in = i < a.n_records;
        const uint32_t c = in ? size_class(record_windows(a, (uint32_t)i), r) : kMaxRoutes;
        for (uint32_t k = 0; k < r.n; ++k) {
            const uint64_t m = ballot(c == k);
            if (!m) continue;
            uint32_t base = 0;
            if (lane_id() == 0) base = atomicAdd(&a.route_meta[2 * kMaxRoutes + k], popc64(m));
            base = shfl_idx(base, 0);
            if (c == k) a.route_queue[base + rank_below(m)] = (uint32_t)i;
        }
    }
}

// Workgroups of the large-list pass: one a CU at most (its list takes most of
// a CU's LDS), one per 4,096 records of the launch, 8 to 512. A workgroup of
// this pass can start only on a CU that every other kernel's groups have
// left, so a pass launched next to other batches' kernels (a served mix)
// drains the CUs it is given; the records it takes are rare (none at all in
// the configured workloads, whose lists stay within the fast path's
// capacity), so it is kept small.
inline unsigned large_pass_groups(uint32_t n_records) {
    return (unsigned)std::min<uint32_t>(512u, std::max<uint32_t>(8u, n_records / 4096u));
}

template <bool C>
void launch_large_c(const QueryArgs& a, uint32_t groups, hipStream_t st) {
    const dim3 grid(groups ? std::min<uint32_t>(groups, 512u) : large_pass_groups(a.n_records));
    if (a.S <= 64)
        hipLaunchKernelGGL((k_classify<kListLarge, 1, 1, C>), grid, dim3(64), 0, st, a, 1, -1);
    else if (a.S <= 128)
        hipLaunchKernelGGL((k_classify<kListLarge, 1, 2, C>), grid, dim3(64), 0, st, a, 1, -1);
    else
        hipLaunchKernelGGL((k_classify<kListLarge, 1, 4, C>), grid, dim3(64), 0, st, a, 1, -1);
}

}  // namespace

bool classify_config_valid(const ClassifyConfig& c) {
    return (c.list_cap == 256 || c.list_cap == 512 || c.list_cap == 1024) &&
           (c.waves_per_block == 2 || c.waves_per_block == 4 || c.waves_per_block == 8) &&
           c.max_blocks >= 1;
}

hipError_t launch_classify_fast(const QueryArgs& a, const ClassifyConfig& c, hipStream_t st) {
    return launch_fast_any(a, c, -1, st);
}

hipError_t launch_route(const QueryArgs& a, const RouteConfig& r, hipStream_t st) {
    if (a.n_records == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<uint64_t>(4096, (a.n_records + 255) / 256);
    hipLaunchKernelGGL(k_route_count, dim3(grid), dim3(256), 0, st, a, r);
    hipLaunchKernelGGL(k_route_scan, dim3(1), dim3(64), 0, st, a, r);
    hipLaunchKernelGGL(k_route_scatter, dim3(grid), dim3(256), 0, st, a, r);
    return hipGetLastError();
}

hipError_t launch_classify_class(const QueryArgs& a, const ClassifyConfig& c, uint32_t cls,
                                 hipStream_t st) {
    return launch_fast_any(a, c, (int)cls, st);
}

hipError_t launch_classify_huge(const QueryArgs& a, hipStream_t st) {
    if (a.n_records == 0) return hipSuccess;
    const dim3 grid(a.huge_groups ? a.huge_groups : kHugeGroups), blk(kHugeThreads);
    if (a.cval) {
        if (a.S <= 64) hipLaunchKernelGGL((k_classify_huge<1, true>), grid, blk, 0, st, a);
        else if (a.S <= 128) hipLaunchKernelGGL((k_classify_huge<2, true>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((k_classify_huge<4, true>), grid, blk, 0, st, a);
    } else {
        if (a.S <= 64) hipLaunchKernelGGL((k_classify_huge<1, false>), grid, blk, 0, st, a);
        else if (a.S <= 128) hipLaunchKernelGGL((k_classify_huge<2, false>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((k_classify_huge<4, false>), grid, blk, 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_classify_large(const QueryArgs& a, hipStream_t st, uint32_t groups) {
    if (a.n_records == 0) return hipSuccess;
    if (a.cval) launch_large_c<true>(a, groups, st);
    else launch_large_c<false>(a, groups, st);
    return hipGetLastError();
}

}  // namespace mc
