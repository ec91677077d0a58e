// Device building blocks of the minhash classifier (gfx950, wave64).
//
// Everything here runs inside the library's kernels: 2-bit encoding of ASCII
// text staged in LDS, canonical k-mer extraction by funnel shifts, h1, a
// register bitonic sort across the 64 lanes of a wave, bottom-s selection with
// ballots, and the bucketed open-addressing table (16 x 64-bit slots = one
// 128-byte line per bucket).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_internal.hpp"

namespace mc {

constexpr uint32_t kWindowBits = 18;
constexpr uint32_t kWindowMask = (1u << kWindowBits) - 1;
constexpr uint32_t kNone = 0xFFFFFFFFu;        // unclassified label / unused hit
constexpr uint64_t kEmpty = ~0ull;             // empty table slot
// Location field of a capped-away entry (tombstone). Real locations stay below
// 0xFFFC0000 (targets < 16383), and a tombstone never equals an empty slot,
// not even for feature 0xFFFFFFFF.
constexpr uint32_t kTombLoc = 0xFFFFFFFEu;

// A slot holding a stored pair (neither empty nor a tombstone).
__device__ __forceinline__ bool live_entry(uint64_t e) { return (uint32_t)e < kTombLoc; }

constexpr int kWave = 64;

// ------------------------------------------------------------------ lanes --
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Lanes whose predicate holds (the builtin takes the compare result directly;
// going through an int would materialise it in a VGPR first).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Whether the calling lane's bit of a wave-uniform mask is set (the mask is
// used as the lane predicate as it is, without a per-lane shift and test).
// Combining the ballots of single compares with scalar ANDs, then taking
// lanes from the result, avoids the select-and-compare a ballot of a compound
// predicate compiles to.
__device__ __forceinline__ bool lane_in(uint64_t mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Number of set bits of `mask` in lanes below the calling lane, plus `base`.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask, uint32_t base = 0u) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, base));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint32_t shfl_idx(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

__device__ __forceinline__ uint32_t shfl_xor(uint32_t v, int m) {
    return shfl_idx(v, lane_id() ^ m);
}

// Value of lane (lane ^ M), M a power of two < 64: DPP quad permutes for 1
// and 2, a row rotate for 8 (rotating a 16-lane row by 8 is xor 8),
// ds_swizzle's xor mode for 4 and 16 (within 32-lane halves), and a
// backwards permute for 32.
template <int M>
__device__ __forceinline__ uint32_t xor_lanes(uint32_t v) {
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
    } else if constexpr (M == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, true);
    } else if constexpr (M == 4 || M == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (M << 10) | 0x1F);
    } else {
        return shfl_idx(v, lane_id() ^ M);
    }
}

__device__ __forceinline__ uint32_t xor_lanes_c(uint32_t v, int m) {
    switch (m) {
        case 1: return xor_lanes<1>(v);
        case 2: return xor_lanes<2>(v);
        case 4: return xor_lanes<4>(v);
        case 8: return xor_lanes<8>(v);
        case 16: return xor_lanes<16>(v);
        default: return xor_lanes<32>(v);
    }
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        uint32_t lo = shfl_xor((uint32_t)v, m), hi = shfl_xor((uint32_t)(v >> 32), m);
        uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o > v ? o : v;
    }
    return v;
}

// Maximum over the wave: row rotations by 1, 2, 4 and 8 (DPP) reduce each
// 16-lane row, then the four row results are combined in scalar registers.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    uint32_t o;
    o = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x121, 0xF, 0xF, false); v = v > o ? v : o;
    o = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x122, 0xF, 0xF, false); v = v > o ? v : o;
    o = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, false); v = v > o ? v : o;
    o = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false); v = v > o ? v : o;
    uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    r0 = r0 > r1 ? r0 : r1;
    r2 = r2 > r3 ? r2 : r3;
    return r0 > r2 ? r0 : r2;
}

// Orders LDS accesses of different lanes of one wave (LDS executes a wave's
// operations in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- mixers --
// h1: MurmurHash3's 32-bit finalizer, a bijection on 32-bit words.
__device__ __forceinline__ uint32_t h1(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Slot hash h2 (Sec. 4.1 uses a second hash so that the skewed sketch values
// spread over the table): the two-round xorshift-multiply mixer published as
// "lowbias32" (C. Wellons, hash prospector), a bijection unrelated to h1.
__device__ __forceinline__ uint32_t h2(uint32_t f) {
    f ^= f >> 16;
    f *= 0x7feb352du;
    f ^= f >> 15;
    f *= 0x846ca68bu;
    f ^= f >> 16;
    return f;
}

// Home bucket: floor(h2 * nb / 2^32) (tables have fewer than 2^32 buckets).
__device__ __forceinline__ uint64_t home_bucket(uint32_t f, uint64_t nb) {
    return __umulhi(h2(f), (uint32_t)nb);
}

__device__ __forceinline__ uint64_t next_bucket(uint64_t b, uint64_t nb) {
    return b + 1 == nb ? 0 : b + 1;
}

// ------------------------------------------------------------- encoding --
// 16 bases packed as 2-bit codes (first base in bits 31..30) plus an invalid
// mask with the same layout (0b11 in the two bits of every invalid base), and
// the complements of the same bases in the opposite order (base j of the word
// in bits 2j+1..2j), from which reverse complements are read by a funnel
// shift. A=0 C=1 G=2 T=3, case-insensitive; every other byte is invalid.
struct Word {
    uint32_t code;
    uint32_t mask;
    uint32_t rc;
    uint32_t pad;
};

// The complement word of a code word: every 2-bit group complemented and the
// groups' order reversed (bit reversal, then the two bits of each group
// swapped back).
__device__ __forceinline__ uint32_t rc_word(uint32_t code) {
    const uint32_t r = __builtin_bitreverse32(~code);
    return ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
}

// Four 2-bit fields held in bits 8i..8i+1 (i = byte) packed into one byte,
// byte 0's field in bits 7..6: reverse the bytes, then fold pairs twice.
__device__ __forceinline__ uint32_t pack_fields(uint32_t v) {
    const uint32_t r = __builtin_amdgcn_perm(0u, v, 0x00010203u);
    const uint32_t t = r | (r >> 6);
    return (t | (t >> 12)) & 0xFFu;
}

// Codes of 4 ASCII bytes x (byte 0 = first base). Bits 1..2 of a letter give
// its code, ((x >> 1) ^ (x >> 2)) & 3 maps A/a C/c G/g T/t to 0 1 2 3; a byte
// is a base iff it equals "acgt"[code] once lower-cased (v_perm looks the
// letter up). c: the 4 codes, one per byte (those of non-bases are
// arbitrary). Returns 0x80 in each byte that is not a base.
__device__ __forceinline__ uint32_t codes4(uint32_t x, uint32_t& c) {
    c = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    const uint32_t expect = __builtin_amdgcn_perm(0u, 0x74676361u, c);
    const uint32_t diff = (x | 0x20202020u) ^ expect;           // zero byte: a base
    const uint32_t t = (diff & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    return (t | diff) & 0x80808080u;
}

// Encode 4 ASCII bytes x; ok: 0x80 in each byte that lies inside the
// sequence. c8: the 4 codes (those of invalid bases are arbitrary), first base
// in bits 7..6; m8: 0b11 in the positions of invalid bases; r8: their
// complements, first base in bits 1..0. Returns whether a byte inside the
// sequence is not a base.
__device__ __forceinline__ bool encode4(uint32_t x, uint32_t ok, uint32_t& c8, uint32_t& m8,
                                        uint32_t& r8) {
    uint32_t c;
    const uint32_t bad = codes4(x, c) & ok;                      // 0x80 per non-base inside
    const uint32_t cc = c ^ 0x03030303u;
    const uint32_t t2 = cc | (cc >> 6);
    r8 = (t2 | (t2 >> 12)) & 0xFFu;
    const uint32_t inv = bad | (~ok & 0x80808080u);               // 0x80 per invalid base
    c8 = pack_fields(c);
    m8 = pack_fields((inv >> 6) | (inv >> 7));
    return bad != 0u;
}

// 0x80 in the bytes [lo, hi) of a dword (0 <= lo < hi <= 4).
__device__ __forceinline__ uint32_t inside_bytes(uint32_t lo, uint32_t hi) {
    return (0x80808080u << (8 * lo)) & (0x80808080u >> (8 * (4 - hi)));
}

// Word covering absolute bytes [a, a+16), a 16-byte aligned. Bytes outside
// [vlo, vhi) count as invalid. A word that overlaps [vlo, vhi) is read with
// one 16-byte load: an aligned 16-byte block never crosses a page, so it lies
// in the same mapped page as the valid byte it contains. A word that does not
// overlap is not read at all. `bad` is set if a byte inside [vlo, vhi) is not
// a base. Words wholly inside [vlo, vhi) (nearly all) need no per-byte range
// test, and words without an invalid base no mask packing.
__device__ __forceinline__ Word load_word(uintptr_t a, uintptr_t vlo, uintptr_t vhi, bool& bad) {
    if (a + 16 <= vlo || a >= vhi) return Word{0u, 0xFFFFFFFFu, 0u, 0u};
    // the address is global memory; saying so gives a global (not flat) load
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = *reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(a);
    uint32_t c[4], inv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) inv[i] = codes4(i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w, c[i]);
    if (a < vlo || a + 16 > vhi) {
        // bytes [lo, hi) of the word lie inside [vlo, vhi)
        const uint32_t lo = vlo > a ? (uint32_t)(vlo - a) : 0u;
        const uint32_t hi = vhi - a < 16 ? (uint32_t)(vhi - a) : 16u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t dlo = lo > 4u * i ? min(lo - 4u * i, 4u) : 0u;
            const uint32_t dhi = hi > 4u * i ? min(hi - 4u * i, 4u) : 0u;
            const uint32_t ok = dlo < dhi ? inside_bytes(dlo, dhi) : 0u;
            bad |= (inv[i] & ok) != 0u;
            inv[i] = (inv[i] & ok) | (~ok & 0x80808080u);
        }
    } else {
        bad |= (inv[0] | inv[1] | inv[2] | inv[3]) != 0u;
    }
    Word w;
    w.code = (pack_fields(c[0]) << 24) | (pack_fields(c[1]) << 16) | (pack_fields(c[2]) << 8) |
             pack_fields(c[3]);
    w.mask = 0u;
    if ((inv[0] | inv[1] | inv[2] | inv[3]) != 0u) {
        uint32_t m = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) m = (m << 8) | pack_fields((inv[i] >> 6) | (inv[i] >> 7));
        w.mask = m;
    }
    w.rc = rc_word(w.code);
    w.pad = 0u;
    return w;
}

// Stage one dword (4 bases) of a word covering [A0, ...): dword d of word
// d >> 2 goes to byte 3 - (d & 3) of that word's code and mask (first base in
// the top byte) and to byte d & 3 of its complement word. Positions are
// 32-bit offsets from `base` (16-byte aligned), A0 a multiple of 16. Bytes
// outside [vlo, vhi) count as invalid; a dword that does not overlap them is
// not read. Aligned 4-byte loads never cross a page. Returns whether a byte
// inside [vlo, vhi) is not a base.
__device__ __forceinline__ uint32_t stage_dword(Word* W, uintptr_t base, uint32_t A0, uint32_t d,
                                                uint32_t vlo, uint32_t vhi) {
    const uint32_t a = A0 + 4u * d;
    // every lane loads (no branch): a dword outside [vlo, vhi) reads the
    // nearest dword that overlaps it (vlo < vhi) and marks all its bytes
    // invalid; its codes are then arbitrary
    const uint32_t ac = min(max(a, vlo & ~3u), (vhi - 1u) & ~3u);
    const uint32_t x = *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(base + ac);
    const uint32_t lo = vlo > a ? min(vlo - a, 4u) : 0u;
    const uint32_t hi = vhi > a ? min(vhi - a, 4u) : 0u;
    uint32_t c8, m8, r8;
    const bool bad = encode4(x, lo < hi ? inside_bytes(lo, hi) : 0u, c8, m8, r8);
    uint8_t* w = reinterpret_cast<uint8_t*>(W + (d >> 2));
    w[3 - (d & 3u)] = (uint8_t)c8;
    w[7 - (d & 3u)] = (uint8_t)m8;
    w[8 + (d & 3u)] = (uint8_t)r8;
    return bad ? 1u : 0u;
}

// Canonical k-mer (k <= 16) starting o bases into word pair (a, b), both
// strands by a funnel shift: the forward k-mer is the top 2k bits of
// (a:b) << 2o, the reverse complement (its first base the complement of the
// k-mer's last) comes from the complement words, kmask = 4^k - 1. lo is b for
// o > 0 and a itself for o = 0: the forward funnel shift by 32 - 2o (taken mod
// 32) then needs no select between its two cases. Without kCheck the caller
// knows every base of the k-mer is valid; with it, returns false if one is
// not.
template <bool kCheck>
__device__ __forceinline__ bool kmer_of(const Word& a, const Word& lo, const Word& b, uint32_t o,
                                        uint32_t k, uint32_t kmask, uint32_t& canon) {
    const uint32_t top = __builtin_amdgcn_alignbit(a.code, lo.code, 32u - 2u * o);
    const uint32_t fwd = top >> (32 - 2 * k);
    bool bad = false;
    if constexpr (kCheck) {
        const uint32_t mtop = __builtin_amdgcn_alignbit(a.mask, lo.mask, 32u - 2u * o);
        bad = (mtop >> (32 - 2 * k)) != 0u;
    }
    const uint32_t r = __builtin_amdgcn_alignbit(b.rc, a.rc, 2u * o) & kmask;
    canon = fwd < r ? fwd : r;
    return !bad;
}

__device__ __forceinline__ uint32_t kmer_mask(uint32_t k) {
    return k >= 16 ? 0xFFFFFFFFu : (1u << (2 * k)) - 1u;
}

// Canonical k-mer starting x bases after the first staged word (k <= 16).
// Returns false if any of its bases is invalid.
__device__ __forceinline__ bool kmer_at(const Word* W, uint32_t x, uint32_t k, uint32_t& canon) {
    const uint32_t q = x >> 4, o = x & 15u;
    return kmer_of<true>(W[q], W[q + (o != 0u)], W[q + 1], o, k, kmer_mask(k), canon);
}

// ------------------------------------------------------- bitonic in regs --
// Lanes of a compare-exchange step of a bitonic network that keep the smaller
// key: those whose block of `size` runs ascending ((element & size) == 0) and
// that are the lower partner ((lane & stride) == 0), or neither. The elements
// are r * 64 + lane, or, for two independent 32-lane networks (halves), lane
// & 31. A constant of the step.
__host__ __device__ constexpr uint64_t keep_low_lanes(int size, int stride, int r,
                                                      bool halves = false) {
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l) {
        const int e = halves ? (l & 31) : r * 64 + l;
        const bool asc = (e & size) == 0;
        const bool lower = (l & stride) == 0;
        if (asc == lower) m |= 1ull << l;
    }
    return m;
}
static_assert(keep_low_lanes(2, 1, 0) == 0x9999999999999999ull, "first step: up, down, ...");
static_assert(keep_low_lanes(64, 32, 0) == 0x00000000FFFFFFFFull, "last merge runs ascending");
static_assert(keep_low_lanes(64, 1, 1) == 0xAAAAAAAAAAAAAAAAull, "second register descends");
static_assert(keep_low_lanes(32, 16, 0, true) == 0x0000FFFF0000FFFFull,
              "both halves' last merge runs ascending");
static_assert(keep_low_lanes(16, 8, 0, true) == keep_low_lanes(16, 8, 0), "halves agree below 32");

// Compile-time check of the step masks: the networks of wave_sort (KPL keys a
// lane) and wave_sort_halves, run on the host over a few key patterns with
// these masks, leave every sequence ascending.
template <int KPL>
constexpr bool bitonic_masks_sort(bool halves, uint32_t seed) {
    constexpr int N = 64 * KPL;
    uint32_t v[N] = {};
    for (int e = 0; e < N; ++e) v[e] = ((uint32_t)e * 2654435761u + seed) % 97u;   // duplicates too
    const int top = halves ? 32 : N;
    for (int size = 2; size <= top; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            uint64_t mask[KPL] = {};
            for (int r = 0; r < KPL && stride < 64; ++r)
                mask[r] = keep_low_lanes(size, stride, r, halves);
            uint32_t nv[N] = {};
            for (int e = 0; e < N; ++e) {
                const int r = e / 64, l = e % 64;
                const uint32_t o = v[e ^ stride];
                const uint32_t lo = v[e] < o ? v[e] : o, hi = v[e] < o ? o : v[e];
                const bool low = stride >= 64
                                     ? ((((r * 64) & size) == 0) == ((e & stride) == 0))
                                     : ((mask[r] >> l) & 1u) != 0;
                nv[e] = low ? lo : hi;
            }
            for (int e = 0; e < N; ++e) v[e] = nv[e];
        }
    for (int e = 1; e < N; ++e)
        if ((!halves || (e & 31) != 0) && v[e - 1] > v[e]) return false;
    return true;
}
static_assert(bitonic_masks_sort<1>(false, 0) && bitonic_masks_sort<1>(false, 5),
              "64-key network");
static_assert(bitonic_masks_sort<2>(false, 1) && bitonic_masks_sort<4>(false, 3),
              "128- and 256-key networks");
static_assert(bitonic_masks_sort<1>(true, 0) && bitonic_masks_sort<1>(true, 7),
              "two 32-key networks");

// The lanes of a constant 64-bit mask as a per-lane predicate. The mask is
// written by two scalar moves of immediates where it is used (volatile, so
// they are not hoisted): a mask computed once outside the enclosing loops
// would stay live in scalar registers across them and be spilled.
__device__ __forceinline__ bool lanes_of(uint64_t mask) {
    uint32_t lo, hi;
    asm volatile("s_mov_b32 %0, %1" : "=s"(lo) : "i"((uint32_t)mask));
    asm volatile("s_mov_b32 %0, %1" : "=s"(hi) : "i"((uint32_t)(mask >> 32)));
    return __builtin_amdgcn_inverse_ballot_w64(((uint64_t)hi << 32) | lo);
}

// Ascending sort of 64*KPL keys held KPL per lane; element index r*64 + lane.
template <int KPL>
__device__ __forceinline__ void wave_sort(uint32_t (&v)[KPL]) {
    constexpr int N = kWave * KPL;
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= kWave) {
                const int rs = stride / kWave;
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    const int p = r ^ rs;
                    if (p > r) {
                        const bool asc = ((r * kWave) & size) == 0;
                        uint32_t a = v[r], b = v[p];
                        uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                        v[r] = asc ? lo : hi;
                        v[p] = asc ? hi : lo;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    uint32_t o = xor_lanes_c(v[r], stride);
                    uint32_t lo = v[r] < o ? v[r] : o, hi = v[r] < o ? o : v[r];
                    v[r] = lanes_of(keep_low_lanes(size, stride, r)) ? lo : hi;
                }
            }
        }
    }
}

// After wave_sort: write the s smallest distinct keys (0xFFFFFFFF excluded)
// to sk[0..] in ascending order and return their number; `distinct` receives
// the number of distinct keys below 0xFFFFFFFF. If a valid k-mer hashed to
// 0xFFFFFFFF (has_top) and fewer than s smaller distinct values exist, that
// value is appended as the last element.
template <int KPL>
__device__ __forceinline__ uint32_t select_distinct(const uint32_t (&v)[KPL], bool has_top,
                                                    uint32_t s, uint32_t* sk,
                                                    uint32_t& distinct) {
    const int lane = lane_id();
    uint32_t base = 0, prev_last = 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        uint32_t up = shfl_idx(v[r], lane > 0 ? lane - 1 : 0);
        bool has_prev = lane > 0 || r > 0;
        uint32_t prev = lane > 0 ? up : prev_last;
        bool first = v[r] != 0xFFFFFFFFu && (!has_prev || v[r] != prev);
        uint64_t bal = ballot(first);
        uint32_t rank = base + rank_below(bal);
        if (first && rank < s) sk[rank] = v[r];
        base += popc64(bal);
        prev_last = (uint32_t)__builtin_amdgcn_readlane((int)v[r], kWave - 1);
    }
    distinct = base;
    uint32_t n = base < s ? base : s;
    if (has_top && base < s) {
        if (lane == 0) sk[base] = 0xFFFFFFFFu;
        n = base + 1;
    }
    return n;
}

// Hash threshold below which about `expect` of the nk hashes of a window are
// expected (uniform hashes). Any value is correct: callers verify that enough
// distinct candidates fell below it and otherwise take every hash.
__device__ __forceinline__ uint32_t hash_threshold(float expect, uint32_t nk) {
    const float t = expect * 4294967296.0f / (float)nk;
    return t >= 4294967040.0f ? 0xFFFFFFFFu : (uint32_t)t;
}

// Candidate threshold of sketch_pair (hash_threshold of 1.5 s): computed once
// for the full window of S k-mers, divided out only for shorter windows.
struct Threshold {
    uint32_t S, tS;
    __device__ __forceinline__ Threshold(uint32_t S_, uint32_t s)
        : S(S_), tS(hash_threshold(1.5f * (float)s, S_)) {}
    __device__ __forceinline__ uint32_t of(uint32_t nk, uint32_t s) const {
        if (nk == S) return tS;
        return hash_threshold(1.5f * (float)s, nk);
    }
};

// h1 of the canonical k-mers of one window whose nk k-mer starts begin x0
// bases after the first staged word: key[r] belongs to k-mer r*64 + lane and is
// 0xFFFFFFFF for an invalid k-mer or past nk. Returns whether some valid k-mer
// hashed to 0xFFFFFFFF (that value then still counts as a distinct feature).
// kCheck = false: the caller knows the window holds no invalid base. K-mer
// r*64 + lane starts 4r words after k-mer lane, at the same offset in its word.
// kAll: every lane hashes, with no branch around lanes past nk (they read
// staged words beyond the window and drop them; W must then hold 4 * KPL + 2
// words from the window's first word on, x0 < 16). That saves the scalar
// branch work per key where vector issue has room (the build); without it,
// lanes past nk skip the hash.
template <int KPL, bool kCheck, bool kAll = false>
__device__ __forceinline__ bool window_keys_t(const Word* W, uint32_t x0, uint32_t nk, uint32_t k,
                                              uint32_t (&key)[KPL]) {
    const int lane = lane_id();
    const uint32_t x = x0 + (uint32_t)lane;
    const Word* Wq = W + (x >> 4);
    const uint32_t o = x & 15u;
    const Word* Wl = Wq + (o != 0u);
    const uint32_t kmask = kmer_mask(k);
    if constexpr (kAll) {
        uint32_t top = 0u;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const uint32_t i = (uint32_t)(r * kWave + lane);
            uint32_t c;
            const bool ok = kmer_of<kCheck>(Wq[4 * r], Wl[4 * r], Wq[4 * r + 1], o, k, kmask, c);
            const uint32_t h = h1(c);
            const bool use = i < nk && ok;
            key[r] = use ? h : 0xFFFFFFFFu;
            top |= use && h == 0xFFFFFFFFu ? 1u : 0u;
        }
        return ballot(top != 0u) != 0;
    } else {
        bool top = false;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const uint32_t i = (uint32_t)(r * kWave + lane);
            key[r] = 0xFFFFFFFFu;
            if (i < nk) {
                uint32_t c;
                if (kmer_of<kCheck>(Wq[4 * r], Wl[4 * r], Wq[4 * r + 1], o, k, kmask, c)) {
                    const uint32_t h = h1(c);
                    key[r] = h;
                    top |= (h == 0xFFFFFFFFu);
                }
            }
        }
        return ballot(top) != 0;
    }
}

template <int KPL>
__device__ __forceinline__ bool window_keys(const Word* W, uint32_t x0, uint32_t nk, uint32_t k,
                                            uint32_t (&key)[KPL]) {
    return window_keys_t<KPL, true>(W, x0, nk, k, key);
}

// The s smallest distinct keys of one window (its nk keys as left by
// window_keys) into sk[0..), ascending; returns their number. scratch: 64
// words of LDS owned by the wave.
//
// For windows of more than 64 k-mers the wave first keeps only hashes below a
// threshold chosen so that about 1.75 s of them are expected; if at least s
// distinct values lie below it, the s smallest of the window are exactly the s
// smallest of those candidates, which fit one per lane. Otherwise (fewer than
// s distinct candidates, or more than 64) it sorts every hash of the window.
template <int KPL>
__device__ __forceinline__ uint32_t sketch_keys(uint32_t (&key)[KPL], uint32_t nk, bool has_top,
                                                uint32_t s, uint32_t* sk, uint32_t* scratch) {
    const int lane = lane_id();
    uint32_t distinct;
    if constexpr (KPL >= 2) {
        if (nk > (uint32_t)kWave) {
            const uint32_t T = hash_threshold(1.75f * (float)s, nk);
            uint64_t bal[KPL];
            uint32_t c = 0;
#pragma unroll
            for (int r = 0; r < KPL; ++r) {
                bal[r] = ballot(key[r] < T);
                c += popc64(bal[r]);
            }
            if (c >= s && c <= (uint32_t)kWave) {
                uint32_t base = 0;
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    if (key[r] < T) scratch[base + rank_below(bal[r])] = key[r];
                    base += popc64(bal[r]);
                }
                wave_lds_sync();
                uint32_t v[1] = {(uint32_t)lane < c ? scratch[lane] : 0xFFFFFFFFu};
                wave_lds_sync();
                wave_sort<1>(v);
                uint32_t n = select_distinct<1>(v, false, s, sk, distinct);
                if (distinct >= s) return n;
            }
        }
        if (nk <= (uint32_t)kWave) {   // one key per lane: a 64-wide sort suffices
            uint32_t v[1] = {key[0]};
            wave_sort<1>(v);
            return select_distinct<1>(v, has_top, s, sk, distinct);
        }
    }
    wave_sort<KPL>(key);
    return select_distinct<KPL>(key, has_top, s, sk, distinct);
}

// Sketch of one window (B2-B4, Q2).
template <int KPL>
__device__ __forceinline__ uint32_t sketch_window(const Word* W, uint32_t x0, uint32_t nk,
                                                  uint32_t k, uint32_t s, uint32_t* sk,
                                                  uint32_t* scratch) {
    uint32_t key[KPL];
    const bool top = window_keys<KPL>(W, x0, nk, k, key);
    return sketch_keys<KPL>(key, nk, top, s, sk, scratch);
}

// Out-of-line copy for rare paths, so that the hot loops stay small in the
// instruction cache. Its pointers are LDS pointers (address space 3), so that
// the out-of-line code still uses LDS instructions rather than flat ones.
#define MC_LDS __attribute__((address_space(3)))
template <int KPL>
__device__ __attribute__((noinline)) uint32_t sketch_window_lds(const MC_LDS Word* W, uint32_t x0,
                                                                uint32_t nk, uint32_t k,
                                                                uint32_t s, MC_LDS uint32_t* sk,
                                                                MC_LDS uint32_t* scratch) {
    return sketch_window<KPL>((const Word*)W, x0, nk, k, s, (uint32_t*)sk, (uint32_t*)scratch);
}

template <int KPL>
__device__ __forceinline__ uint32_t sketch_window_rare(const Word* W, uint32_t x0, uint32_t nk,
                                                       uint32_t k, uint32_t s, uint32_t* sk,
                                                       uint32_t* scratch) {
    return sketch_window_lds<KPL>((const MC_LDS Word*)W, x0, nk, k, s, (MC_LDS uint32_t*)sk,
                                  (MC_LDS uint32_t*)scratch);
}

// Ascending bitonic sort of each 32-lane half of the wave (one key per lane).
__device__ __forceinline__ void wave_sort_halves(uint32_t& v) {
#pragma unroll
    for (int size = 2; size <= 32; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            uint32_t o = xor_lanes_c(v, stride);
            uint32_t lo = v < o ? v : o, hi = v < o ? o : v;
            v = lanes_of(keep_low_lanes(size, stride, 0, true)) ? lo : hi;
        }
    }
}

// Candidates of one window for a 32-entry half of scratch. A window of at
// most 32 k-mers contributes all its keys (mode 0, exact). A longer one
// contributes its keys below a threshold that about 1.5 s of them pass (mode
// 1), valid only if at least s distinct values end up below it; if fewer than
// s or more than 32 keys pass, it contributes nothing (mode 2) and is
// sketched on its own. Returns the number of entries written.
template <int KPL>
__device__ __forceinline__ uint32_t half_candidates(const uint32_t (&key)[KPL], uint32_t nk,
                                                    uint32_t s, const Threshold& th,
                                                    uint32_t* half, int& mode) {
    const int lane = lane_id();
    if (nk <= 32u) {
        if (lane < 32) half[lane] = key[0];
        mode = 0;
        return 32u;
    }
    const uint32_t T = th.of(nk, s);
    uint64_t bal[KPL];
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        bal[r] = ballot(key[r] < T);
        c += popc64(bal[r]);
    }
    if (c < s || c > 32u) {
        mode = 2;
        return 0u;
    }
    uint32_t base = 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (key[r] < T) half[rank_below(bal[r], base)] = key[r];
        base += popc64(bal[r]);
    }
    mode = 1;
    return c;
}

// Sketches of two windows A and B (either may be empty, nk = 0) at once: the
// candidates of A fill lanes 0..31 and those of B lanes 32..63, one 32-wide
// sort orders both halves, and one ballot ranks the distinct values of both.
// A window whose candidates do not decide its sketch is redone alone (its
// staged words must still be in place). All pointers are to LDS. Writes
// skA[0..nA) and skB[0..nB). scratch: 64 words of LDS owned by the wave.
// dirtyA / dirtyB (wave-uniform): the window may hold an invalid base; when
// false its k-mers skip the validity test. kAll: as for window_keys_t.
template <int KPL, bool kAll = false>
__device__ __forceinline__ void sketch_pair(const Word* WA, uint32_t xA, uint32_t nkA,
                                            const Word* WB, uint32_t xB, uint32_t nkB,
                                            uint32_t k, uint32_t s, const Threshold& th,
                                            uint32_t* skA, uint32_t* skB,
                                            uint32_t* scratch, uint32_t& nA, uint32_t& nB,
                                            bool dirtyA = true, bool dirtyB = true) {
    const int lane = lane_id();
    int modeA, modeB;
    uint32_t cA, cB;
    bool topA, topB;
    {
        uint32_t key[KPL];
        topA = dirtyA ? window_keys_t<KPL, true, kAll>(WA, xA, nkA, k, key)
                      : window_keys_t<KPL, false, kAll>(WA, xA, nkA, k, key);
        cA = half_candidates<KPL>(key, nkA, s, th, scratch, modeA);
        topB = dirtyB ? window_keys_t<KPL, true, kAll>(WB, xB, nkB, k, key)
                      : window_keys_t<KPL, false, kAll>(WB, xB, nkB, k, key);
        cB = half_candidates<KPL>(key, nkB, s, th, scratch + 32, modeB);
    }
    wave_lds_sync();
    const uint32_t hl = (uint32_t)lane & 31u;
    uint32_t v = hl < (lane < 32 ? cA : cB) ? scratch[lane] : 0xFFFFFFFFu;
    wave_lds_sync();
    wave_sort_halves(v);
    // previous lane's key (whole-wave shift right by one lane)
    const uint32_t prev = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, false);
    // first of its value in its half: not the padding key, and lane 0 of the
    // half or unlike the lane before
    const uint64_t bal = ballot(v != 0xFFFFFFFFu) & (ballot(v != prev) | 0x0000000100000001ull);
    const bool first = lane_in(bal);
    const uint32_t dA = popc64(bal & 0xFFFFFFFFull), dB = popc64(bal >> 32);
    const bool okA = modeA == 0 || (modeA == 1 && dA >= s);
    const bool okB = modeB == 0 || (modeB == 1 && dB >= s);
    const uint32_t rank = rank_below(bal) - (lane < 32 ? 0u : dA);
    if (first && rank < s) {
        if (lane < 32) {
            if (okA) skA[rank] = v;
        } else if (okB) {
            skB[rank] = v;
        }
    }
    nA = dA < s ? dA : s;
    nB = dB < s ? dB : s;
    if (okA && topA && dA < s) {
        if (lane == 0) skA[dA] = 0xFFFFFFFFu;
        nA = dA + 1;
    }
    if (okB && topB && dB < s) {
        if (lane == 0) skB[dB] = 0xFFFFFFFFu;
        nB = dB + 1;
    }
    // rare: the keys of an undecided window are recomputed from the staged words
    if (!okA) {
        wave_lds_sync();
        nA = uniform(sketch_window_rare<KPL>(WA, xA, nkA, k, s, skA, scratch));
    }
    if (!okB) {
        wave_lds_sync();
        nB = uniform(sketch_window_rare<KPL>(WB, xB, nkB, k, s, skB, scratch));
    }
    // the counts are wave-uniform; saying so keeps the callers' loops scalar
    nA = uniform(nA);
    nB = uniform(nB);
}

// Stage the bytes [lo, hi) into words relative to A0 = lo & ~15, one word per
// participating thread (tid in [0, nthreads)); bytes outside [vlo, vhi) are
// invalid. Returns whether a word of this thread holds a byte inside
// [vlo, vhi) that is not a base; callers synchronise before reading W.
__device__ __forceinline__ bool stage_words(Word* W, uintptr_t lo, uintptr_t hi, uintptr_t vlo,
                                            uintptr_t vhi, int tid, int nthreads) {
    uintptr_t A0 = lo & ~(uintptr_t)15;
    int nw = (int)((hi - A0 + 15) / 16) + 1;
    bool bad = false;
    for (int q = tid; q < nw; q += nthreads)
        W[q] = load_word(A0 + 16 * (uintptr_t)q, vlo, vhi, bad);
    return bad;
}

// ------------------------------------------------------------ LCA / taxa --
__device__ __forceinline__ uint32_t lca(uint32_t a, uint32_t b, const uint32_t* parent,
                                        const uint32_t* depth) {
    uint32_t da = depth[a], db = depth[b];
    while (da > db) { a = parent[a]; --da; }
    while (db > da) { b = parent[b]; --db; }
    while (a != b) { a = parent[a]; b = parent[b]; }
    return a;
}

}  // namespace mc
