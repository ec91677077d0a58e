// Launch interfaces between the host-side C ABI (mc_api.hip) and the kernel
// translation units (mc_build.hip, mc_query.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct mc_db;

namespace mc {

constexpr int kSlots = 16;   // 64-bit slots per table bucket (one 128-byte line)

// One reference sequence of an add call.
struct TargetDesc {
    uint64_t off;        // byte offset of the sequence in the call's text buffer
    uint64_t len;        // bases
    uint64_t win_base;   // index of its window 0 among all windows of the call
    uint32_t id;         // global target id
    uint32_t nw;         // windows
};

// Build-side counters (device, u64).
enum BuildCounter {
    kCntInserted = 0,    // pairs inserted
    kCntProbe = 1,       // sum over inserts of (buckets probed - 1)
    kCntCand = 2,        // cap candidates pushed (may exceed the list capacity)
    kCntFull = 3,        // inserts that found no free slot
    kCntMoved = 4,       // entries re-inserted by a rehash
    kCntDefer = 5,       // slice-local inserts whose chain ran past their slice
    kNumBuildCounters = 8
};

struct BuildArgs {
    const uint8_t* text;
    uint64_t text_len;
    const TargetDesc* targets;
    uint32_t n_targets;
    const uint64_t* tile_first;   // n_targets + 1 prefix of tiles per target
    uint64_t n_tiles;
    uint32_t k, w, S, s;
    // insert mode
    unsigned long long* table;
    uint32_t* bcount;             // per-bucket fill counters (slots claimed)
    uint64_t nb;                  // buckets
    uint32_t cap_dist;            // inserts at this probe distance or more are cap candidates
    uint32_t* cand;
    uint64_t cand_cap;
    unsigned long long* counters;
    // sketch-export mode
    uint32_t* out_counts;
    uint32_t* out_feats;
    // pair mode: per-window pairs, their partition histogram, partitioned copy
    unsigned long long* pairs;          // n_windows * s slots
    unsigned long long* parted;         // pairs in partition order
    uint32_t part_shift;                // partition of a pair: home bucket >> part_shift
    uint32_t n_parts;                   // partitions (<= kMaxParts)
    uint32_t chunk_tiles;               // sketch tiles per level-1 scatter chunk
    uint64_t* chunk_slot;               // first slot of each level-1 scatter chunk, then
                                        // the end of the slots (n_chunks + 1)
    uint32_t* hist;                     // pairs per (scatter group g, partition p) at
                                        // g * kMaxParts + p
    unsigned long long* part_start;     // n_parts + 1 offsets
    unsigned long long* cursor;         // scatter cursor of (g, p) at g * kMaxParts + p
    // slice mode: partitions split into 2^fine_bits slices of 2^slice_shift
    // buckets each; a workgroup inserts one slice's pairs with LDS counters
    uint32_t slice_mode;
    uint32_t slice_shift;
    uint32_t fine_bits;                 // part_shift = slice_shift + fine_bits
    uint32_t* hist2;                    // n_parts << fine_bits counters
    unsigned long long* slice_start;    // (n_parts << fine_bits) + 1 offsets
    unsigned long long* cursor2;        // n_parts << fine_bits scatter cursors
    unsigned long long* chunk_first;    // [0, n_parts]: prefix of histogram chunks per
                                        // partition; [kMaxParts + 1, ...]: scatter chunks;
                                        // [kChunkMaxAt]: most scatter chunks of a partition
    uint32_t fresh;                     // slice mode: table and counters uncleared; the
                                        // insert writes every bucket of every slice
    // forced by mc_db_set_insert_path (tests): LDS staging entries of the slice
    // insert (0 = as many as fit) and the direct path for every slice
    uint32_t stage_entries;
    uint32_t force_direct;
};

constexpr uint32_t kMaxParts = 256;         // partitions (8 bits)
constexpr uint32_t kMaxFineBits = 10;       // slices per partition: at most 1024
// Level-1 scatter chunks are spread over kScatGroups cursor sets (chunk m
// uses set m % kScatGroups), so the chunks in flight do not all serialise on
// the same 256 atomics.
constexpr uint32_t kScatGroups = 8;
constexpr uint32_t kChunkFirstLen = 2 * (kMaxParts + 1) + 1;
constexpr uint32_t kChunkMaxAt = 2 * (kMaxParts + 1);
constexpr uint32_t kMaxSliceShift = 13;     // slice of at most 8192 buckets (32 KiB counters)
constexpr uint32_t kMinSliceShift = 10;
constexpr uint32_t kMaxSlices = kMaxParts << kMaxFineBits;

constexpr int kTileWindows = 32;  // windows per build workgroup tile
constexpr int kBuildThreads = 256;
constexpr int kScatThreads = 1024;                     // scatter workgroup (one per CU)
constexpr int kScatPer = 16;                           // pairs per thread held in registers
constexpr int kScatChunk = kScatThreads * kScatPer;    // most pairs of a scatter chunk
// Sketch tiles per level-1 scatter chunk (a tile holds at most 32 * s slots).
inline uint32_t scatter_chunk_tiles(uint32_t s) {
    const uint32_t c = (uint32_t)kScatChunk / ((uint32_t)kTileWindows * s);
    return c ? c : 1u;
}

// Query-side counters (device, u32).
enum QueryCounter {
    kQOverflow = 0,      // records queued for the large-list pass
    kQHuge = 1,          // records queued for the HBM-list pass
    kQTooLong = 2,       // records beyond every pass's capacity (left unclassified)
    kNumQueryCounters = 4
};

// HBM-list pass: one workgroup a record, its lists in device memory. Each of
// kHugeGroups workgroups owns one region of the workspace's huge scratch.
constexpr int kHugeThreads = 256;
constexpr uint32_t kHugeGroups = 4;
constexpr uint32_t kHugeFeats = 1u << 14;      // sketch elements of one record
constexpr uint32_t kHugeLocs = 1u << 20;       // candidate locations of one record
constexpr uint32_t kHugeSlots = 2 * kHugeLocs; // counting hash table (keys + counts)
constexpr uint32_t kHugeTargets = 16384;       // per-target best range (> MC_MAX_TARGETS)
// Bytes of one region: features, locations, hash keys, hash counts (u32 each),
// per-target best (u64) and the list of targets hit (u32).
constexpr uint64_t kHugeRegionBytes =
    4ull * (kHugeFeats + kHugeLocs + 2ull * kHugeSlots) + 8ull * kHugeTargets + 4ull * kHugeTargets;
constexpr uint64_t kHugeBytes = kHugeRegionBytes * kHugeGroups;

// Unsigned 32-bit division by a divisor fixed per database (the window
// stride) as a multiply-high and two shifts: with L = ceil(log2 d) and
// m = floor(2^32 (2^L - d) / d) + 1, floor(n / d) = (t + ((n - t) >> min(L, 1)))
// >> max(L - 1, 0) where t = floor(m n / 2^32), for every 32-bit n (Granlund
// and Montgomery, PLDI 1994). Uniform operands keep it in scalar registers.
struct DivU32 {
    uint32_t m = 1, sh1 = 0, sh2 = 0;
};

inline DivU32 make_divu32(uint32_t d) {
    uint32_t L = 0;
    while ((1ull << L) < d) ++L;
    DivU32 r;
    r.m = (uint32_t)(((1ull << 32) * ((1ull << L) - d)) / d + 1);
    r.sh1 = L ? 1u : 0u;
    r.sh2 = L ? L - 1u : 0u;
    return r;
}

struct QueryArgs {
    const unsigned long long* table;
    uint64_t nb;
    const uint8_t* reads;
    const uint64_t* offsets;
    uint32_t n_records;
    uint32_t paired;
    uint32_t k, w, S, s;
    DivU32 divS;                  // division by S
    uint32_t top_m, min_hits, hit_diff, insert_size;
    const uint32_t* target_taxon;
    const uint32_t* parents;
    const uint32_t* depth;
    uint32_t* out_labels;
    uint32_t* out_top;            // n_records * top_m * 3 u32, or null
    uint32_t* queue;              // record ids: [0, n) large-list pass, [n, 2n) HBM-list pass
    uint32_t* counters;
    unsigned long long* qstats;   // kQsWords: kQsCopies partial totals (or null)
    unsigned char* huge;          // HBM-list scratch: huge_groups regions of kHugeRegionBytes
                                  // (per-target bests zero)
    uint32_t huge_groups;         // regions (workgroups of the HBM-list pass), 0 = kHugeGroups
    // condensed layout (when cval is set): `table` holds nb index buckets of
    // kCondEntries 16-byte entries, and cval the runs of locations
    const uint32_t* cval;
    // size classes (routed launches): record ids grouped by class, and per
    // class c its count at route_meta[c] and first id at route_meta[kMaxRoutes + c]
    uint32_t* route_queue;
    uint32_t* route_meta;         // kRouteMetaWords
};

// Routing of records into size classes by their number of windows: class c
// takes the records with at most max_windows[c] windows not taken by an
// earlier class (the last class takes the rest); each class has its own
// launch shape.
constexpr uint32_t kMaxRoutes = 4;
constexpr uint32_t kRouteMetaWords = 3 * kMaxRoutes;   // counts, first ids, cursors
struct RouteConfig {
    uint32_t n = 1;
    uint32_t max_windows[kMaxRoutes] = {0, 0, 0, 0};
};

// Totals kept by the classify passes: sketch elements looked up, locations
// gathered, bucket lines read, and records handed on to the large-list pass
// and to the HBM-list pass.
enum QueryStat {
    kQsFeatures = 0, kQsLocations = 1, kQsProbes = 2, kQsLarge = 3, kQsHuge = 4,
    kNumQueryStats = 5
};
// The query statistics are kept as kQsCopies partial totals, each on its own
// 128-byte line: a wave adds its counts to copy (wave id mod kQsCopies), so
// the waves of a launch do not all queue their atomics on one line (at about
// 12 ns an atomic, three a wave cost a launch of 16,384 four-wave workgroups
// 2.4 ms on a single line). The host sums the copies.
constexpr uint32_t kQsCopies = 64;
constexpr uint32_t kQsStride = 16;                     // u64 words between copies
constexpr uint32_t kQsWords = kQsCopies * kQsStride;

constexpr uint32_t kListSmall = 512;     // candidate locations per record, fast path
constexpr uint32_t kListLarge = 16384;   // large-list pass (one wave per workgroup)
static_assert(kListLarge < 0x10000, "top-m keys pack a distinct-location index in 16 bits");
constexpr uint32_t kMaxTopM = 8;

// Condensed layout (Sec. 4.2, Sec. 5.1): per feature one 16-byte index entry
// {feature, count, a, b} in buckets of kCondEntries entries (one 128-byte
// line), count 0 = empty; a feature with at most two locations holds them in
// a and b, one with more holds the 64-bit offset a | b << 32 of its run of
// locations (ascending) in the value array. The home bucket of a feature is
// home_bucket(feature, index buckets); entries of a bucket fill in order, a
// feature lies between its home bucket and the first bucket that is not full.
constexpr uint32_t kCondEntries = 8;
constexpr uint32_t kCondInline = 2;
constexpr uint32_t kCondSliceShift = 8;   // bucket-table buckets per conversion slice
constexpr uint32_t kCondCap = 8192;       // entries homed in one slice (held in LDS)

struct CondArgs {
    const unsigned long long* table;   // bucket table
    uint64_t nb;
    uint32_t n_slices;
    uint64_t nbc;                      // index buckets
    uint32_t* slice_feats;             // count pass: distinct features per slice
    unsigned long long* slice_vals;    // count pass: run values per slice; then their
                                       // exclusive prefix (n_slices + 1)
    unsigned int* idx;                 // nbc * kCondEntries * 4 u32
    uint32_t* fill;                    // entries claimed per index bucket
    uint32_t* val;                     // run values
    uint32_t* err;                     // [0]: a slice over kCondCap entries, [1]: no free entry
};

// Launchers (return hipError_t of the launch).
// Build pipeline: sketch (pairs + partition histogram, or the sketch export),
// partition scan + scatter, insert.
hipError_t launch_sketch(const BuildArgs& a, bool pairs, hipStream_t st);
hipError_t launch_partition(const BuildArgs& a, uint64_t n_slots, hipStream_t st);
hipError_t launch_insert(const BuildArgs& a, uint64_t max_items, hipStream_t st);
bool slice_mode_fits(uint32_t slice_shift);
hipError_t launch_cap_finalize(unsigned long long* table, uint64_t nb, uint32_t cap,
                               const uint32_t* cand, uint64_t n_cand, hipStream_t st);
hipError_t launch_cap_scan(unsigned long long* table, uint64_t nb, uint32_t cap,
                           uint32_t cap_dist, hipStream_t st);
hipError_t launch_rehash(const unsigned long long* old_table, uint64_t old_nb,
                         unsigned long long* table, uint32_t* bcount, uint64_t nb,
                         unsigned long long* counters, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v,
                           hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
hipError_t launch_dump(const unsigned long long* table, uint64_t nb, uint32_t lo, uint32_t hi,
                       unsigned long long* out, uint64_t cap, unsigned long long* count,
                       hipStream_t st);
// Table census into count[0..3): live entries, tombstones, distinct features
// of the live entries.
hipError_t launch_census(const unsigned long long* table, uint64_t nb,
                         unsigned long long* count, hipStream_t st);
// Every live entry whose target is first_target or later becomes a tombstone.
hipError_t launch_rollback(unsigned long long* table, uint64_t nb, uint32_t first_target,
                           hipStream_t st);
// Launch shape of the fast classification path: candidate locations held in
// LDS per record (256, 512 or 1024), waves per workgroup (2, 4 or 8) and the
// largest grid (records beyond it are taken grid-stride).
struct ClassifyConfig {
    uint32_t list_cap = kListSmall;
    uint32_t waves_per_block = 4;
    uint32_t max_blocks = 16384;
};
bool classify_config_valid(const ClassifyConfig& c);

// Fast path (one wave per record, small LDS list) and the large-list pass
// over the records the fast path queued.
hipError_t launch_classify_fast(const QueryArgs& a, const ClassifyConfig& c, hipStream_t st);
// groups: workgroups of the large-list pass (0: sized by the launch's records).
hipError_t launch_classify_large(const QueryArgs& a, hipStream_t st, uint32_t groups);
// Routing: the records' size classes into route_queue / route_meta, then one
// fast-path launch per class with that class's shape.
hipError_t launch_route(const QueryArgs& a, const RouteConfig& r, hipStream_t st);
hipError_t launch_classify_class(const QueryArgs& a, const ClassifyConfig& c, uint32_t cls,
                                 hipStream_t st);
hipError_t launch_classify_huge(const QueryArgs& a, hipStream_t st);
// Condensed layout build: the count pass (per slice), the prefix of the run
// values, and the write pass (runs and index entries).
hipError_t launch_condense_count(const CondArgs& c, hipStream_t st);
hipError_t launch_condense_scan(const CondArgs& c, unsigned long long* total_feats,
                                hipStream_t st);
hipError_t launch_condense_write(const CondArgs& c, hipStream_t st);
// Sum of the condensed entries' location counts into *total (which the caller zeroes).
hipError_t launch_condense_pairs(const unsigned int* idx, uint64_t nbc, unsigned long long* total,
                                 hipStream_t st);
hipError_t launch_condense_dump(const unsigned int* idx, uint64_t nbc, const uint32_t* val,
                                uint32_t lo, uint32_t hi, unsigned long long* out, uint64_t cap,
                                unsigned long long* count, hipStream_t st);

// Device of a database handle (for threads that must select it).
int db_device(const struct ::mc_db* db);

// The query workspace of stream `st` made ready now for classifications of up
// to n_records records (a server creates its slots' workspaces up front, so
// that no batch pays for their allocation), and its release once the stream
// is retired (the stream is synchronised first). Callers serialise calls on
// one handle.
int prepare_workspace(struct ::mc_db* db, hipStream_t st, uint64_t n_records);
int release_workspace(struct ::mc_db* db, hipStream_t st);

// Device scratch of one classification supplied by the caller: counters
// (kNumQueryCounters u32), routing data (kRouteMetaWords u32), record queues
// (3 * queue_cap u32) and huge_groups regions of the HBM-list pass.
struct ScratchView {
    uint32_t* counters;
    uint32_t* route_meta;
    uint32_t* queue;
    uint64_t queue_cap;
    unsigned char* huge;
    uint32_t huge_groups;
};
// A classification (as mc_classify_ex) that takes every device buffer beyond
// its inputs and outputs from `scratch` and allocates nothing: the scratch is
// cleared where it must start at zero (fill kernels on `st`), no statistics
// are kept and the too-long count stays in scratch.counters[kQTooLong].
// n_records must not exceed scratch.queue_cap.
int classify_into(struct ::mc_db* db, const char* reads, const uint64_t* offsets,
                  uint32_t n_records, const struct mc_query_opts* opts, uint32_t* out_labels,
                  struct mc_tophit* out_top, const ScratchView& scratch, hipStream_t st);

// Classification of the records [r0, r1) of a served batch (offsets: the
// batch's offsets array) in three phases, each queued on st: phase 0 clears
// `counters` (kNumQueryCounters u32 of device memory owned by the caller) and
// queues the fast pass; phase 1 the large-list pass over the n_queued records
// the fast pass passed on (counters[kQOverflow]); phase 2 the HBM-list pass
// over those the large-list pass passed on (counters[kQHuge]). The caller
// reads the counters back and queues phases 1 and 2 only when they hold
// records: a large-list workgroup needs a CU of its own, which a busy device
// frees only when its other kernels drain. The records' queue ids sit at
// 2 r0 .. 2 r1 of st's workspace queue, which prepare_workspace must have
// sized for r1 records.
int served_classify(struct ::mc_db* db, int phase, const char* reads, const uint64_t* offsets,
                    uint32_t r0, uint32_t r1, const struct mc_query_opts& opts,
                    uint32_t* out_labels, struct mc_tophit* out_top, uint32_t* counters,
                    uint32_t n_queued, hipStream_t st);

// Set the calling thread's mc_last_error text; returns code.
int set_error(int code, const char* msg);

}  // namespace mc
