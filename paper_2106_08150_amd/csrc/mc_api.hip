// Host side of the C ABI declared in include/mc.h: argument checks, the db
// handle (device table, targets, taxonomy, per-stream workspaces), table
// sizing and growth, and the launch sequence of every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mc.h"
#include "mc_internal.hpp"

using namespace mc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? MC_ERR_OOM : MC_ERR_HIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

constexpr double kDefaultLoad = 0.5;
// Pair slots of one build chunk (16 bytes each: the pairs and their
// partitioned copy): about 60% of the device memory free at the add, within
// [kMinChunkSlots, kMaxChunkSlots], so that a reference set that fits builds
// in one pass over the table's slices. Build scratch larger than
// kKeepScratchBytes is released when the add returns.
constexpr uint64_t kMinChunkSlots = 1ull << 26;
constexpr uint64_t kKeepScratchBytes = 512ull << 20;   // build scratch kept after an add
constexpr uint64_t kMaxChunkSlots = 1ull << 32;
constexpr uint64_t kPartBytes = 256ull << 20;           // target table bytes per partition
constexpr uint64_t kMinBuckets = 64;
constexpr uint64_t kCandCapMax = 1ull << 24;

// Launch plan of the fast path: size classes and one shape per class (one
// class: every record in one launch with shape[0]).
struct LaunchPlan {
    RouteConfig route;
    ClassifyConfig shape[kMaxRoutes];
};

struct Workspace {
    uint32_t* queue = nullptr;               // 3 * queue_cap record ids: large-list pass,
                                             // HBM-list pass, size classes
    uint32_t* route_meta = nullptr;          // kRouteMetaWords
    uint64_t queue_cap = 0;                  // records
    uint32_t* counters = nullptr;            // kNumQueryCounters
    unsigned long long* qstats = nullptr;    // kQsWords
    unsigned char* huge = nullptr;           // kHugeBytes (HBM-list pass)
    uint32_t huge_groups = 0;                // regions in huge (0 = kHugeGroups)
};



// Event pairs bracketing profiled launches.
struct Timed {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct mc_db {
    int device = 0;
    uint32_t k = 16, w = 128, s = 16, cap = 254, S = 113;
    uint32_t cap_dist = 15;
    double load = kDefaultLoad;
    // table
    unsigned long long* table = nullptr;
    uint32_t* bcount = nullptr;       // fill counter per bucket
    uint64_t nb = 0;
    uint64_t slots_used = 0;          // occupied slots (stored + tombstones) since the last rehash
    bool touched = false;             // an insert ran on this table (it may hold entries)
    bool fill_pending = false;        // table and counters not yet cleared (left to the insert)
    unsigned long long* counters = nullptr;   // kNumBuildCounters
    uint32_t* cand = nullptr;
    uint64_t cand_cap = 0;
    // targets
    std::vector<uint32_t> taxa;
    uint32_t* d_taxa = nullptr;
    uint64_t d_taxa_cap = 0;
    uint64_t n_windows = 0;
    // taxonomy
    std::vector<uint32_t> parents;
    uint32_t* d_parents = nullptr;
    uint32_t* d_depth = nullptr;
    // stats
    mc_db_stats st{};
    // per-stream query workspaces
    std::map<hipStream_t, Workspace> ws;
    // queues a stream's workspace outgrew: work still queued may use them, and
    // freeing them now would wait for the whole device (every stream), so they
    // are freed with the handle
    std::vector<uint32_t*> retired;
    // build scratch (grow-only): per-window pairs, partitioned pairs, partition data
    unsigned long long* pairs = nullptr;
    unsigned long long* parted = nullptr;
    uint64_t pairs_cap = 0;
    uint32_t* hist = nullptr;
    unsigned long long* part_start = nullptr;
    unsigned long long* cursor = nullptr;
    uint32_t* hist2 = nullptr;                  // slice-mode insert: kMaxSlices
    unsigned long long* slice_start = nullptr;  // kMaxSlices + 1
    unsigned long long* cursor2 = nullptr;      // kMaxSlices
    unsigned long long* chunk_first = nullptr;  // kChunkFirstLen
    // insert path forced by mc_db_set_insert_path (tests); zero = automatic
    mc_insert_path ipath{};
    // condensed layout (mc_db_condense): classifications use it while it is set
    unsigned int* cidx = nullptr;      // nbc buckets of kCondEntries 16-byte entries
    uint64_t nbc = 0;
    uint32_t* cval = nullptr;          // runs of locations
    uint64_t cval_n = 0;
    uint64_t c_features = 0, c_pairs = 0;
    bool table_released = false;       // only the condensed layout is left
    // fast-path launch plan (mc_db_set_launch_config / mc_db_set_routing /
    // mc_db_autotune)
    LaunchPlan plan;
    // bumped whenever device arrays a captured graph refers to may have moved
    uint64_t version = 1;
    // profiling: one timer per profiled kernel kind (MC_K_*)
    bool profiling = false;
    Timed timers[MC_K_COUNT];
};

namespace {

uint64_t num_windows(uint64_t len, uint32_t k, uint32_t S) {
    if (len < k) return 0;
    return (len - k + 1 + S - 1) / S;
}

// Device blocks can be kept for reuse after they are released: hipMalloc and
// hipFree of tens of GB cost hundreds of milliseconds to seconds once the
// runtime stops deferring them (about 28 ms per GB to free and 4 ms per GB to
// map), far more than the build that uses them, so a process that rebuilds
// databases would pay that on every build; a new handle's query workspace
// (record queues and HBM-list scratch, a few hundred MB) took about 0.4 ms
// to map on its first classification. Keeping is opt-in
// (mc_set_cached_memory_limit): a released block of at least kCacheMinBytes
// stays mapped (idle) while the idle blocks of its device stay within the
// limit; otherwise it is freed at once. An allocation takes an idle block of
// its device whose size is within 25% above the request. An allocation that
// fails releases every idle block of the device and tries once more.
// mc_release_cached_memory() gives all idle blocks back.
constexpr size_t kCacheMinBytes = size_t(1) << 20;

struct BlockCache {
    std::mutex mu;
    std::unordered_map<void*, std::pair<int, size_t>> live;   // block -> (device, bytes)
    std::multimap<std::pair<int, size_t>, void*> idle;        // (device, bytes) -> block
    std::map<int, size_t> idle_bytes;
    uint64_t limit = 0;                                       // idle bytes kept per device
};

BlockCache& block_cache() {
    static BlockCache* c = new BlockCache;   // never destroyed: blocks outlive static teardown
    return *c;
}

// Frees the idle blocks of `device` (every device if device < 0) and returns
// the first error; the caller holds the cache lock.
hipError_t release_idle(BlockCache& c, int device) {
    hipError_t err = hipSuccess;
    for (auto it = c.idle.begin(); it != c.idle.end();) {
        if (device >= 0 && it->first.first != device) { ++it; continue; }
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != it->first.first) (void)hipSetDevice(it->first.first);
        const hipError_t e = hipFree(it->second);
        if (err == hipSuccess) err = e;
        if (cur != it->first.first) (void)hipSetDevice(cur);
        c.idle_bytes[it->first.first] -= it->first.second;
        it = c.idle.erase(it);
    }
    return err;
}

int block_alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes < kCacheMinBytes) {
        HIP_TRY(hipMalloc(p, bytes));
        return MC_OK;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.idle.lower_bound({dev, bytes});
    if (it != c.idle.end() && it->first.first == dev && it->first.second <= bytes + bytes / 4) {
        *p = it->second;
        c.live[*p] = it->first;
        c.idle_bytes[dev] -= it->first.second;
        c.idle.erase(it);
        return MC_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)release_idle(c, dev);
        HIP_TRY(hipMalloc(p, bytes));
    }
    c.live[*p] = {dev, bytes};
    return MC_OK;
}

// Bytes of the idle blocks of the current device (memory the next
// allocations can take although the runtime counts it as used).
uint64_t idle_cached_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.idle_bytes.find(dev);
    return it == c.idle_bytes.end() ? 0 : it->second;
}

template <typename T>
int dev_alloc(T** p, uint64_t n) {
    if (n == 0) n = 1;
    void* v = nullptr;
    const int rc = block_alloc(&v, n * sizeof(T));
    *p = static_cast<T*>(v);
    return rc;
}

// Release a block from dev_alloc (any other device pointer is freed). A block
// kept for reuse is parked only after the device has finished the work queued
// so far, so no queued work still uses it when it is handed out again
// (hipFree waits the same way).
hipError_t dev_free(void* p) {
    if (!p) return hipSuccess;
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return hipFree(p);
    const std::pair<int, size_t> key = it->second;
    c.live.erase(it);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != key.first) (void)hipSetDevice(key.first);
    hipError_t e = hipSuccess;
    if (c.idle_bytes[key.first] + key.second <= c.limit) {
        e = hipDeviceSynchronize();
        if (e == hipSuccess) {
            c.idle.insert({key, p});
            c.idle_bytes[key.first] += key.second;
        }
    } else {
        e = hipFree(p);
    }
    if (cur != key.first) (void)hipSetDevice(cur);
    return e;
}

// Make room for `extra` more occupied slots at the handle's load factor,
// re-inserting the current entries into a larger table when needed.
// Clear a table whose clearing was left to the insert (empty slots, zero counters).
int materialize(mc_db* db, hipStream_t st) {
    if (!db->fill_pending) return MC_OK;
    HIP_TRY(launch_fill_u64(db->table, db->nb * kSlots, ~0ull, st));
    HIP_TRY(launch_fill_u32(db->bcount, db->nb, 0u, st));
    db->fill_pending = false;
    return MC_OK;
}

// Grow the table for `extra` more slots at the load factor. A table that an
// insert has touched is rehashed into the new one; an untouched one is simply
// replaced, and with defer_fill the new table is left uncleared for the next
// slice-mode insert to write whole (materialize() clears it otherwise).
int ensure_capacity(mc_db* db, uint64_t extra, hipStream_t st, bool defer_fill = false) {
    const double slots_per_bucket = (double)kSlots;
    uint64_t need = db->slots_used + extra;
    if (db->table && (double)need <= db->load * slots_per_bucket * (double)db->nb) return MC_OK;
    uint64_t nb = (uint64_t)std::ceil((double)need / (db->load * slots_per_bucket));
    if (db->table) nb = std::max<uint64_t>(nb, db->nb + db->nb / 2);   // grow by >= 1.5x
    nb = std::max<uint64_t>(nb, kMinBuckets);
    // bucket indices are 32-bit in the query kernels (2^32 buckets = 512 GiB)
    if (nb > 0xFFFFFFFFull)
        return fail(MC_ERR_OOM, "table of %llu buckets exceeds 2^32 - 1", (unsigned long long)nb);
    unsigned long long* t = nullptr;
    uint32_t* cnt = nullptr;
    int rc = dev_alloc(&t, nb * kSlots);
    if (rc) return rc;
    rc = dev_alloc(&cnt, nb);
    if (rc) { (void)dev_free(t); return rc; }
    const bool grow = db->table != nullptr;
    if (grow && db->touched) {
        HIP_TRY(launch_fill_u64(t, nb * kSlots, ~0ull, st));
        HIP_TRY(launch_fill_u32(cnt, nb, 0u, st));
        HIP_TRY(launch_fill_u64(db->counters, kNumBuildCounters, 0ull, st));
        HIP_TRY(launch_rehash(db->table, db->nb, t, cnt, nb, db->counters, st));
        unsigned long long c[kNumBuildCounters];
        HIP_TRY(hipMemcpyAsync(c, db->counters, sizeof c, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (c[kCntFull]) {
            (void)dev_free(t);
            (void)dev_free(cnt);
            return fail(MC_ERR_TABLE_FULL, "rehash found no free slot for %llu entries",
                        (unsigned long long)c[kCntFull]);
        }
        db->slots_used = c[kCntMoved];
        db->touched = c[kCntMoved] != 0;
        db->fill_pending = false;
    } else {
        db->slots_used = 0;
        db->touched = false;
        db->fill_pending = defer_fill;
        if (!defer_fill) {
            HIP_TRY(launch_fill_u64(t, nb * kSlots, ~0ull, st));
            HIP_TRY(launch_fill_u32(cnt, nb, 0u, st));
        }
    }
    if (grow) {
        HIP_TRY(dev_free(db->table));
        HIP_TRY(dev_free(db->bcount));
        db->st.n_rehash += 1;
    }
    db->bcount = cnt;
    db->table = t;
    db->nb = nb;
    db->version += 1;
    return MC_OK;
}

int upload_taxa(mc_db* db, hipStream_t st) {
    uint64_t n = db->taxa.size();
    if (n > db->d_taxa_cap) {
        uint32_t* p = nullptr;
        uint64_t c = std::max<uint64_t>(n, db->d_taxa_cap * 2);
        int rc = dev_alloc(&p, c);
        if (rc) return rc;
        if (db->d_taxa) HIP_TRY(dev_free(db->d_taxa));
        db->d_taxa = p;
        db->d_taxa_cap = c;
        db->version += 1;
    }
    if (n) HIP_TRY(hipMemcpyAsync(db->d_taxa, db->taxa.data(), n * 4, hipMemcpyHostToDevice, st));
    return MC_OK;
}

// Record an event pair around `launch` when profiling is on.
template <typename F>
hipError_t timed_launch(mc_db* db, Timed& t, hipStream_t st, F launch) {
    if (!db->profiling) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) {
        t.ev.emplace_back(a, b);
    } else {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    return e;
}

hipError_t drain(Timed& t, double* ms, uint64_t* n) {
    double total = 0.0;
    hipError_t err = hipSuccess;
    for (auto& p : t.ev) {
        float x = 0.f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&x, p.first, p.second);
        if (e != hipSuccess) err = e;
        total += x;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (ms) *ms = total;
    if (n) *n = t.ev.size();
    t.ev.clear();
    return err;
}

int ensure_scratch(mc_db* db, uint64_t slots) {
    if (!db->hist) {
        int rc = dev_alloc(&db->hist, kScatGroups * kMaxParts);
        if (!rc) rc = dev_alloc(&db->part_start, kMaxParts + 1);
        if (!rc) rc = dev_alloc(&db->cursor, kScatGroups * kMaxParts);
        if (!rc) rc = dev_alloc(&db->hist2, kMaxSlices);
        if (!rc) rc = dev_alloc(&db->slice_start, kMaxSlices + 1);
        if (!rc) rc = dev_alloc(&db->cursor2, kMaxSlices);
        if (!rc) rc = dev_alloc(&db->chunk_first, kChunkFirstLen);
        if (rc) return rc;
    }
    if (slots <= db->pairs_cap) return MC_OK;
    (void)dev_free(db->pairs);
    (void)dev_free(db->parted);
    db->pairs = db->parted = nullptr;
    db->pairs_cap = 0;
    int rc = dev_alloc(&db->pairs, slots);
    if (!rc) rc = dev_alloc(&db->parted, slots);
    if (rc) return rc;
    db->pairs_cap = slots;
    return MC_OK;
}

uint32_t ceil_log2(uint64_t x) {
    uint32_t b = 0;
    while (b < 63 && (1ull << b) < x) ++b;
    return b;
}

// Partitioning of the insert pass. Slice mode (the default): slices of
// 2^slice_shift buckets (at most kMaxSlices = 2^18 slices), 2^fine_bits
// slices per partition (at most 1024), at most 256 partitions. Otherwise
// (tables too large for that, or the global insert forced by
// mc_db_set_insert_path) partitions of about kPartBytes of table each with
// global counters.
void plan_partitions(const mc_db* db, BuildArgs& a) {
    const uint64_t nb = db->nb;
    const uint32_t lg = ceil_log2(nb);
    // slices of 2^11 buckets (about 16K pairs at load 0.5) from 2^27 buckets up,
    // 2^10 below; larger only past 2^29 buckets (256 x 1024 slices)
    uint32_t sb = std::max<uint32_t>(kMinSliceShift, std::min<uint32_t>(11, lg > 16 ? lg - 16 : 0));
    sb = std::max<uint32_t>(sb, lg > 8 + kMaxFineBits ? lg - 8 - kMaxFineBits : 0);
    // forced by mc_db_set_insert_path (tests): a slice size, the slice bits
    // taken by level 2, the global-counter insert and its partition size
    const mc_insert_path& ip = db->ipath;
    if (ip.slice_shift >= 4 && ip.slice_shift <= kMaxSliceShift) sb = ip.slice_shift;
    if (!ip.global_insert && slice_mode_fits(sb) && lg <= sb + 8 + kMaxFineBits) {
        const uint32_t ns_bits = lg > sb ? lg - sb : 0;       // slices: 2^ns_bits >= nb >> sb
        uint32_t fb = ns_bits > 8 ? ns_bits - 8 : 0;
        if (ip.fine_bits >= fb && ip.fine_bits <= std::min<uint32_t>(ns_bits, kMaxFineBits))
            fb = ip.fine_bits;
        a.slice_mode = 1;
        a.slice_shift = sb;
        a.fine_bits = fb;
        a.part_shift = sb + fb;
    } else {
        uint64_t part = kPartBytes;
        if (ip.part_mb > 0) part = (uint64_t)ip.part_mb << 20;
        const uint64_t per = std::max<uint64_t>(1, part / (kSlots * 8));   // buckets
        uint32_t sh = ceil_log2(per);
        while (((nb - 1) >> sh) + 1 > kMaxParts) ++sh;
        a.slice_mode = 0;
        a.slice_shift = a.fine_bits = 0;
        a.part_shift = sh;
    }
    a.n_parts = (uint32_t)(((nb - 1) >> a.part_shift) + 1);
}

// Host copies of the chunks' descriptors, kept until the call's stream work is
// done (the uploads read them asynchronously).
struct ChunkHost {
    std::vector<std::vector<TargetDesc>> td;
    std::vector<std::vector<uint64_t>> tile_first;
};

// Build pipeline over targets [t0, t1) of the call (one chunk). d_td holds
// t1 - t0 descriptors and d_tf the tile and chunk bounds (device buffers of
// the call, sized for its largest chunk).
int build_chunk(mc_db* db, const uint8_t* genomes, const std::vector<TargetDesc>& all,
                uint32_t t0, uint32_t t1, TargetDesc* d_td, uint64_t* d_tf,
                ChunkHost& keep, hipStream_t st) {
    const uint32_t n = t1 - t0;
    keep.td.emplace_back(all.begin() + t0, all.begin() + t1);
    keep.tile_first.emplace_back(n + 1, 0);
    std::vector<TargetDesc>& td = keep.td.back();
    std::vector<uint64_t>& tile_first = keep.tile_first.back();
    const uint64_t off0 = td[0].off, win0 = td[0].win_base;
    for (uint32_t i = 0; i < n; ++i) {
        td[i].off -= off0;
        td[i].win_base -= win0;
        tile_first[i + 1] = tile_first[i] + (td[i].nw + kTileWindows - 1) / kTileWindows;
    }
    const uint64_t wins = td[n - 1].win_base + td[n - 1].nw;
    const uint64_t slots = wins * db->s;
    if (slots == 0) return MC_OK;
    int rc = ensure_scratch(db, slots);
    if (rc) return rc;
    // d_tf: tile_first (n + 1), then the first slot of each level-1 scatter
    // chunk and the end of the slots (written by the sketch kernel)
    const uint32_t chunk_tiles = scatter_chunk_tiles(db->s);
    HIP_TRY(hipMemcpyAsync(d_td, td.data(), n * sizeof(TargetDesc), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_tf, tile_first.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_fill_u32(db->hist, kScatGroups * kMaxParts, 0u, st));

    BuildArgs a{};
    a.text = genomes + off0;
    a.text_len = td[n - 1].off + td[n - 1].len;
    a.targets = d_td;
    a.n_targets = n;
    a.tile_first = d_tf;
    a.n_tiles = tile_first[n];
    a.k = db->k; a.w = db->w; a.S = db->S; a.s = db->s;
    a.chunk_tiles = chunk_tiles;
    a.chunk_slot = d_tf + n + 1;
    a.table = db->table;
    a.bcount = db->bcount;
    a.nb = db->nb;
    a.cap_dist = db->cap_dist;
    a.cand = db->cand;
    a.cand_cap = db->cand_cap;
    a.counters = db->counters;
    a.pairs = db->pairs;
    a.parted = db->parted;
    plan_partitions(db, a);
    if (!a.slice_mode) {
        rc = materialize(db, st);
        if (rc) return rc;
    }
    a.fresh = db->fill_pending ? 1u : 0u;   // the slice insert writes every bucket
    a.hist = db->hist;
    a.part_start = db->part_start;
    a.cursor = db->cursor;
    a.hist2 = db->hist2;
    a.slice_start = db->slice_start;
    a.cursor2 = db->cursor2;
    a.chunk_first = db->chunk_first;
    a.stage_entries = db->ipath.stage_entries;
    a.force_direct = db->ipath.direct;
    if (a.slice_mode) {
        HIP_TRY(launch_fill_u32(db->hist2, (uint64_t)a.n_parts << a.fine_bits, 0u, st));
        HIP_TRY(launch_fill_u64(db->counters + kCntDefer, 1, 0ull, st));
    }
    HIP_TRY(timed_launch(db, db->timers[MC_K_SKETCH], st, [&] { return launch_sketch(a, true, st); }));
    HIP_TRY(timed_launch(db, db->timers[MC_K_SCATTER], st,
                         [&] { return launch_partition(a, slots, st); }));
    HIP_TRY(timed_launch(db, db->timers[MC_K_INSERT], st, [&] { return launch_insert(a, slots, st); }));
    db->fill_pending = false;
    db->touched = true;
    return MC_OK;
}

// Forget the condensed layout (after the bucket table changed).
void drop_condensed(mc_db* db) {
    if (!db->cidx) return;
    (void)dev_free(db->cidx);
    (void)dev_free(db->cval);
    db->cidx = nullptr;
    db->cval = nullptr;
    db->nbc = db->cval_n = db->c_features = db->c_pairs = 0;
    db->version += 1;
}

// Shared by the host and device entry points: genomes is a device pointer.
int add_targets_dev(mc_db* db, const uint8_t* genomes, const uint64_t* lengths,
                    const uint32_t* taxa, uint32_t n, hipStream_t st) {
    if (db->table_released)
        return fail(MC_ERR_STATE, "the bucket table was released by mc_db_condense: no additions");
    if (n == 0) return MC_OK;
    if ((uint64_t)db->taxa.size() + n > MC_MAX_TARGETS)
        return fail(MC_ERR_CAPACITY, "at most %u targets (have %zu, adding %u)", MC_MAX_TARGETS,
                    db->taxa.size(), n);
    std::vector<TargetDesc> td(n);
    uint64_t off = 0, wins = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t nw = num_windows(lengths[i], db->k, db->S);
        if (nw > MC_MAX_WINDOWS)
            return fail(MC_ERR_CAPACITY, "sequence %u has %llu windows (max %u)", i,
                        (unsigned long long)nw, MC_MAX_WINDOWS);
        td[i] = TargetDesc{off, lengths[i], wins, (uint32_t)db->taxa.size() + i, (uint32_t)nw};
        off += lengths[i];
        wins += nw;
    }
    const uint64_t upper = wins * db->s;
    // classifications queued earlier on any stream may still read the table
    // (and a graph replay its arrays): they finish before the table changes
    HIP_TRY(hipDeviceSynchronize());
    drop_condensed(db);   // classifications use the bucket table from here on
    const uint32_t first_target = (uint32_t)db->taxa.size();
    int rc = MC_OK;
    uint64_t cand_need = std::min<uint64_t>(std::max<uint64_t>(upper, 1), kCandCapMax);
    if (cand_need > db->cand_cap) {
        if (db->cand) HIP_TRY(dev_free(db->cand));
        db->cand = nullptr;
        db->cand_cap = 0;
        rc = dev_alloc(&db->cand, cand_need);
        if (rc) return rc;
        db->cand_cap = cand_need;
    }
    rc = ensure_capacity(db, upper, st, true);
    if (rc) return rc;
    auto insert_all = [&]() -> int {
        HIP_TRY(launch_fill_u64(db->counters, kNumBuildCounters, 0ull, st));
        // chunks of whole targets with at most max_chunk pair slots
        uint64_t max_chunk = kMinChunkSlots;
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
            // held scratch and idle cached blocks are reused
            const uint64_t avail = (uint64_t)free_b + db->pairs_cap * 16 + idle_cached_bytes();
            max_chunk = std::min(kMaxChunkSlots, std::max(kMinChunkSlots, avail / 16 / 10 * 6));
        }
        if (db->ipath.chunk_slots) max_chunk = db->ipath.chunk_slots;   // forced (tests)
        std::vector<uint32_t> cuts{0};
        uint64_t most = 0;
        for (uint32_t t0 = 0; t0 < n;) {
            uint32_t t1 = t0;
            uint64_t slots = 0;
            while (t1 < n &&
                   (t1 == t0 || slots + (uint64_t)td[t1].nw * db->s <= max_chunk)) {
                slots += (uint64_t)td[t1].nw * db->s;
                ++t1;
            }
            cuts.push_back(t1);
            most = std::max(most, slots);
            t0 = t1;
        }
        // every buffer the chunks use is allocated before the first insert: an
        // allocation failure then leaves the table as it was
        if (most == 0) return MC_OK;
        if (int r = ensure_scratch(db, most)) return r;
        uint64_t tiles = 0;
        for (uint32_t i = 0; i < n; ++i) tiles += (td[i].nw + kTileWindows - 1) / kTileWindows;
        TargetDesc* d_td = nullptr;
        uint64_t* d_tf = nullptr;
        if (int r = dev_alloc(&d_td, n)) return r;
        // n + 1 tile bounds, at most tiles + 1 chunk bounds and the end, for any chunk
        if (int r = dev_alloc(&d_tf, (uint64_t)n + tiles + 3)) { (void)dev_free(d_td); return r; }
        ChunkHost keep;
        keep.td.reserve(cuts.size());
        keep.tile_first.reserve(cuts.size());
        int r = MC_OK;
        for (size_t c = 0; c + 1 < cuts.size() && r == MC_OK; ++c)
            r = build_chunk(db, genomes, td, cuts[c], cuts[c + 1], d_td, d_tf, keep, st);
        // hipFree waits for the stream work that reads d_td, d_tf and keep
        const hipError_t e1 = dev_free(d_td), e2 = dev_free(d_tf);
        if (r == MC_OK && (e1 != hipSuccess || e2 != hipSuccess))
            r = fail(MC_ERR_HIP, "hipFree: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return r;
    };
    rc = insert_all();
    // a table still uncleared (no insert ran, or one failed first) is cleared now
    const int rc_clear = materialize(db, st);
    if (rc == MC_OK) rc = rc_clear;
    unsigned long long c[kNumBuildCounters] = {};
    if (hipMemcpyAsync(c, db->counters, sizeof c, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        if (rc == MC_OK) rc = fail(MC_ERR_HIP, "build counters could not be read");
    }
    if (rc == MC_OK && c[kCntFull])
        rc = fail(MC_ERR_TABLE_FULL, "%llu inserts found no free slot",
                  (unsigned long long)c[kCntFull]);
    if (rc == MC_OK && db->ipath.fail_after) {   // forced by a test (mc_db_set_insert_path)
        db->ipath.fail_after = 0;
        rc = fail(MC_ERR_TABLE_FULL, "failure forced after %llu inserts",
                  (unsigned long long)c[kCntInserted]);
    }
    if (rc != MC_OK) {
        // nothing of the call stays: every entry of its targets (ids from
        // first_target on) becomes a tombstone; the cap has not run yet, so
        // the earlier targets' entries are as they were
        const std::string msg = g_err;
        if (db->touched) {
            db->slots_used += c[kCntInserted];   // tombstones still occupy their slots
            if (launch_rollback(db->table, db->nb, first_target, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                g_err = msg + "; the rollback of the call's entries failed too: destroy the handle";
            else
                g_err = msg;
        }
        return rc;
    }
    if (c[kCntCand] <= db->cand_cap) {
        HIP_TRY(launch_cap_finalize(db->table, db->nb, db->cap, db->cand, c[kCntCand], st));
    } else {
        HIP_TRY(launch_cap_scan(db->table, db->nb, db->cap, db->cap_dist, st));
    }
    for (uint32_t i = 0; i < n; ++i) db->taxa.push_back(taxa[i]);
    rc = upload_taxa(db, st);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    db->slots_used += c[kCntInserted];
    db->n_windows += wins;
    db->st.n_pairs_inserted += c[kCntInserted];
    db->st.probe_sum += c[kCntProbe];
    db->st.n_cap_candidates += c[kCntCand];
    // build scratch beyond a small amount (enough for additions of a few
    // hundred Mbp) is released: a resident database does not carry dead pairs
    if (db->pairs_cap * 16 > kKeepScratchBytes) {
        HIP_TRY(dev_free(db->pairs));
        HIP_TRY(dev_free(db->parted));
        db->pairs = db->parted = nullptr;
        db->pairs_cap = 0;
    }
    return MC_OK;
}

int check_db(mc_db* db) {
    if (!db) return fail(MC_ERR_INVALID_ARG, "db is NULL");
    return MC_OK;
}

// Device buffers of a workspace that do not depend on the batch size: the
// counters and the HBM-list scratch, whose per-target bests start at zero
// (the pass leaves them at zero).
int init_workspace(Workspace& w, hipStream_t st) {
    if (int rc = dev_alloc(&w.counters, kNumQueryCounters)) return rc;
    if (int rc = dev_alloc(&w.qstats, kQsWords)) return rc;
    if (int rc = dev_alloc(&w.huge, kHugeBytes)) return rc;
    if (int rc = dev_alloc(&w.route_meta, kRouteMetaWords)) return rc;
    HIP_TRY(launch_fill_u32(w.counters, kNumQueryCounters, 0u, st));
    HIP_TRY(launch_fill_u64(w.qstats, kQsWords, 0ull, st));
    for (uint32_t r = 0; r < kHugeGroups; ++r)
        HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(w.huge + r * kHugeRegionBytes),
                                kHugeTargets, 0ull, st));
    return MC_OK;
}

Workspace* workspace(mc_db* db, hipStream_t st, uint64_t n_records, int* rc) {
    Workspace& w = db->ws[st];
    *rc = MC_OK;
    if (!w.huge) {
        if ((*rc = init_workspace(w, st))) return nullptr;
    }
    if (n_records > w.queue_cap) {
        uint32_t* q = nullptr;
        const uint64_t c = std::max<uint64_t>(std::max<uint64_t>(n_records, 1024), 2 * w.queue_cap);
        if ((*rc = dev_alloc(&q, 3 * c))) return nullptr;
        if (w.queue) db->retired.push_back(w.queue);
        w.queue = q;
        w.queue_cap = c;
    }
    return &w;
}

}  // namespace

namespace {

int check_classify(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                   const mc_query_opts* opts, const uint32_t* out_labels) {
    if (int rc = check_db(db)) return rc;
    if (!opts) return fail(MC_ERR_INVALID_ARG, "opts is NULL");
    if (opts->top_m < 1 || opts->top_m > kMaxTopM)
        return fail(MC_ERR_INVALID_ARG, "top_m %u not in [1, %u]", opts->top_m, kMaxTopM);
    if (opts->paired > 1) return fail(MC_ERR_INVALID_ARG, "paired must be 0 or 1");
    if (n_records == 0) return MC_OK;
    if (!reads || !offsets || !out_labels) return fail(MC_ERR_INVALID_ARG, "NULL pointer");
    if (!db->taxa.empty()) {
        if (db->parents.empty()) return fail(MC_ERR_STATE, "taxonomy not set");
        for (size_t t = 0; t < db->taxa.size(); ++t)
            if (db->taxa[t] >= db->parents.size())
                return fail(MC_ERR_STATE, "target %zu has taxon %u outside the taxonomy", t,
                            db->taxa[t]);
    }
    return MC_OK;
}

// Kernel arguments of a classification of n_records records with workspace w.
QueryArgs query_args(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                     const mc_query_opts& opts, uint32_t* out_labels, mc_tophit* out_top,
                     Workspace& w) {
    QueryArgs a{};
    if (db->cidx) {   // condensed layout
        a.table = reinterpret_cast<const unsigned long long*>(db->cidx);
        a.nb = db->nbc;
        a.cval = db->cval;
    } else {
        a.table = db->table;
        a.nb = db->nb;
    }
    a.reads = reinterpret_cast<const uint8_t*>(reads);
    a.offsets = offsets;
    a.n_records = n_records;
    a.paired = opts.paired;
    a.k = db->k; a.w = db->w; a.S = db->S; a.s = db->s;
    a.divS = make_divu32(db->S);
    a.top_m = opts.top_m;
    a.min_hits = opts.min_hits;
    a.hit_diff = opts.hit_diff;
    a.insert_size = opts.insert_size;
    a.target_taxon = db->d_taxa;
    a.parents = db->d_parents;
    a.depth = db->d_depth;
    a.out_labels = out_labels;
    a.out_top = reinterpret_cast<uint32_t*>(out_top);
    a.queue = w.queue;
    a.counters = w.counters;
    a.qstats = w.qstats;
    a.huge = w.huge;
    a.huge_groups = w.huge_groups;
    a.route_queue = w.queue + 2 * w.queue_cap;
    a.route_meta = w.route_meta;
    return a;
}

// The fast pass of a classification: one launch, or the routing launches and
// one launch per size class.
int launch_fast_phase(mc_db* db, const QueryArgs& a, Workspace& w, const LaunchPlan& plan,
                      hipStream_t st, bool profile) {
    auto fast = [&]() -> hipError_t {
        if (plan.route.n <= 1) return launch_classify_fast(a, plan.shape[0], st);
        hipError_t e = launch_fill_u32(w.route_meta, kRouteMetaWords, 0u, st);
        if (e == hipSuccess) e = launch_route(a, plan.route, st);
        for (uint32_t c = 0; c < plan.route.n && e == hipSuccess; ++c)
            e = launch_classify_class(a, plan.shape[c], c, st);
        return e;
    };
    if (profile) {
        HIP_TRY(timed_launch(db, db->timers[MC_K_CLASSIFY], st, fast));
    } else {
        HIP_TRY(fast());
    }
    return MC_OK;
}

// Queue the classification launches on st with workspace w (no allocation, no
// synchronisation: usable under stream capture).
int classify_launch(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                    const mc_query_opts& opts, uint32_t* out_labels, mc_tophit* out_top,
                    Workspace& w, const LaunchPlan& plan, hipStream_t st, bool profile) {
    static_assert(kQOverflow == 0 && kQHuge == 1, "the per-launch queue counters lead");
    HIP_TRY(launch_fill_u32(w.counters, 2, 0u, st));
    const QueryArgs a = query_args(db, reads, offsets, n_records, opts, out_labels, out_top, w);
    if (int rc = launch_fast_phase(db, a, w, plan, st, profile)) return rc;
    HIP_TRY(launch_classify_large(a, st, 0));
    HIP_TRY(launch_classify_huge(a, st));
    return MC_OK;
}

int alloc_workspace(Workspace& w, uint64_t n_records, hipStream_t st) {
    if (int rc = init_workspace(w, st)) return rc;
    w.queue_cap = std::max<uint64_t>(n_records, 1);
    return dev_alloc(&w.queue, 3 * w.queue_cap);
}

void free_workspace(Workspace& w) {
    (void)dev_free(w.queue);
    (void)dev_free(w.counters);
    (void)dev_free(w.qstats);
    (void)dev_free(w.huge);
    (void)dev_free(w.route_meta);
    w = Workspace();
}

}  // namespace

// A classification call captured into a HIP graph with its own workspace.
// It is captured again (transparently) when the database's device arrays
// have changed since the capture.
struct mc_graph {
    mc_db* db = nullptr;
    const char* reads = nullptr;
    const uint64_t* offsets = nullptr;
    uint32_t n = 0;
    mc_query_opts opts{};
    uint32_t* out_labels = nullptr;
    mc_tophit* out_top = nullptr;
    Workspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t version = 0;
};

namespace {

void release_graph(mc_graph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
}

int capture_graph(mc_graph* g, hipStream_t st) {
    mc_db* db = g->db;
    release_graph(g);
    // capture needs a stream other than the legacy default stream
    hipStream_t cs = st;
    bool own = false;
    if (cs == nullptr) {
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        own = true;
    }
    int rc = MC_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = classify_launch(db, g->reads, g->offsets, g->n, g->opts, g->out_labels, g->out_top,
                             g->ws, db->plan, cs, false);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e2 != hipSuccess && rc == MC_OK) rc = fail(MC_ERR_HIP, "graph capture failed");
        g->graph = graph;
        if (rc == MC_OK) {
            e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = fail(MC_ERR_HIP, "graph instantiation failed");
        }
    } else {
        rc = fail(MC_ERR_HIP, "stream capture could not begin");
    }
    if (own) (void)hipStreamDestroy(cs);
    if (rc == MC_OK) g->version = db->version;
    else release_graph(g);
    return rc;
}

}  // namespace

namespace mc {
int db_device(const struct ::mc_db* db) { return db->device; }

int prepare_workspace(struct ::mc_db* db, hipStream_t st, uint64_t n_records) {
    if (int rc = check_db(db)) return rc;
    DeviceGuard dg(db->device);
    int rc = MC_OK;
    (void)workspace(db, st, n_records, &rc);
    return rc;
}

int release_workspace(struct ::mc_db* db, hipStream_t st) {
    if (int rc = check_db(db)) return rc;
    auto it = db->ws.find(st);
    if (it == db->ws.end()) return MC_OK;
    DeviceGuard dg(db->device);
    HIP_TRY(hipStreamSynchronize(st));
    free_workspace(it->second);
    db->ws.erase(it);
    return MC_OK;
}

int classify_into(struct ::mc_db* db, const char* reads, const uint64_t* offsets,
                  uint32_t n_records, const mc_query_opts* opts, uint32_t* out_labels,
                  mc_tophit* out_top, const ScratchView& scratch, hipStream_t st) {
    if (int rc = check_classify(db, reads, offsets, n_records, opts, out_labels)) return rc;
    if (n_records == 0) return MC_OK;
    if (n_records > scratch.queue_cap)
        return fail(MC_ERR_INVALID_ARG, "%u records exceed the scratch's %llu", n_records,
                    (unsigned long long)scratch.queue_cap);
    DeviceGuard dg(db->device);
    Workspace w;
    w.counters = scratch.counters;
    w.route_meta = scratch.route_meta;
    w.queue = scratch.queue;
    w.queue_cap = scratch.queue_cap;
    w.huge = scratch.huge;
    w.huge_groups = scratch.huge_groups;
    // what the passes expect at zero: the counters and the per-target bests
    HIP_TRY(launch_fill_u32(w.counters, kNumQueryCounters, 0u, st));
    for (uint32_t r = 0; r < scratch.huge_groups; ++r)
        HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(w.huge + r * kHugeRegionBytes),
                                kHugeTargets, 0ull, st));
    return classify_launch(db, reads, offsets, n_records, *opts, out_labels, out_top, w, db->plan,
                           st, false);
}
int served_classify(struct ::mc_db* db, int phase, const char* reads, const uint64_t* offsets,
                    uint32_t r0, uint32_t r1, const mc_query_opts& opts, uint32_t* out_labels,
                    mc_tophit* out_top, uint32_t* counters, uint32_t n_queued, hipStream_t st) {
    if (phase == 0) {
        if (int rc = check_classify(db, reads, offsets, r1 - r0, &opts, out_labels)) return rc;
    }
    if (r1 <= r0) return MC_OK;
    DeviceGuard dg(db->device);
    auto it = db->ws.find(st);
    if (it == db->ws.end() || it->second.queue_cap < r1)
        return fail(MC_ERR_STATE, "the stream's workspace holds fewer than %u records", r1);
    Workspace& w = it->second;
    const uint64_t per = opts.paired ? 2 : 1;
    QueryArgs a = query_args(db, reads, offsets + per * r0, r1 - r0, opts, out_labels + r0,
                             out_top ? out_top + (uint64_t)r0 * opts.top_m : nullptr, w);
    a.counters = counters;
    a.queue = w.queue + 2ull * r0;   // ids [0, 2 (r1 - r0)) of the range's records
    if (phase == 0) {
        HIP_TRY(launch_fill_u32(counters, kNumQueryCounters, 0u, st));
        return launch_fast_phase(db, a, w, db->plan, st, db->profiling);
    }
    if (phase == 1) {
        HIP_TRY(launch_classify_large(a, st, n_queued));
        return MC_OK;
    }
    HIP_TRY(launch_classify_huge(a, st));
    return MC_OK;
}

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace mc

extern "C" {

const char* mc_last_error(void) { return g_err.c_str(); }

mc_db* mc_db_create(uint32_t k, uint32_t window, uint32_t sketch_size, uint32_t max_locations) {
    if (k < 1 || k > 16 || window < k || window - k + 1 > 256 || sketch_size < 1 ||
        sketch_size > 64 || sketch_size > window - k + 1 || max_locations < 1 ||
        max_locations > 65535) {
        fail(MC_ERR_INVALID_ARG,
             "invalid parameters k=%u window=%u sketch_size=%u max_locations=%u", k, window,
             sketch_size, max_locations);
        return nullptr;
    }
    mc_db* db = new mc_db();
    if (hipGetDevice(&db->device) != hipSuccess) {
        fail(MC_ERR_HIP, "no HIP device");
        delete db;
        return nullptr;
    }
    db->k = k; db->w = window; db->s = sketch_size; db->cap = max_locations;
    db->S = window - k + 1;
    // a feature with more than `cap` entries spans at least ceil((cap+1)/16)
    // buckets of its chain, so one of its inserts lands this far or farther
    db->cap_dist = (max_locations + 1 + kSlots - 1) / kSlots - 1;
    if (dev_alloc(&db->counters, kNumBuildCounters) || ensure_capacity(db, 0, nullptr) ||
        hipDeviceSynchronize() != hipSuccess) {
        std::string e = g_err;
        mc_db_destroy(db);
        g_err = e.empty() ? "allocation failed" : e;
        return nullptr;
    }
    return db;
}

int mc_set_cached_memory_limit(uint64_t bytes_per_device) {
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    c.limit = bytes_per_device;
    hipError_t err = hipSuccess;
    for (auto& kv : c.idle_bytes) {
        if (kv.second <= bytes_per_device) continue;
        const hipError_t e = release_idle(c, kv.first);
        if (err == hipSuccess) err = e;
    }
    if (err != hipSuccess) return fail(MC_ERR_HIP, "release of cached blocks: %s", hipGetErrorString(err));
    return MC_OK;
}

int mc_db_set_insert_path(mc_db* db, const mc_insert_path* path) {
    if (int rc = check_db(db)) return rc;
    if (!path) {
        db->ipath = mc_insert_path{};
        return MC_OK;
    }
    if (path->slice_shift != 0 && (path->slice_shift < 4 || path->slice_shift > kMaxSliceShift))
        return fail(MC_ERR_INVALID_ARG, "slice_shift %u not in 4..%u", path->slice_shift,
                    kMaxSliceShift);
    db->ipath = *path;
    return MC_OK;
}

int mc_release_cached_memory(void) {
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    const hipError_t e = release_idle(c, -1);
    if (e != hipSuccess) return fail(MC_ERR_HIP, "release of cached blocks: %s", hipGetErrorString(e));
    return MC_OK;
}

int mc_db_destroy(mc_db* db) {
    if (!db) return MC_OK;
    DeviceGuard dg(db->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : db->ws) free_workspace(kv.second);
    for (uint32_t* q : db->retired) (void)dev_free(q);
    for (auto& t : db->timers) (void)drain(t, nullptr, nullptr);
    (void)dev_free(db->cidx);
    (void)dev_free(db->cval);
    (void)dev_free(db->pairs);
    (void)dev_free(db->parted);
    (void)dev_free(db->hist);
    (void)dev_free(db->part_start);
    (void)dev_free(db->cursor);
    (void)dev_free(db->hist2);
    (void)dev_free(db->slice_start);
    (void)dev_free(db->cursor2);
    (void)dev_free(db->chunk_first);
    (void)dev_free(db->table);
    (void)dev_free(db->bcount);
    (void)dev_free(db->counters);
    (void)dev_free(db->cand);
    (void)dev_free(db->d_taxa);
    (void)dev_free(db->d_parents);
    (void)dev_free(db->d_depth);
    delete db;
    return MC_OK;
}

int mc_db_reserve(mc_db* db, uint64_t n_pairs, double load_factor) {
    if (int rc = check_db(db)) return rc;
    if (db->table_released) return fail(MC_ERR_STATE, "the bucket table was released");
    if (load_factor < 0.0 || load_factor > 0.9 || std::isnan(load_factor))
        return fail(MC_ERR_INVALID_ARG, "load_factor %g not in (0, 0.9]", load_factor);
    DeviceGuard dg(db->device);
    if (load_factor > 0.0) db->load = load_factor;
    uint64_t have = db->slots_used;
    uint64_t extra = n_pairs > have ? n_pairs - have : 0;
    int rc = ensure_capacity(db, extra, nullptr);
    if (rc) return rc;
    HIP_TRY(hipDeviceSynchronize());
    return MC_OK;
}

int mc_db_add_targets(mc_db* db, const char* genomes, const uint64_t* lengths,
                      const uint32_t* taxon_ids, uint32_t n) {
    if (int rc = check_db(db)) return rc;
    if (n && (!lengths || !taxon_ids)) return fail(MC_ERR_INVALID_ARG, "NULL array");
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += lengths[i];
    if (total && !genomes) return fail(MC_ERR_INVALID_ARG, "genomes is NULL");
    DeviceGuard dg(db->device);
    uint8_t* d = nullptr;
    int rc = dev_alloc(&d, total + 16);
    if (rc) return rc;
    hipError_t e = total ? hipMemcpy(d, genomes, total, hipMemcpyHostToDevice) : hipSuccess;
    if (e != hipSuccess) {
        (void)dev_free(d);
        return fail(MC_ERR_HIP, "copy of genomes failed: %s", hipGetErrorString(e));
    }
    rc = add_targets_dev(db, d, lengths, taxon_ids, n, nullptr);
    (void)dev_free(d);
    return rc;
}

int mc_db_add_targets_device(mc_db* db, const char* genomes_dev, const uint64_t* lengths,
                             const uint32_t* taxon_ids, uint32_t n, void* stream) {
    if (int rc = check_db(db)) return rc;
    if (n && (!lengths || !taxon_ids)) return fail(MC_ERR_INVALID_ARG, "NULL array");
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += lengths[i];
    if (total && !genomes_dev) return fail(MC_ERR_INVALID_ARG, "genomes_dev is NULL");
    DeviceGuard dg(db->device);
    return add_targets_dev(db, reinterpret_cast<const uint8_t*>(genomes_dev), lengths, taxon_ids,
                           n, static_cast<hipStream_t>(stream));
}

int mc_db_set_taxonomy(mc_db* db, const uint32_t* parents, uint32_t n_nodes) {
    if (int rc = check_db(db)) return rc;
    if (!parents || n_nodes == 0) return fail(MC_ERR_INVALID_ARG, "empty taxonomy");
    uint32_t roots = 0;
    for (uint32_t i = 0; i < n_nodes; ++i) {
        if (parents[i] >= n_nodes)
            return fail(MC_ERR_INVALID_ARG, "parent of node %u out of range", i);
        roots += parents[i] == i;
    }
    if (roots != 1) return fail(MC_ERR_INVALID_ARG, "taxonomy has %u roots (need 1)", roots);
    // depth by walking up with memoisation; a walk longer than n_nodes is a cycle
    std::vector<uint32_t> depth(n_nodes, 0xFFFFFFFFu);
    std::vector<uint32_t> path;
    for (uint32_t i = 0; i < n_nodes; ++i) {
        uint32_t x = i;
        path.clear();
        while (depth[x] == 0xFFFFFFFFu && parents[x] != x) {
            path.push_back(x);
            if (path.size() > n_nodes) return fail(MC_ERR_INVALID_ARG, "taxonomy has a cycle");
            x = parents[x];
        }
        uint32_t d = parents[x] == x && depth[x] == 0xFFFFFFFFu ? 0 : depth[x];
        depth[x] = d;
        for (size_t p = path.size(); p-- > 0;) depth[path[p]] = ++d;
    }
    DeviceGuard dg(db->device);
    uint32_t *dp = nullptr, *dd = nullptr;
    int rc = dev_alloc(&dp, n_nodes);
    if (rc) return rc;
    rc = dev_alloc(&dd, n_nodes);
    if (rc) { (void)dev_free(dp); return rc; }
    hipError_t e1 = hipMemcpy(dp, parents, n_nodes * 4ull, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(dd, depth.data(), n_nodes * 4ull, hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)dev_free(dp);
        (void)dev_free(dd);
        return fail(MC_ERR_HIP, "taxonomy upload failed");
    }
    HIP_TRY(hipDeviceSynchronize());   // no classify may still read the old arrays
    (void)dev_free(db->d_parents);
    (void)dev_free(db->d_depth);
    db->d_parents = dp;
    db->d_depth = dd;
    db->version += 1;
    db->parents.assign(parents, parents + n_nodes);
    return MC_OK;
}

int mc_classify_ex(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                   const mc_query_opts* opts, uint32_t* out_labels, mc_tophit* out_top,
                   void* stream) {
    if (int rc = check_classify(db, reads, offsets, n_records, opts, out_labels)) return rc;
    if (n_records == 0) return MC_OK;
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = 0;
    Workspace* w = workspace(db, st, n_records, &rc);
    if (!w) return rc;
    return classify_launch(db, reads, offsets, n_records, *opts, out_labels, out_top, *w,
                           db->plan, st, db->profiling);
}

int mc_classify(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_reads,
                uint32_t* out_labels, void* stream) {
    mc_query_opts o{4, 4, 0, 0, 0};
    return mc_classify_ex(db, reads, offsets, n_reads, &o, out_labels, nullptr, stream);
}

int mc_db_query_status(mc_db* db, void* stream, uint64_t* n_too_long) {
    if (int rc = check_db(db)) return rc;
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(st));
    uint64_t n = 0;
    auto it = db->ws.find(st);
    if (it != db->ws.end() && it->second.counters) {
        uint32_t c = 0;
        HIP_TRY(hipMemcpy(&c, it->second.counters + kQTooLong, 4, hipMemcpyDeviceToHost));
        HIP_TRY(launch_fill_u32(it->second.counters + kQTooLong, 1, 0u, st));
        HIP_TRY(hipStreamSynchronize(st));
        n = c;
    }
    if (n_too_long) *n_too_long = n;
    if (n) return fail(MC_ERR_LIST, "%llu records had too many candidate locations",
                       (unsigned long long)n);
    return MC_OK;
}

int mc_db_get_stats(mc_db* db, mc_db_stats* out) {
    if (int rc = check_db(db)) return rc;
    if (!out) return fail(MC_ERR_INVALID_ARG, "out is NULL");
    DeviceGuard dg(db->device);
    unsigned long long* cnt = nullptr;
    int rc = dev_alloc(&cnt, 3);
    if (rc) return rc;
    unsigned long long census[3] = {0, 0, 0};   // live, tombstones, distinct features
    hipError_t e = hipSuccess;
    if (db->table_released) {   // the condensed layout's counts
        census[0] = db->c_pairs;
        census[2] = db->c_features;
    } else {
        e = materialize(db, nullptr) == MC_OK ? hipSuccess : hipErrorUnknown;
        if (e == hipSuccess) e = launch_fill_u64(cnt, 3, 0ull, nullptr);
        if (e == hipSuccess) e = launch_census(db->table, db->nb, cnt, nullptr);
        if (e == hipSuccess) e = hipMemcpy(census, cnt, sizeof census, hipMemcpyDeviceToHost);
    }
    (void)dev_free(cnt);
    if (e != hipSuccess) return fail(MC_ERR_HIP, "stats: %s", hipGetErrorString(e));
    *out = db->st;
    for (auto& kv : db->ws) {
        if (!kv.second.qstats) continue;
        std::vector<unsigned long long> q(kQsWords);
        HIP_TRY(hipStreamSynchronize(kv.first));
        HIP_TRY(hipMemcpy(q.data(), kv.second.qstats, kQsWords * 8ull, hipMemcpyDeviceToHost));
        for (uint32_t c = 0; c < kQsCopies; ++c) {
            out->q_features += q[c * kQsStride + kQsFeatures];
            out->q_locations += q[c * kQsStride + kQsLocations];
            out->q_probes += q[c * kQsStride + kQsProbes];
            out->q_large_records += q[c * kQsStride + kQsLarge];
            out->q_hbm_records += q[c * kQsStride + kQsHuge];
        }
    }
    out->n_targets = db->taxa.size();
    out->n_windows = db->n_windows;
    out->n_pairs_stored = census[0];
    out->n_tombstones = census[1];
    out->n_features = census[2];
    out->n_buckets = db->table_released ? 0 : db->nb;
    out->table_bytes = db->table_released ? 0 : db->nb * (kSlots * 8 + 4);
    out->load_factor = db->nb && !db->table_released
                           ? (double)(census[0] + census[1]) / (double)(db->nb * kSlots) : 0.0;
    out->condensed_bytes = db->cidx ? db->nbc * kCondEntries * 16 + db->cval_n * 4 : 0;
    return MC_OK;
}

int mc_db_condense(mc_db* db, int release_table) {
    if (int rc = check_db(db)) return rc;
    if (db->table_released) return fail(MC_ERR_STATE, "the bucket table was released");
    DeviceGuard dg(db->device);
    HIP_TRY(hipDeviceSynchronize());   // classifications in flight read the old layout
    drop_condensed(db);
    if (int rc = materialize(db, nullptr)) return rc;
    CondArgs c{};
    c.table = db->table;
    c.nb = db->nb;
    c.n_slices = (uint32_t)(((db->nb - 1) >> kCondSliceShift) + 1);
    unsigned long long* tf = nullptr;
    int rc = dev_alloc(&c.slice_feats, c.n_slices);
    if (!rc) rc = dev_alloc(&c.slice_vals, (uint64_t)c.n_slices + 1);
    if (!rc) rc = dev_alloc(&c.err, 2);
    if (!rc) rc = dev_alloc(&tf, 1);
    auto release = [&]() {
        (void)dev_free(c.slice_feats);
        (void)dev_free(c.slice_vals);
        (void)dev_free(c.err);
        (void)dev_free(tf);
        (void)dev_free(c.fill);
    };
    if (rc) { release(); return rc; }
    uint32_t err[2] = {0, 0};
    unsigned long long total_feats = 0, total_vals = 0;
    hipError_t e = launch_fill_u32(c.err, 2, 0u, nullptr);
    if (e == hipSuccess) e = launch_condense_count(c, nullptr);
    if (e == hipSuccess) e = launch_condense_scan(c, tf, nullptr);
    if (e == hipSuccess) e = hipMemcpy(err, c.err, sizeof err, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&total_feats, tf, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&total_vals, c.slice_vals + c.n_slices, 8,
                                       hipMemcpyDeviceToHost);
    if (e != hipSuccess) { release(); return fail(MC_ERR_HIP, "condense: %s", hipGetErrorString(e)); }
    if (err[0]) {
        release();
        return fail(MC_ERR_CAPACITY, "a slice of %u buckets holds more than %u entries",
                    1u << kCondSliceShift, kCondCap);
    }
    // index buckets for about four entries of eight each (load 0.5)
    c.nbc = std::max<uint64_t>(kMinBuckets, (total_feats + 3) / 4);
    if (c.nbc > 0xFFFFFFFFull) { release(); return fail(MC_ERR_OOM, "index too large"); }
    rc = dev_alloc(&c.idx, c.nbc * kCondEntries * 4);
    if (!rc) rc = dev_alloc(&c.fill, c.nbc);
    if (!rc) rc = dev_alloc(&c.val, std::max<uint64_t>(total_vals, 1));
    if (rc) {
        (void)dev_free(c.idx);
        (void)dev_free(c.val);
        release();
        return rc;
    }
    e = launch_fill_u64(reinterpret_cast<unsigned long long*>(c.idx), c.nbc * kCondEntries * 2, 0ull,
                        nullptr);
    if (e == hipSuccess) e = launch_fill_u32(c.fill, c.nbc, 0u, nullptr);
    if (e == hipSuccess) e = launch_condense_write(c, nullptr);
    if (e == hipSuccess) e = hipMemcpy(err, c.err, sizeof err, hipMemcpyDeviceToHost);
    if (e != hipSuccess || err[1]) {
        (void)dev_free(c.idx);
        (void)dev_free(c.val);
        release();
        if (e != hipSuccess) return fail(MC_ERR_HIP, "condense: %s", hipGetErrorString(e));
        return fail(MC_ERR_TABLE_FULL, "condensed index without a free entry");
    }
    release();
    db->cidx = c.idx;
    db->nbc = c.nbc;
    db->cval = c.val;
    db->cval_n = total_vals;
    db->c_features = total_feats;
    db->version += 1;
    // pairs stored: features with one or two locations hold them inline
    {
        unsigned long long* cnt = nullptr;
        if (dev_alloc(&cnt, 1) == MC_OK) {
            unsigned long long n = 0;
            if (launch_fill_u64(cnt, 1, 0ull, nullptr) == hipSuccess &&
                launch_condense_pairs(db->cidx, db->nbc, cnt, nullptr) == hipSuccess &&
                hipMemcpy(&n, cnt, 8, hipMemcpyDeviceToHost) == hipSuccess)
                db->c_pairs = n;
            (void)dev_free(cnt);
        }
    }
    if (release_table) {
        HIP_TRY(dev_free(db->table));
        HIP_TRY(dev_free(db->bcount));
        db->table = nullptr;
        db->bcount = nullptr;
        db->table_released = true;
        (void)dev_free(db->pairs);
        (void)dev_free(db->parted);
        db->pairs = db->parted = nullptr;
        db->pairs_cap = 0;
    }
    return MC_OK;
}

int mc_db_set_profiling(mc_db* db, int enable) {
    if (int rc = check_db(db)) return rc;
    db->profiling = enable != 0;
    return MC_OK;
}

int mc_db_kernel_times(mc_db* db, double* ms, uint64_t* launches) {
    if (int rc = check_db(db)) return rc;
    if (!ms || !launches) return fail(MC_ERR_INVALID_ARG, "NULL output");
    DeviceGuard dg(db->device);
    hipError_t err = hipSuccess;
    for (int k = 0; k < MC_K_COUNT; ++k) {
        hipError_t e = drain(db->timers[k], &ms[k], &launches[k]);
        if (e != hipSuccess) err = e;
    }
    if (err != hipSuccess) return fail(MC_ERR_HIP, "kernel timing: %s", hipGetErrorString(err));
    return MC_OK;
}

int mc_db_dump(mc_db* db, uint32_t feature_lo, uint32_t feature_hi, uint32_t* features,
               uint32_t* locations, uint64_t capacity, uint64_t* n_out) {
    if (int rc = check_db(db)) return rc;
    if (!n_out || (capacity && (!features || !locations)))
        return fail(MC_ERR_INVALID_ARG, "NULL output");
    DeviceGuard dg(db->device);
    unsigned long long *cnt = nullptr, *buf = nullptr;
    int rc = dev_alloc(&cnt, 1);
    if (rc) return rc;
    rc = dev_alloc(&buf, std::max<uint64_t>(capacity, 1));
    if (rc) { (void)dev_free(cnt); return rc; }
    unsigned long long n = 0;
    std::vector<unsigned long long> host;
    hipError_t e = launch_fill_u64(cnt, 1, 0ull, nullptr);
    if (e == hipSuccess) {
        if (db->table_released)   // only the condensed layout is left
            e = launch_condense_dump(db->cidx, db->nbc, db->cval, feature_lo, feature_hi, buf,
                                     capacity, cnt, nullptr);
        else
            e = launch_dump(db->table, db->nb, feature_lo, feature_hi, buf, capacity, cnt,
                            nullptr);
    }
    if (e == hipSuccess) e = hipMemcpy(&n, cnt, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && n <= capacity && n) {
        host.resize(n);
        e = hipMemcpy(host.data(), buf, n * 8, hipMemcpyDeviceToHost);
    }
    (void)dev_free(cnt);
    (void)dev_free(buf);
    if (e != hipSuccess) return fail(MC_ERR_HIP, "dump: %s", hipGetErrorString(e));
    *n_out = n;
    if (n <= capacity) {
        std::sort(host.begin(), host.end());   // export order: feature, then location
        for (uint64_t i = 0; i < n; ++i) {
            features[i] = (uint32_t)(host[i] >> 32);
            locations[i] = (uint32_t)host[i];
        }
    }
    return MC_OK;
}

int mc_db_sketch(mc_db* db, const char* seqs_dev, const uint64_t* lengths, uint32_t n,
                 uint32_t* out_counts, uint32_t* out_features, void* stream) {
    if (int rc = check_db(db)) return rc;
    if (n == 0) return MC_OK;
    if (!seqs_dev || !lengths || !out_counts || !out_features)
        return fail(MC_ERR_INVALID_ARG, "NULL pointer");
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<TargetDesc> td(n);
    std::vector<uint64_t> tile_first(n + 1, 0);
    uint64_t off = 0, wins = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t nw = num_windows(lengths[i], db->k, db->S);
        if (nw > 0xFFFFFFFFull) return fail(MC_ERR_CAPACITY, "sequence too long");
        td[i] = TargetDesc{off, lengths[i], wins, i, (uint32_t)nw};
        tile_first[i + 1] = tile_first[i] + (nw + kTileWindows - 1) / kTileWindows;
        off += lengths[i];
        wins += nw;
    }
    TargetDesc* d_td = nullptr;
    uint64_t* d_tf = nullptr;
    int rc = dev_alloc(&d_td, n);
    if (rc) return rc;
    rc = dev_alloc(&d_tf, n + 1);
    if (rc) { (void)dev_free(d_td); return rc; }
    BuildArgs a{};
    a.text = reinterpret_cast<const uint8_t*>(seqs_dev);
    a.text_len = off;
    a.targets = d_td;
    a.n_targets = n;
    a.tile_first = d_tf;
    a.n_tiles = tile_first[n];
    a.k = db->k; a.w = db->w; a.S = db->S; a.s = db->s;
    a.chunk_tiles = scatter_chunk_tiles(db->s);
    a.out_counts = out_counts;
    a.out_feats = out_features;
    hipError_t e = hipMemcpyAsync(d_td, td.data(), n * sizeof(TargetDesc), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_tf, tile_first.data(), (n + 1) * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_sketch(a, false, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)dev_free(d_td);
    (void)dev_free(d_tf);
    if (e != hipSuccess) return fail(MC_ERR_HIP, "sketch: %s", hipGetErrorString(e));
    return MC_OK;
}

int mc_db_set_launch_config(mc_db* db, const mc_launch_config* cfg) {
    if (int rc = check_db(db)) return rc;
    if (!cfg) return fail(MC_ERR_INVALID_ARG, "cfg is NULL");
    ClassifyConfig c{cfg->list_capacity, cfg->waves_per_block, cfg->max_blocks};
    if (!classify_config_valid(c)) return fail(MC_ERR_INVALID_ARG, "unsupported launch config");
    for (auto& x : db->plan.shape) x = c;
    db->version += 1;
    return MC_OK;
}

int mc_db_get_launch_config(mc_db* db, mc_launch_config* cfg) {
    if (int rc = check_db(db)) return rc;
    if (!cfg) return fail(MC_ERR_INVALID_ARG, "cfg is NULL");
    cfg->list_capacity = db->plan.shape[0].list_cap;
    cfg->waves_per_block = db->plan.shape[0].waves_per_block;
    cfg->max_blocks = db->plan.shape[0].max_blocks;
    return MC_OK;
}

int mc_db_autotune(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                   const mc_query_opts* opts, uint32_t* out_labels, void* stream,
                   mc_launch_config* best, double* best_ms) {
    if (int rc = check_classify(db, reads, offsets, n_records, opts, out_labels)) return rc;
    if (n_records == 0) return fail(MC_ERR_INVALID_ARG, "autotune needs records");
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = 0;
    Workspace* w = workspace(db, st, n_records, &rc);
    if (!w) return rc;
    std::vector<uint32_t> ref(n_records), cur(n_records);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const uint32_t caps[] = {256, 512, 1024};
    const uint32_t wpbs[] = {2, 4, 8};
    const uint32_t grids[] = {2048, 8192, 16384, 32768, 1u << 30};
    // each size class in turn (the others keep their shapes); per class the
    // current shape first: it is kept unless another is faster by more than 2%
    // (timings are the best of three runs after a warm-up run). The tuned
    // shapes stay in the handle: a cache of one shape per size class.
    LaunchPlan plan = db->plan;
    double win_ms = 1e30;
    bool first = true;
    for (uint32_t cls = 0; cls < std::max<uint32_t>(1, plan.route.n); ++cls) {
        std::vector<ClassifyConfig> cands{plan.shape[cls]};
        for (uint32_t lc : caps)
            for (uint32_t wp : wpbs)
                for (uint32_t gb : grids) cands.push_back(ClassifyConfig{lc, wp, gb});
        ClassifyConfig win = plan.shape[cls];
        double cls_ms = 1e30;
        bool cls_first = true;
        for (const ClassifyConfig& c : cands) {
            LaunchPlan trial = plan;
            trial.shape[cls] = c;
            double ms = 1e30;
            for (int rep = 0; rep < 4; ++rep) {
                float t = 0.f;
                HIP_TRY(hipEventRecord(e0, st));
                rc = classify_launch(db, reads, offsets, n_records, *opts, out_labels, nullptr,
                                     *w, trial, st, false);
                if (rc) return rc;
                HIP_TRY(hipEventRecord(e1, st));
                HIP_TRY(hipEventSynchronize(e1));
                HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                if (rep > 0) ms = std::min(ms, (double)t);
            }
            HIP_TRY(hipMemcpy(first ? ref.data() : cur.data(), out_labels,
                              (size_t)n_records * 4, hipMemcpyDeviceToHost));
            if (!first && cur != ref)
                return fail(MC_ERR_STATE, "launch shapes disagree (class %u: %u, %u, %u)", cls,
                            c.list_cap, c.waves_per_block, c.max_blocks);
            first = false;
            if (cls_first || ms < 0.98 * cls_ms) {
                cls_ms = ms;
                win = c;
            }
            cls_first = false;
        }
        plan.shape[cls] = win;
        win_ms = cls_ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    db->plan = plan;
    db->version += 1;
    const ClassifyConfig& w0 = plan.shape[0];
    if (best) *best = mc_launch_config{w0.list_cap, w0.waves_per_block, w0.max_blocks};
    if (best_ms) *best_ms = win_ms;
    return MC_OK;
}

int mc_db_set_routing(mc_db* db, const mc_route_config* r) {
    if (int rc = check_db(db)) return rc;
    if (!r) return fail(MC_ERR_INVALID_ARG, "routing is NULL");
    if (r->n_classes < 1 || r->n_classes > kMaxRoutes)
        return fail(MC_ERR_INVALID_ARG, "n_classes %u not in 1..%u", r->n_classes, kMaxRoutes);
    LaunchPlan p;
    p.route.n = r->n_classes;
    for (uint32_t c = 0; c < kMaxRoutes; ++c) {
        const uint32_t lim = c < r->n_classes ? c : r->n_classes - 1;
        p.shape[c] = ClassifyConfig{r->shape[lim].list_capacity, r->shape[lim].waves_per_block,
                                    r->shape[lim].max_blocks};
        if (c < r->n_classes && !classify_config_valid(p.shape[c]))
            return fail(MC_ERR_INVALID_ARG, "unsupported launch shape of class %u", c);
        p.route.max_windows[c] = c + 1 < r->n_classes ? r->max_windows[c] : 0;
        if (c + 1 < r->n_classes && c > 0 && r->max_windows[c] <= r->max_windows[c - 1])
            return fail(MC_ERR_INVALID_ARG, "max_windows must ascend");
    }
    db->plan = p;
    db->version += 1;
    return MC_OK;
}

int mc_db_get_routing(mc_db* db, mc_route_config* r) {
    if (int rc = check_db(db)) return rc;
    if (!r) return fail(MC_ERR_INVALID_ARG, "routing is NULL");
    *r = mc_route_config{};
    r->n_classes = db->plan.route.n;
    for (uint32_t c = 0; c < kMaxRoutes; ++c) {
        r->max_windows[c] = db->plan.route.max_windows[c];
        r->shape[c] = mc_launch_config{db->plan.shape[c].list_cap,
                                       db->plan.shape[c].waves_per_block,
                                       db->plan.shape[c].max_blocks};
    }
    return MC_OK;
}

mc_graph* mc_classify_graph_create(mc_db* db, const char* reads, const uint64_t* offsets,
                                   uint32_t n_records, const mc_query_opts* opts,
                                   uint32_t* out_labels, mc_tophit* out_top, void* stream) {
    if (check_classify(db, reads, offsets, n_records, opts, out_labels)) return nullptr;
    if (n_records == 0) {
        fail(MC_ERR_INVALID_ARG, "a graph needs records");
        return nullptr;
    }
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    mc_graph* g = new mc_graph();
    g->db = db;
    g->reads = reads;
    g->offsets = offsets;
    g->n = n_records;
    g->opts = *opts;
    g->out_labels = out_labels;
    g->out_top = out_top;
    if (alloc_workspace(g->ws, n_records, st) != MC_OK || hipStreamSynchronize(st) != hipSuccess ||
        capture_graph(g, st) != MC_OK) {
        std::string e = g_err;
        mc_classify_graph_destroy(g);
        g_err = e;
        return nullptr;
    }
    return g;
}

int mc_classify_graph_launch(mc_graph* g, void* stream) {
    if (!g) return fail(MC_ERR_INVALID_ARG, "graph is NULL");
    DeviceGuard dg(g->db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->version != g->db->version) {
        if (int rc = check_classify(g->db, g->reads, g->offsets, g->n, &g->opts, g->out_labels))
            return rc;
        HIP_TRY(hipDeviceSynchronize());   // no replay of the old graph may still run
        if (int rc = capture_graph(g, st)) return rc;
    }
    HIP_TRY(hipGraphLaunch(g->exec, st));
    return MC_OK;
}

int mc_classify_graph_destroy(mc_graph* g) {
    if (!g) return MC_OK;
    DeviceGuard dg(g->db->device);
    (void)hipDeviceSynchronize();
    release_graph(g);
    free_workspace(g->ws);
    delete g;
    return MC_OK;
}

}  // extern "C"
