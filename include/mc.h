/*
 * mc.h — C ABI of the MI355X minhash metagenomic classifier.
 *
 * Method: "MetaCache-GPU: Ultra-Fast Metagenomic Classification" (Kobus,
 * Mueller, Juenger, Hundt, Schmidt; ICPP'21). Build (Sec. 4.1, Sec. 5.2):
 * reference sequences are cut into windows of `window` bases overlapping by
 * k-1; every window is represented by its minhash sketch, the `sketch_size`
 * smallest distinct hashes h1 of its canonical k-mers (Sec. 2), and every
 * sketch element is stored in a multi-value hash table as
 * feature -> location (target id, window id), at most `max_locations` per
 * feature (Sec. 4.1). Query (Sec. 4.2, Sec. 5.2-5.6): every window of a read
 * (or read pair) is sketched the same way, the location lists of all sketch
 * elements are merged and counted per reference window, the best contiguous
 * window range per target is found with a sliding window, and the read is
 * labelled from its top hits, by lowest common ancestor when they are close.
 *
 * Every compute step runs in the library's HIP kernels on the current device
 * (gfx950). Functions return MC_OK (0) or a negative MC_ERR_* code; the text
 * of the last error of the calling thread is available from mc_last_error().
 * A db handle is not thread-safe: calls on one handle must not overlap.
 *
 * Fixed formats:
 *   base codes     A/a=0, C/c=1, G/g=2, T/t=3; any other byte is invalid and
 *                  no valid k-mer covers it.
 *   feature        h1(canonical k-mer), 32 bits; h1 is MurmurHash3's 32-bit
 *                  finalizer; canonical = min(forward, reverse complement)
 *                  with the first base most significant.
 *   location       (target << 18) | window; target < 16383, window < 2^18.
 *   labels         taxon ids from mc_db_set_taxonomy, or MC_UNCLASSIFIED.
 */
#ifndef MC_H
#define MC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_OK               0
#define MC_ERR_INVALID_ARG (-1)  /* bad pointer, size or parameter           */
#define MC_ERR_CAPACITY    (-2)  /* target or window id does not fit         */
#define MC_ERR_OOM         (-3)  /* device or pinned host allocation failed  */
#define MC_ERR_TABLE_FULL  (-4)  /* probe sequence exhausted (should not occur
                                    at the library's load factors)           */
#define MC_ERR_STATE       (-5)  /* call not valid in the handle's state     */
#define MC_ERR_HIP         (-6)  /* a HIP runtime call failed                */
#define MC_ERR_LIST        (-7)  /* a record's candidate list exceeded the
                                    largest supported size (see mc_classify_ex) */

#define MC_UNCLASSIFIED 0xFFFFFFFFu
#define MC_MAX_TARGETS  16383u
#define MC_MAX_WINDOWS  262144u

typedef struct mc_db mc_db;

/* Query options (Sec. 4.2, Sec. 5.6, Sec. 6.5).
 *   top_m       number of top hits kept per record (1..8); the paper uses 2..4.
 *   min_hits    hit threshold: a record whose best score is below it is
 *               unclassified.
 *   hit_diff    if best - second > hit_diff the label is the best target's
 *               taxon; otherwise the LCA of the taxa of all top hits whose
 *               score is at least best - hit_diff.
 *   insert_size fragment length used for pairs: the sliding window spans
 *               ceil((F-k)/S)+1 reference windows with F = max(l1+l2,
 *               insert_size) for a pair, F = read length otherwise.
 *   paired      0: record i is reads[offsets[i], offsets[i+1]).
 *               1: record i is mate 1 reads[offsets[2i], offsets[2i+1]) and
 *                  mate 2 reads[offsets[2i+1], offsets[2i+2]); an empty mate
 *                  marks a single-end record.
 * Defaults (mc_classify): {4, 4, 0, 0, 0}. */
typedef struct mc_query_opts {
    uint32_t top_m;
    uint32_t min_hits;
    uint32_t hit_diff;
    uint32_t insert_size;
    uint32_t paired;
} mc_query_opts;

/* One top hit: target id, score (hits summed over the best window range of
 * that target) and the first window of the range that holds a hit.
 * Unused entries are {MC_UNCLASSIFIED, 0, 0}. */
typedef struct mc_tophit {
    uint32_t target;
    uint32_t score;
    uint32_t window_begin;
} mc_tophit;

typedef struct mc_db_stats {
    uint64_t n_targets;
    uint64_t n_windows;        /* windows of all targets added so far       */
    uint64_t n_pairs_inserted; /* sketch elements inserted, before the cap  */
    uint64_t n_pairs_stored;   /* valid (feature, location) pairs stored    */
    uint64_t n_buckets;        /* 16 slots of 8 bytes per bucket            */
    uint64_t table_bytes;
    uint64_t n_cap_candidates; /* features re-checked against the cap       */
    uint64_t probe_sum;        /* sum over inserts of buckets probed - 1    */
    uint64_t n_rehash;         /* table growths                             */
    uint64_t q_features;       /* sketch elements looked up by classify     */
    uint64_t q_locations;      /* locations gathered by classify            */
    uint64_t q_probes;         /* bucket lines read by classify lookups     */
    uint64_t n_features;       /* distinct features among the stored pairs  */
    uint64_t n_tombstones;     /* slots of entries removed by the cap or by
                                  the rollback of a failed add              */
    double load_factor;        /* occupied slots (stored + tombstones) over
                                  all slots of the table                    */
    uint64_t condensed_bytes;  /* device bytes of the condensed layout (0 if
                                  none, see mc_db_condense)                 */
    uint64_t q_large_records;  /* records classify handed to its large-list
                                  pass (list over the launch's capacity)    */
    uint64_t q_hbm_records;    /* records handed on to the HBM-list pass
                                  (list over 16384 locations)               */
} mc_db_stats;

/* Text of the calling thread's last error ("" if none). Never NULL. */
const char* mc_last_error(void);

/* Create an empty database on the current HIP device.
 * 1 <= k <= 16; k <= window; S = window - k + 1 <= 256;
 * 1 <= sketch_size <= min(S, 64); 1 <= max_locations <= 65535.
 * Returns NULL (and sets mc_last_error) on invalid arguments or failure. */
mc_db* mc_db_create(uint32_t k, uint32_t window, uint32_t sketch_size,
                    uint32_t max_locations);

/* Free every device and host resource of the handle. NULL is accepted.
 * Device blocks of 1 MiB or more (the table, build scratch, query workspaces)
 * are freed, or kept mapped for reuse if mc_set_cached_memory_limit allows it. */
int mc_db_destroy(mc_db* db);

/* Reuse of large device blocks (process-wide, every device). Mapping and
 * unmapping tens of GB costs far more than a build (hundreds of milliseconds
 * to seconds), so a process that rebuilds databases may keep released blocks
 * of 1 MiB or more mapped, idle, for later allocations of the library on the
 * same device (a block serves a request up to 25% smaller than itself), while
 * the idle blocks of a device stay within `bytes_per_device`. Default 0:
 * nothing is kept, every release frees at once. Idle blocks are memory the
 * runtime counts as used: an allocation of the library that fails gives them
 * back and retries, other code must call mc_release_cached_memory. Lowering
 * the limit below what a device keeps releases that device's idle blocks.
 * Returns MC_OK, or MC_ERR_HIP if a release failed. */
int mc_set_cached_memory_limit(uint64_t bytes_per_device);

/* Give every device block the library keeps for reuse back to the runtime
 * (all devices), e.g. before other code needs that memory. Blocks in use by
 * live handles are not affected. Returns MC_OK, or MC_ERR_HIP. */
int mc_release_cached_memory(void);

/* Size the table for at least n_pairs stored pairs (optional; tables also
 * grow by themselves). load_factor in (0, 0.9]; 0 selects the default 0.5. */
int mc_db_reserve(mc_db* db, uint64_t n_pairs, double load_factor);

/* Add n reference sequences (Sec. 4.1). genomes: host bytes, all sequences
 * back to back (sum of lengths bytes); lengths, taxon_ids: host arrays of n.
 * Targets get consecutive ids starting at the current target count, in array
 * order. The caller keeps ownership; the call is synchronous. May be called
 * again after mc_classify (on-demand addition); new targets always get larger
 * ids, so the per-feature cap keeps its meaning. The call first waits for the
 * device: classifications still queued on any stream finish on the old table.
 * On any error nothing of the call is added: argument, capacity and
 * allocation errors are detected before the table is written; if inserts had
 * begun (MC_ERR_TABLE_FULL, MC_ERR_HIP), every entry of the call's targets is
 * turned into a tombstone (its slot stays occupied) before the call returns.
 * Only if that rollback fails as well does the error text say so: then the
 * handle must be destroyed.
 * MC_ERR_CAPACITY: more than MC_MAX_TARGETS targets in total, or a sequence
 * with more than MC_MAX_WINDOWS windows.
 * Device memory: besides the table (16 slots of 8 bytes a bucket, grown to
 * keep the load factor), the build uses 16 bytes per pair slot (sketch_size
 * slots a window) of its largest chunk; an add is cut into chunks of whole
 * sequences that fit about 60% of the free device memory, and scratch larger
 * than 512 MiB is released before the call returns. */
int mc_db_add_targets(mc_db* db, const char* genomes, const uint64_t* lengths,
                      const uint32_t* taxon_ids, uint32_t n);

/* Same as mc_db_add_targets, but genomes is a device pointer (already
 * resident in HBM); lengths and taxon_ids stay host arrays. Work is queued on
 * `stream` (a hipStream_t, NULL = default stream); the call returns after the
 * stream has finished it. */
int mc_db_add_targets_device(mc_db* db, const char* genomes_dev, const uint64_t* lengths,
                             const uint32_t* taxon_ids, uint32_t n, void* stream);

/* Set (or replace with a superset) the taxonomy (Sec. 4.1): parents[i] is the
 * parent of node i, host array of n_nodes. Exactly one root r with
 * parents[r] == r; every other chain must reach it (no cycles). */
int mc_db_set_taxonomy(mc_db* db, const uint32_t* parents, uint32_t n_nodes);

/* Classify n_reads single-end reads with the default options. reads, offsets
 * (n_reads+1 entries, u64) and out_labels (n_reads) are device pointers owned
 * by the caller. Asynchronous on `stream` (hipStream_t): labels are valid once
 * the stream has reached this point. Argument errors are returned at once;
 * MC_ERR_STATE if a target's taxon is not in the taxonomy. */
int mc_classify(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_reads,
                uint32_t* out_labels, void* stream);

/* Classify with options (see mc_query_opts). out_top: device array of
 * n_records * top_m entries, or NULL. Records of any length are classified
 * up to 16384 sketch elements and 2^20 merged candidate locations (a 40 kbp
 * read against 300 copies of one genome exceeds that); a record beyond
 * either limit is labelled MC_UNCLASSIFIED and counted, and
 * mc_db_query_status reports it. */
int mc_classify_ex(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                   const mc_query_opts* opts, uint32_t* out_labels, mc_tophit* out_top,
                   void* stream);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * classification as mc_classify_ex, bit for bit, with every device buffer
 * beyond the caller's inputs and outputs taken from a fixed scratch array of
 * MC_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends (its address is looked up on the first call on a
 * device). It calls no allocating routine. n_records must not exceed
 * MC_NOALLOC_MAX_RECORDS (MC_ERR_INVALID_ARG otherwise, nothing launched).
 * All calls on one device share that device's scratch: calls that overlap on
 * one GPU (other streams, other threads, other handles) race and must be
 * ordered by the caller. The scratch's counters are cleared by each call;
 * records too long for every pass are labelled MC_UNCLASSIFIED but not
 * reported through mc_db_query_status, and the handle's query statistics are
 * not updated. The handle must not change (additions, taxonomy, condensing)
 * while a call is in flight. */
#define MC_NOALLOC_MAX_RECORDS   1048576u
#define MC_NOALLOC_SCRATCH_BYTES 33817088u
int mc_classify_noalloc(mc_db* db, const char* reads, const uint64_t* offsets,
                        uint32_t n_records, const mc_query_opts* opts, uint32_t* out_labels,
                        mc_tophit* out_top, void* stream);

/* Waits for `stream`, then reports (and clears) the number of records since
 * the last call whose candidate list was too long (MC_ERR_LIST if > 0). */
int mc_db_query_status(mc_db* db, void* stream, uint64_t* n_too_long);

/* Inspection: when profiling is enabled, the library brackets its main
 * launches with HIP events on the launch stream: the three build kernels of
 * mc_db_add_targets* (sketch, partition scatter, insert) and the fast-path
 * classify kernel of mc_classify*. mc_db_kernel_times waits for those events
 * and writes, per kind (MC_K_*), the summed milliseconds and the number of
 * launches since the previous call into ms[MC_K_COUNT] and
 * launches[MC_K_COUNT] (host arrays), then resets them. */
#define MC_K_SKETCH   0
#define MC_K_SCATTER  1
#define MC_K_INSERT   2
#define MC_K_CLASSIFY 3
#define MC_K_COUNT    4
int mc_db_set_profiling(mc_db* db, int enable);
int mc_db_kernel_times(mc_db* db, double* ms, uint64_t* launches);

/* Launch shape of the fast classification path (tuning only; results never
 * depend on it): candidate locations held in LDS per record (256, 512 or
 * 1024; longer lists take the large-list pass), waves per workgroup (2, 4 or
 * 8) and the largest grid (records beyond it are taken grid-stride).
 * Default {512, 4, 16384}. */
typedef struct mc_launch_config {
    uint32_t list_capacity;
    uint32_t waves_per_block;
    uint32_t max_blocks;
} mc_launch_config;
int mc_db_set_launch_config(mc_db* db, const mc_launch_config* cfg);
int mc_db_get_launch_config(mc_db* db, mc_launch_config* cfg);

/* Size-class routing of uneven batches (Sec. 5.5: size-specialised launches
 * of the sort, here of the whole classification). Before the fast path, a
 * routing pass on the device groups the records by their number of windows
 * (both mates): class c takes the records with at most max_windows[c] windows
 * not taken by an earlier class, the last class all others; each class is
 * classified by its own launch with its own shape. n_classes = 1 (the
 * default) classifies all records in one launch. mc_db_set_launch_config sets
 * the shape of every class; mc_db_autotune tunes each class's shape in turn
 * and keeps them in the handle (one tuned shape per size class). Results never
 * depend on the routing. max_windows must ascend; shapes as for
 * mc_db_set_launch_config. */
#define MC_MAX_CLASSES 4
typedef struct mc_route_config {
    uint32_t n_classes;
    uint32_t max_windows[MC_MAX_CLASSES];
    mc_launch_config shape[MC_MAX_CLASSES];
} mc_route_config;
int mc_db_set_routing(mc_db* db, const mc_route_config* routing);
int mc_db_get_routing(mc_db* db, mc_route_config* routing);

/* Autotuner: classifies the given batch (device buffers, as mc_classify_ex)
 * with the current and every supported launch shape (best of three timed
 * runs after a warm-up each), checks that all give identical labels
 * (MC_ERR_STATE otherwise), keeps the fastest in the handle for later calls
 * (the current shape stays unless another is more than 2% faster) and reports
 * it (best and best_ms may be NULL). With size classes (mc_db_set_routing)
 * each class is tuned in turn, the others keeping their shapes; best reports
 * class 0's. Synchronous on `stream`. */
int mc_db_autotune(mc_db* db, const char* reads, const uint64_t* offsets, uint32_t n_records,
                   const mc_query_opts* opts, uint32_t* out_labels, void* stream,
                   mc_launch_config* best, double* best_ms);

/* A classification call (fixed device buffers and sizes, as mc_classify_ex)
 * captured once into a HIP graph and replayed with one launch; the buffers'
 * contents may change between replays. The graph owns its own workspace, so
 * replays must not overlap each other. If the database changed since the
 * capture (targets added, taxonomy or launch shape replaced), the next launch
 * captures it again. */
typedef struct mc_graph mc_graph;
mc_graph* mc_classify_graph_create(mc_db* db, const char* reads, const uint64_t* offsets,
                                   uint32_t n_records, const mc_query_opts* opts,
                                   uint32_t* out_labels, mc_tophit* out_top, void* stream);
int mc_classify_graph_launch(mc_graph* g, void* stream);
int mc_classify_graph_destroy(mc_graph* g);

/* Condensed query layout (Sec. 4.2, Sec. 5.1). Converts the current bucket
 * table (synchronously) into one 16-byte index entry per feature, in buckets
 * of eight (one 128-byte line) sized for a load of about one half, plus an
 * array with the ascending locations of every feature that has more than two
 * (a feature with one or two holds them in its entry). Later classifications
 * use it: a lookup reads one index line, and one contiguous run for features
 * with more than two locations, instead of the feature's bucket chain.
 * Results are the same as from the bucket table.
 * release_table = 0: the bucket table stays; an add (mc_db_add_targets*)
 *   drops the condensed layout and later classifications use the table again
 *   until mc_db_condense is called anew.
 * release_table = 1: the bucket table is freed (the query-only form): adds and
 *   mc_db_reserve then fail with MC_ERR_STATE; mc_db_dump reads the condensed
 *   layout; mc_db_get_stats reports its counts (no buckets, no tombstones).
 * Device memory during the call: the layout itself plus 12 bytes per 256
 * buckets of the table. Errors: MC_ERR_STATE (table already released),
 * MC_ERR_CAPACITY (more than 8,192 entries homed in 256 consecutive buckets,
 * which a table at the library's load factors does not reach), MC_ERR_OOM. */
int mc_db_condense(mc_db* db, int release_table);

/* Counters of the handle (synchronous; counts the table's slots). */
int mc_db_get_stats(mc_db* db, mc_db_stats* out);

/* Test entry point, not for production use: forces the insert path of later
 * mc_db_add_targets* calls on this handle, so that tests reach every path of
 * the build on small inputs. The stored table never depends on it. NULL (or
 * all fields zero) restores the automatic choice. Fields:
 *   global_insert  1: insert with global per-bucket counters in partitions of
 *                  part_mb MiB of table (0 = 256) instead of slice-local;
 *   slice_shift    slice insert: 2^slice_shift buckets per slice, 4..13;
 *   fine_bits      slice insert: 2^fine_bits slices per partition (used when
 *                  not below the automatic value and at most 10);
 *   stage_entries  slice insert: pairs staged in LDS per round (at least half
 *                  a slice's buckets and 64);
 *   direct         slice insert: 1 = every slice takes the direct path;
 *   chunk_slots    most pair slots of one build chunk;
 *   fail_after     1 = the next add reports MC_ERR_TABLE_FULL after all its
 *                  inserts ran, so that tests reach the rollback (the flag
 *                  clears itself).
 * MC_ERR_INVALID_ARG for slice_shift outside 4..13 (0 excepted). */
typedef struct mc_insert_path {
    uint32_t global_insert;
    uint32_t part_mb;
    uint32_t slice_shift;
    uint32_t fine_bits;
    uint32_t stage_entries;
    uint32_t direct;
    uint64_t chunk_slots;
    uint32_t fail_after;
    uint32_t reserved;
} mc_insert_path;
int mc_db_set_insert_path(mc_db* db, const mc_insert_path* path);

/* Test/inspection export, not part of the hot path: every stored pair whose
 * feature lies in [feature_lo, feature_hi], sorted by feature then location,
 * into host arrays of `capacity` entries. *n_out receives the number of pairs
 * (even when larger than capacity, in which case nothing is written). */
int mc_db_dump(mc_db* db, uint32_t feature_lo, uint32_t feature_hi, uint32_t* features,
               uint32_t* locations, uint64_t capacity, uint64_t* n_out);

/* Per-window sketches of n sequences with the handle's k, window and
 * sketch_size, computed by the same kernel code as the build (device inputs
 * and outputs; test/inspection export). seqs: device bytes back to back;
 * lengths: host array of n; out_counts: device u32 per window; out_features:
 * device u32, sketch_size per window; windows are numbered per sequence in
 * order, sequence after sequence. Synchronous. */
int mc_db_sketch(mc_db* db, const char* seqs_dev, const uint64_t* lengths, uint32_t n,
                 uint32_t* out_counts, uint32_t* out_features, void* stream);

/* ------------------------------------------------------------------------
 * Served form: a persistent request loop over a resident database.
 *
 * Interactive use keeps the database in memory between queries (Sec. 4); the
 * server adds continuous batching on top: a dispatcher thread admits queued
 * read batches, in order, into `slots` in-flight slots while the device memory
 * they need stays within `memory_budget`. Each slot has a worker thread, a HIP
 * stream, device buffers and pinned staging, so host staging, copies and
 * kernels of different batches overlap; batches complete out of order. Genome additions are queued
 * in the same order as batches: an addition waits for the batches submitted
 * before it, runs, and the batches submitted after it see the new targets.
 * While a server is attached, the database must not be used directly.
 * ------------------------------------------------------------------------ */
typedef struct mc_server mc_server;

typedef struct mc_server_opts {
    uint32_t slots;           /* batches in flight at once, 1..16 (0 = 4)            */
    uint64_t memory_budget;   /* device bytes of all slots' batch buffers together
                                 (0 = a quarter of the device memory free at
                                 creation); a batch is admitted when a free slot
                                 holds it, or can grow to hold it within the budget
                                 (the buffers of other free slots are released
                                 to make room)                                       */
    uint64_t staging_bytes;   /* initial device + pinned buffer per slot, grown in
                                 32 MiB steps when a batch needs more (0 = 64 MiB)   */
} mc_server_opts;

typedef struct mc_server_stats {
    uint64_t batches;         /* completed classification batches                   */
    uint64_t records;         /* records in them                                    */
    uint64_t bases;           /* read bytes in them                                 */
    uint64_t additions;       /* completed genome additions                          */
    double p50_ms, p99_ms;    /* batch latency percentiles: submit -> results in the
                                 caller's buffers                                    */
    double mean_ms, max_ms;
    double span_s;            /* first submit -> last completion                     */
} mc_server_stats;

/* Start a server on db (which it uses exclusively until destroyed). */
mc_server* mc_server_create(mc_db* db, const mc_server_opts* opts);

/* Queue a batch. reads/offsets/out_labels/out_top are HOST buffers owned by the
 * caller, laid out as for mc_classify_ex (offsets need not start at 0); they
 * must stay valid until mc_server_wait returns for the ticket. out_top may be
 * NULL. opts is copied. Returns at once with a ticket. A batch whose buffers
 * exceed the memory budget is rejected with MC_ERR_INVALID_ARG.
 * flags: MC_SUBMIT_PINNED if `reads` lies in pinned host memory (allocated
 * with hipHostMalloc or as pinned by the caller's framework): the bases are
 * then copied to the device directly, without staging. */
#define MC_SUBMIT_PINNED 1u
int mc_server_submit(mc_server* srv, const char* reads, const uint64_t* offsets,
                     uint32_t n_records, const mc_query_opts* opts, uint32_t* out_labels,
                     mc_tophit* out_top, uint32_t flags, uint64_t* ticket);

/* Queue a genome addition (as mc_db_add_targets) optionally followed by a
 * taxonomy replacement (parents may be NULL). genomes/lengths/taxon_ids/parents
 * are HOST buffers owned by the caller and are not copied: they must stay
 * valid until mc_server_wait returns for the ticket (or the server is
 * destroyed). The addition runs after every earlier batch has finished and
 * before any later one starts. */
int mc_server_add_targets(mc_server* srv, const char* genomes, const uint64_t* lengths,
                          const uint32_t* taxon_ids, uint32_t n, const uint32_t* parents,
                          uint32_t n_nodes, uint64_t* ticket);

/* Block until the job is done; returns its status (MC_OK or an error code) and
 * its latency in milliseconds (may be NULL). Each ticket can be waited once: a
 * second wait on it returns MC_ERR_INVALID_ARG at once. */
int mc_server_wait(mc_server* srv, uint64_t ticket, double* latency_ms);

/* Where a batch's latency went, from the host's clock (milliseconds). The
 * stages follow one another, so they add up to total_ms. For an addition only
 * total_ms is set; for a failed batch only total_ms. */
typedef struct mc_batch_times {
    double admit_ms;    /* submit -> given a slot (waiting for a free slot and memory
                           budget, or for an earlier addition)                       */
    double copy_ms;     /* -> its last read chunk on the device (earlier batches'
                           copies go first: one copy stream, admission order)        */
    double launch_ms;   /* -> its last chunk's kernels queued (earlier batches queue
                           theirs first)                                             */
    double finish_ms;   /* -> results in the caller's buffers (kernels, copy back)   */
    double total_ms;    /* submit -> results: the latency mc_server_wait reports     */
    /* On the device's clock (events on the slot's stream), inside finish_ms and
       the launches before it: from the stream reaching the batch's first
       kernels to its last fast-pass kernel done, and from there to the copies
       of its results back done. */
    double gpu_kernels_ms;
    double gpu_copy_back_ms;
} mc_batch_times;

/* mc_server_wait with the batch's latency split by stage (times may be NULL). */
int mc_server_wait_times(mc_server* srv, uint64_t ticket, mc_batch_times* times);

int mc_server_get_stats(mc_server* srv, mc_server_stats* out);

/* Finish every queued job, stop the dispatcher and free the server's
 * resources (not the database). NULL is accepted. */
int mc_server_destroy(mc_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MC_H */
