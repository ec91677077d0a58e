// Served form: a persistent request loop over a resident database with
// continuous batching (in-flight slots admitted by a device-memory budget),
// ordered genome additions between batches, and per-batch latency records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mc.h"
#include "mc_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t ticket = 0;
    bool is_add = false;
    // classification batch (caller's host buffers)
    const char* reads = nullptr;
    const uint64_t* offsets = nullptr;
    uint32_t n = 0;
    mc_query_opts opts{};
    uint32_t* out_labels = nullptr;
    mc_tophit* out_top = nullptr;
    uint64_t bytes = 0;          // read bytes
    bool pinned = false;         // reads are in pinned host memory
    uint64_t dev_need = 0;       // device bytes while in flight
    uint64_t order = 0;          // admission order (the order of the batches' copies in)
    // genome addition (caller's host buffers, valid until its ticket is waited on)
    const char* genomes = nullptr;
    const uint64_t* lengths = nullptr;
    const uint32_t* taxa = nullptr;
    uint32_t n_targets = 0;
    const uint32_t* parents = nullptr;
    uint32_t n_nodes = 0;
    Clock::time_point t_submit;
    // stages of a classification batch (set by the dispatcher and its worker)
    Clock::time_point t_admit, t_copied, t_launched;
    float gpu_kernels_ms = 0.f, gpu_copy_back_ms = 0.f;
};

struct Done {
    int status = MC_OK;
    double ms = 0.0;
    mc_batch_times times{};
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// One in-flight slot: a worker thread with its own stream, device buffers and
// pinned staging. The dispatcher hands it one batch at a time.
// Chunks of one batch (see mc_server::process).
constexpr uint64_t kChunkRecords = 131072;
constexpr uint32_t kMaxChunks = 16;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t copied[kMaxChunks] = {};   // chunk c of its batch is on the device
    hipEvent_t t_kernels = nullptr, t_kernels_done = nullptr, t_back = nullptr;   // timing
    char* d_buf = nullptr;
    uint64_t d_cap = 0;
    uint64_t d_plan = 0;         // device bytes granted by admission (guarded by the
                                 // server mutex); the worker grows d_buf to it
    char* h_buf = nullptr;       // pinned
    char* h_dev = nullptr;       // h_buf as the device addresses it
    uint64_t h_cap = 0;
    bool busy = false;           // owned by a batch (guarded by the server mutex)
    bool has_job = false;
    Job job;
    std::thread thr;
    std::condition_variable cv;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// A batch's results (labels, top hits, pass counters: one contiguous, 16-byte
// aligned region of the slot's device buffer) stored by the device straight
// into the slot's pinned host buffer. A copy-engine transfer back would queue
// behind other batches' large host-to-device copies; these stores take the
// other direction of the host link and finish with the kernel.
__global__ __launch_bounds__(256) void k_publish(const uint4* __restrict__ src,
                                                 uint4* __restrict__ dst, uint64_t n16) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Slot buffers grow in steps of this size (not by doubling, so that the
// capacity admission counts stays close to what batches need).
constexpr uint64_t kGrain = 32ull << 20;
uint64_t round_grain(uint64_t x) { return (x + kGrain - 1) / kGrain * kGrain; }

}  // namespace

struct mc_server {
    mc_db* db = nullptr;
    int device = 0;
    uint32_t n_slots = 4;
    uint64_t budget = 0;
    uint64_t staging = 64ull << 20;
    std::vector<Slot> slots;
    std::deque<Job> queue;
    std::map<uint64_t, Done> done;
    std::set<uint64_t> collected;   // tickets already waited on
    std::mutex mu;               // queue, slots' ownership, results, stats
    std::mutex launch_mu;        // calls into the database
    // Reads are copied in one batch at a time, in admission order, on one copy
    // stream: a batch's transfer gets the whole host link, as in plain
    // back-to-back launches, while classification and the copies out of
    // earlier batches overlap it on the slots' streams.
    hipStream_t copy_stream = nullptr;
    std::mutex copy_mu;
    std::condition_variable copy_cv;
    uint64_t copy_turn = 0;      // order of the next batch to copy in
    std::mutex launch_turn_mu;
    std::condition_variable launch_cv;
    uint64_t launch_turn = 0;    // order of the next batch to launch its kernels
    uint64_t next_order = 0;
    std::condition_variable cv_queue, cv_done, cv_slot;
    bool stopping = false;
    uint64_t next_ticket = 1;
    uint32_t busy_slots = 0;
    std::thread thr;
    // stats
    std::vector<double> lat_ms;
    uint64_t batches = 0, records = 0, bases = 0, additions = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;

    // Record a finished job (caller holds mu).
    void finish_locked(const Job& j, int status) {
        const Clock::time_point now = Clock::now();
        const double ms = ms_between(j.t_submit, now);
        Done d{status, ms, {}};
        if (!j.is_add && status == MC_OK) {
            d.times.admit_ms = ms_between(j.t_submit, j.t_admit);
            d.times.copy_ms = ms_between(j.t_admit, j.t_copied);
            d.times.launch_ms = ms_between(j.t_copied, j.t_launched);
            d.times.finish_ms = ms_between(j.t_launched, now);
            d.times.gpu_kernels_ms = j.gpu_kernels_ms;
            d.times.gpu_copy_back_ms = j.gpu_copy_back_ms;
        }
        d.times.total_ms = ms;
        done[j.ticket] = d;
        t_last = now;
        if (j.is_add) {
            additions += status == MC_OK;
        } else {
            batches += 1;
            records += j.n;
            bases += j.bytes;
            lat_ms.push_back(ms);
        }
        cv_done.notify_all();
    }

    // Device buffer of a slot to `dev_cap` bytes, pinned staging to at least
    // `need` bytes. Called by the slot's worker (or at creation).
    static int grow(Slot& s, uint64_t need, uint64_t dev_cap) {
        if (dev_cap > s.d_cap) {
            (void)hipFree(s.d_buf);
            s.d_buf = nullptr;
            s.d_cap = 0;
            if (hipMalloc((void**)&s.d_buf, dev_cap) != hipSuccess) return MC_ERR_OOM;
            s.d_cap = dev_cap;
        }
        if (need > s.h_cap) {
            uint64_t cap = std::max(round_grain(need), s.h_cap + s.h_cap / 2);
            (void)hipHostFree(s.h_buf);
            s.h_buf = nullptr;
            s.h_cap = 0;
            if (hipHostMalloc((void**)&s.h_buf, cap, hipHostMallocDefault) != hipSuccess)
                return MC_ERR_OOM;
            if (hipHostGetDevicePointer((void**)&s.h_dev, s.h_buf, 0) != hipSuccess) {
                (void)hipHostFree(s.h_buf);
                s.h_buf = nullptr;
                return MC_ERR_HIP;
            }
            // touch every page now: a page's first write otherwise faults in the
            // batch that reaches it (about 1.5 us a 4-KiB page, milliseconds a batch)
            std::memset(s.h_buf, 0, cap);
            s.h_cap = cap;
        }
        return MC_OK;
    }

    // Stage, copy in, classify, copy out and hand back one batch (worker thread).
    // A batch's turn in one of the server's admission-ordered sequences (the
    // copies in, the launches): taken once, on every path (a batch that fails
    // early still passes its turns on).
    struct Turn {
        std::mutex& mu;
        std::condition_variable& cv;
        uint64_t& next;
        uint64_t order;
        bool passed = false;
        void wait() {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return next == order; });
        }
        void pass() {
            if (passed) return;
            passed = true;
            {
                std::lock_guard<std::mutex> lk(mu);
                next += 1;
            }
            cv.notify_all();
        }
        ~Turn() {
            if (!passed) {
                wait();
                pass();
            }
        }
    };

    // A batch is classified in chunks of at least kChunkRecords records (at
    // most kMaxChunks of them): the copy of chunk c + 1 overlaps the
    // classification of chunk c. Batches copy in, and launch their kernels,
    // in admission order (an older batch's kernels are queued before a
    // younger one's, so it is not slowed down by batches that came after
    // it); their kernels and the copies back overlap on the slots' streams.
    // The reads keep their offsets: the classification's reads pointer is
    // the device buffer shifted by the batch's first offset, so the caller's
    // offsets are copied unchanged.
    //
    // Each chunk's fast pass counts the records it passes on in counters of
    // its own; they come back with the results, and only chunks that passed
    // records on get the large-list pass (then, the same way, the HBM-list
    // pass). A large-list workgroup takes most of a CU's LDS and starts only
    // on a CU that every other kernel has left: queued unconditionally next
    // to other batches' kernels, it would hold up every batch until the
    // device drains.
    int process(Slot& s, Job& j) {
        Turn turn{copy_mu, copy_cv, copy_turn, j.order};
        Turn launch{launch_turn_mu, launch_cv, launch_turn, j.order};
        const uint64_t per = j.opts.paired ? 2ull : 1ull;
        const uint64_t seg = per * j.n;   // offsets - 1
        const uint64_t base = j.offsets[0];
        const uint64_t rb = j.offsets[seg] - base;
        const uint64_t off_offsets = align256(rb);
        const uint64_t off_labels = off_offsets + align256((seg + 1) * 8);
        const uint64_t off_top = off_labels + align256((uint64_t)j.n * 4);
        const uint64_t top_bytes = (uint64_t)j.n * j.opts.top_m * sizeof(mc_tophit);
        const uint64_t off_cnt = off_top + (j.out_top ? align256(top_bytes) : 0);
        const uint64_t total = off_cnt + align256(4ull * mc::kNumQueryCounters * kMaxChunks);
        uint64_t plan;
        {
            std::lock_guard<std::mutex> lk(mu);
            plan = s.d_plan;
        }
        int rc = grow(s, total, std::max(plan, total));
        if (rc != MC_OK) return rc;
        {
            // the stream's record queues hold the whole batch (chunks queue
            // their records at ids of their own)
            std::lock_guard<std::mutex> lk(launch_mu);
            rc = mc::prepare_workspace(db, s.stream, j.n);
        }
        if (rc != MC_OK) return rc;
        std::memcpy(s.h_buf + off_offsets, j.offsets, (seg + 1) * 8);
        if (!j.pinned) std::memcpy(s.h_buf, j.reads + base, rb);
        const char* src = j.pinned ? j.reads + base : s.h_buf;   // pinned: direct DMA
        const uint64_t chunk = std::max<uint64_t>(kChunkRecords, (j.n + kMaxChunks - 1) / kMaxChunks);
        const uint32_t n_chunks = (uint32_t)((j.n + chunk - 1) / chunk);
        turn.wait();
        hipError_t e = hipMemcpyAsync(s.d_buf + off_offsets, s.h_buf + off_offsets,
                                      (seg + 1) * 8, hipMemcpyHostToDevice, copy_stream);
        for (uint32_t c = 0; c < n_chunks && e == hipSuccess; ++c) {
            const uint64_t r0 = c * chunk, r1 = std::min<uint64_t>(j.n, r0 + chunk);
            const uint64_t lo = j.offsets[per * r0] - base, hi = j.offsets[per * r1] - base;
            if (hi > lo)
                e = hipMemcpyAsync(s.d_buf + lo, src + lo, hi - lo, hipMemcpyHostToDevice,
                                   copy_stream);
            if (e == hipSuccess) e = hipEventRecord(s.copied[c], copy_stream);
        }
        turn.pass();
        if (e != hipSuccess) return MC_ERR_HIP;
        launch.wait();
        const char* reads = s.d_buf - base;   // reads + offsets[i] lies in the buffer
        const uint64_t* d_off = reinterpret_cast<const uint64_t*>(s.d_buf + off_offsets);
        uint32_t* d_lab = reinterpret_cast<uint32_t*>(s.d_buf + off_labels);
        mc_tophit* d_top = j.out_top ? reinterpret_cast<mc_tophit*>(s.d_buf + off_top) : nullptr;
        uint32_t* d_cnt = reinterpret_cast<uint32_t*>(s.d_buf + off_cnt);
        const uint32_t* h_cnt = reinterpret_cast<const uint32_t*>(s.h_buf + off_cnt);
        auto chunk_cnt = [&](uint32_t c, int which) { return h_cnt[c * mc::kNumQueryCounters + which]; };
        // phase p of chunk c (records [c chunk, (c + 1) chunk))
        auto classify = [&](int phase, uint32_t c, uint32_t n_queued) {
            const uint64_t r0 = c * chunk, r1 = std::min<uint64_t>(j.n, r0 + chunk);
            std::lock_guard<std::mutex> lk(launch_mu);
            return mc::served_classify(db, phase, reads, d_off, (uint32_t)r0, (uint32_t)r1, j.opts,
                                       d_lab, d_top, d_cnt + c * mc::kNumQueryCounters, n_queued,
                                       s.stream);
        };
        for (uint32_t c = 0; c < n_chunks; ++c) {
            // the worker waits for the chunk's copy itself: a wait queued on
            // the slot's stream would sit in a hardware queue that streams
            // share (more streams than hardware queues) and hold up the work
            // of other slots queued behind it until this batch's copy is done
            if (hipEventSynchronize(s.copied[c]) != hipSuccess) return MC_ERR_HIP;
            if (c + 1 == n_chunks) j.t_copied = Clock::now();
            if (c == 0 && hipEventRecord(s.t_kernels, s.stream) != hipSuccess) return MC_ERR_HIP;
            if ((rc = classify(0, c, 0)) != MC_OK) return rc;
        }
        if (n_chunks && hipEventRecord(s.t_kernels_done, s.stream) != hipSuccess) return MC_ERR_HIP;
        if (n_chunks == 0) j.t_copied = Clock::now();
        j.t_launched = Clock::now();
        launch.pass();
        // counters and results come back together, once after the last
        // chunk: a copy to host memory can hold the calling thread until the
        // stream reaches it (small copies are done by the host), which
        // between chunks would hold back the launches of the next chunks
        // [off_labels, off_cnt + the counters): labels, top hits, counters
        const uint64_t n16 = (off_cnt + 4ull * mc::kNumQueryCounters * n_chunks - off_labels + 15) / 16;
        auto copy_back = [&]() -> int {
            const unsigned grid = (unsigned)std::min<uint64_t>(1024, (n16 + 255) / 256);
            hipLaunchKernelGGL(k_publish, dim3(grid), dim3(256), 0, s.stream,
                               reinterpret_cast<const uint4*>(s.d_buf + off_labels),
                               reinterpret_cast<uint4*>(s.h_dev + off_labels), n16);
            hipError_t e2 = hipGetLastError();
            if (e2 == hipSuccess) e2 = hipEventRecord(s.t_back, s.stream);
            if (e2 != hipSuccess) return MC_ERR_HIP;
            return hipStreamSynchronize(s.stream) == hipSuccess ? MC_OK : MC_ERR_HIP;
        };
        if (n_chunks) {
            if ((rc = copy_back()) != MC_OK) return rc;
            (void)hipEventElapsedTime(&j.gpu_kernels_ms, s.t_kernels, s.t_kernels_done);
            (void)hipEventElapsedTime(&j.gpu_copy_back_ms, s.t_kernels_done, s.t_back);
        }
        // the passes for records with long candidate lists, where there are any
        for (int phase = 1; phase <= 2; ++phase) {
            const int which = phase == 1 ? mc::kQOverflow : mc::kQHuge;
            bool any = false;
            for (uint32_t c = 0; c < n_chunks; ++c) {
                const uint32_t q = chunk_cnt(c, which);
                if (!q) continue;
                any = true;
                if ((rc = classify(phase, c, q)) != MC_OK) return rc;
            }
            if (!any) break;
            if ((rc = copy_back()) != MC_OK) return rc;
        }
        std::memcpy(j.out_labels, s.h_buf + off_labels, (size_t)j.n * 4);
        if (j.out_top) std::memcpy(j.out_top, s.h_buf + off_top, top_bytes);
        return MC_OK;
    }

    void worker(Slot& s) {
        (void)hipSetDevice(device);
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                s.cv.wait(lk, [&] { return s.has_job || stopping; });
                if (!s.has_job) return;
            }
            int rc = process(s, s.job);
            std::lock_guard<std::mutex> lk(mu);
            finish_locked(s.job, rc);
            s.job = Job();
            s.has_job = false;
            s.busy = false;
            busy_slots -= 1;
            cv_slot.notify_all();
        }
    }

    void run_add(Job& j) {
        int rc;
        {
            std::lock_guard<std::mutex> lk(launch_mu);
            rc = mc_db_add_targets(db, j.genomes, j.lengths, j.taxa, j.n_targets);
            if (rc == MC_OK && j.parents && j.n_nodes)
                rc = mc_db_set_taxonomy(db, j.parents, j.n_nodes);
        }
        std::lock_guard<std::mutex> lk(mu);
        finish_locked(j, rc);
    }

    // Device bytes granted to all slots (caller holds mu).
    uint64_t planned_locked() const {
        uint64_t t = 0;
        for (const Slot& s : slots) t += s.d_plan;
        return t;
    }

    // A free slot for a batch needing `need` device bytes within the budget,
    // or null (caller holds mu). The free slot with the smallest buffer that
    // holds the batch is taken; else the free slot with the largest buffer
    // grows, if the buffers of all slots together then stay within the
    // budget; to make room, the buffers of other free slots are released.
    // A batch never needs more than the budget (submit rejects it), so with
    // every slot free it always fits.
    Slot* pick_slot_locked(uint64_t need) {
        Slot *fit = nullptr, *grower = nullptr;
        for (Slot& s : slots) {
            if (s.busy) continue;
            if (s.d_plan >= need) {
                if (!fit || s.d_plan < fit->d_plan) fit = &s;
            } else if (!grower || s.d_plan > grower->d_plan) {
                grower = &s;
            }
        }
        if (fit) return fit;
        if (!grower) return nullptr;
        const uint64_t want = std::max(need, std::min(round_grain(need), budget));
        if (planned_locked() - grower->d_plan + want > budget) {
            for (Slot& s : slots) {
                if (s.busy || &s == grower || !s.d_plan) continue;
                // a free slot's buffer is not in use: its last batch has synced
                (void)hipFree(s.d_buf);
                s.d_buf = nullptr;
                s.d_cap = 0;
                s.d_plan = 0;
            }
            if (planned_locked() - grower->d_plan + want > budget) return nullptr;
        }
        grower->d_plan = want;
        return grower;
    }

    // Dispatcher: FIFO order; a batch waits for a free slot whose buffer,
    // with those of the other slots, fits the memory budget; an addition waits
    // until every earlier batch is done.
    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_queue.wait(lk, [&] { return !queue.empty() || stopping; });
            if (queue.empty()) break;
            Job j = std::move(queue.front());
            queue.pop_front();
            if (j.is_add) {
                cv_slot.wait(lk, [&] { return busy_slots == 0; });
                lk.unlock();
                run_add(j);
                lk.lock();
                continue;
            }
            Slot* free_slot = nullptr;
            cv_slot.wait(lk, [&] {
                free_slot = pick_slot_locked(j.dev_need);
                return free_slot != nullptr;
            });
            j.order = next_order++;
            j.t_admit = Clock::now();
            free_slot->busy = true;
            free_slot->has_job = true;
            busy_slots += 1;
            free_slot->job = std::move(j);
            free_slot->cv.notify_one();
        }
        cv_slot.wait(lk, [&] { return busy_slots == 0; });
    }
};

extern "C" {

mc_server* mc_server_create(mc_db* db, const mc_server_opts* opts) {
    if (!db) {
        mc::set_error(MC_ERR_INVALID_ARG, "db is NULL");
        return nullptr;
    }
    mc_server* s = new mc_server();
    s->db = db;
    s->device = mc::db_device(db);
    s->n_slots = opts && opts->slots ? opts->slots : 4;
    if (s->n_slots > 16) {
        delete s;
        mc::set_error(MC_ERR_INVALID_ARG, "slots must be in 1..16");
        return nullptr;
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    s->budget = opts && opts->memory_budget ? opts->memory_budget : free_b / 4;
    s->slots = std::vector<Slot>(s->n_slots);
    if (opts && opts->staging_bytes) s->staging = opts->staging_bytes;
    bool ok = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) == hipSuccess;
    const uint64_t initial = std::min(round_grain(s->staging), s->budget / s->n_slots);
    for (auto& sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        for (auto& ev : sl.copied)
            ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        for (hipEvent_t* ev : {&sl.t_kernels, &sl.t_kernels_done, &sl.t_back})
            ok = ok && hipEventCreate(ev) == hipSuccess;
        ok = ok && mc_server::grow(sl, s->staging, initial) == MC_OK;
        sl.d_plan = sl.d_cap;
        // the slot stream's query workspace, sized for a whole chunk: a
        // batch that allocated it would wait milliseconds (and hold up the
        // other slots' launches meanwhile)
        ok = ok && sl.stream && mc::prepare_workspace(db, sl.stream, kChunkRecords) == MC_OK;
    }
    (void)hipSetDevice(prev);
    if (!ok) {
        mc_server_destroy(s);
        mc::set_error(MC_ERR_OOM, "stream or staging allocation failed");
        return nullptr;
    }
    for (auto& sl : s->slots) sl.thr = std::thread([s, &sl] { s->worker(sl); });
    s->thr = std::thread([s] { s->loop(); });
    return s;
}

int mc_server_submit(mc_server* srv, const char* reads, const uint64_t* offsets,
                     uint32_t n_records, const mc_query_opts* opts, uint32_t* out_labels,
                     mc_tophit* out_top, uint32_t flags, uint64_t* ticket) {
    if (!srv || !opts || !offsets || !ticket || (n_records && (!reads || !out_labels)))
        return mc::set_error(MC_ERR_INVALID_ARG, "NULL argument");
    if (opts->top_m < 1 || opts->top_m > mc::kMaxTopM || opts->paired > 1)
        return mc::set_error(MC_ERR_INVALID_ARG, "invalid query options");
    Job j;
    j.reads = reads;
    j.offsets = offsets;
    j.n = n_records;
    j.opts = *opts;
    j.out_labels = out_labels;
    j.out_top = out_top;
    j.pinned = (flags & MC_SUBMIT_PINNED) != 0;
    const uint64_t seg = (opts->paired ? 2ull : 1ull) * n_records;
    for (uint64_t i = 0; i < seg; ++i)
        if (offsets[i + 1] < offsets[i])
            return mc::set_error(MC_ERR_INVALID_ARG, "offsets decrease");
    j.bytes = offsets[seg] - offsets[0];
    j.dev_need = align256(j.bytes) + align256((seg + 1) * 8) + align256((uint64_t)n_records * 4) +
                 (out_top ? align256((uint64_t)n_records * opts->top_m * sizeof(mc_tophit)) : 0) +
                 align256(4ull * mc::kNumQueryCounters * kMaxChunks);
    if (j.dev_need > srv->budget)
        return mc::set_error(MC_ERR_INVALID_ARG, "batch larger than the memory budget");
    j.t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->have_first) {
        srv->have_first = true;
        srv->t_first = j.t_submit;
    }
    j.ticket = srv->next_ticket++;
    *ticket = j.ticket;
    srv->queue.push_back(std::move(j));
    srv->cv_queue.notify_one();
    return MC_OK;
}

int mc_server_add_targets(mc_server* srv, const char* genomes, const uint64_t* lengths,
                          const uint32_t* taxon_ids, uint32_t n, const uint32_t* parents,
                          uint32_t n_nodes, uint64_t* ticket) {
    if (!srv || !ticket || (n && (!lengths || !taxon_ids)))
        return mc::set_error(MC_ERR_INVALID_ARG, "NULL argument");
    Job j;
    j.is_add = true;
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += lengths[i];
    if (total && !genomes) return mc::set_error(MC_ERR_INVALID_ARG, "genomes is NULL");
    j.genomes = genomes;
    j.lengths = lengths;
    j.taxa = taxon_ids;
    j.n_targets = n;
    j.parents = n_nodes ? parents : nullptr;
    j.n_nodes = parents ? n_nodes : 0;
    j.t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    j.ticket = srv->next_ticket++;
    *ticket = j.ticket;
    srv->queue.push_back(std::move(j));
    srv->cv_queue.notify_one();
    return MC_OK;
}

int mc_server_wait(mc_server* srv, uint64_t ticket, double* latency_ms) {
    mc_batch_times t{};
    const int rc = mc_server_wait_times(srv, ticket, &t);
    if (latency_ms) *latency_ms = t.total_ms;
    return rc;
}

int mc_server_wait_times(mc_server* srv, uint64_t ticket, mc_batch_times* times) {
    if (!srv) return mc::set_error(MC_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket == 0 || ticket >= srv->next_ticket)
        return mc::set_error(MC_ERR_INVALID_ARG, "unknown ticket");
    if (srv->collected.count(ticket))
        return mc::set_error(MC_ERR_INVALID_ARG, "ticket already waited on");
    srv->collected.insert(ticket);   // a concurrent second wait on it fails too
    srv->cv_done.wait(lk, [&] { return srv->done.count(ticket) != 0; });
    Done d = srv->done[ticket];
    srv->done.erase(ticket);
    if (times) *times = d.times;
    return d.status;
}

int mc_server_get_stats(mc_server* srv, mc_server_stats* out) {
    if (!srv || !out) return mc::set_error(MC_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    mc_server_stats st{};
    st.batches = srv->batches;
    st.records = srv->records;
    st.bases = srv->bases;
    st.additions = srv->additions;
    std::vector<double> v = srv->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {   // nearest rank
            size_t r = (size_t)std::ceil(p / 100.0 * v.size());
            return v[std::min(v.size() - 1, r ? r - 1 : 0)];
        };
        st.p50_ms = pct(50);
        st.p99_ms = pct(99);
        double sum = 0;
        for (double x : v) sum += x;
        st.mean_ms = sum / v.size();
        st.max_ms = v.back();
    }
    if (srv->have_first)
        st.span_s = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
    *out = st;
    return MC_OK;
}

int mc_server_destroy(mc_server* srv) {
    if (!srv) return MC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->cv_queue.notify_all();
    }
    if (srv->thr.joinable()) srv->thr.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (auto& s : srv->slots) s.cv.notify_all();
    }
    for (auto& s : srv->slots)
        if (s.thr.joinable()) s.thr.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (auto& s : srv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.stream) (void)mc::release_workspace(srv->db, s.stream);
        (void)hipFree(s.d_buf);
        (void)hipHostFree(s.h_buf);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        for (auto& ev : s.copied)
            if (ev) (void)hipEventDestroy(ev);
        for (hipEvent_t ev : {s.t_kernels, s.t_kernels_done, s.t_back})
            if (ev) (void)hipEventDestroy(ev);
    }
    if (srv->copy_stream) {
        (void)hipStreamSynchronize(srv->copy_stream);
        (void)hipStreamDestroy(srv->copy_stream);
    }
    (void)hipSetDevice(prev);
    delete srv;
    return MC_OK;
}

}  // extern "C"
