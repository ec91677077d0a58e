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
    uint64_t dev_need = 0;       // device bytes while in flight
    // genome addition (copied)
    std::vector<char> genomes;
    std::vector<uint64_t> lengths;
    std::vector<uint32_t> taxa;
    std::vector<uint32_t> parents;
    Clock::time_point t_submit;
};

struct Done {
    int status = MC_OK;
    double ms = 0.0;
};

// One in-flight slot: stream, device buffers, pinned staging, completion event.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* d_buf = nullptr;
    uint64_t d_cap = 0;
    char* h_buf = nullptr;       // pinned
    uint64_t h_cap = 0;
    bool busy = false;
    Job job;
    // layout of the current job inside the buffers
    uint64_t off_reads = 0, off_offsets = 0, off_labels = 0, off_top = 0;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

}  // namespace

struct mc_server {
    mc_db* db = nullptr;
    int device = 0;
    uint32_t n_slots = 4;
    uint64_t budget = 0;
    std::vector<Slot> slots;
    std::deque<Job> queue;
    std::map<uint64_t, Done> done;
    std::mutex mu;
    std::condition_variable cv_queue, cv_done;
    bool stopping = false;
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0;
    std::thread thr;
    // stats
    std::vector<double> lat_ms;
    uint64_t batches = 0, records = 0, bases = 0, additions = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;

    void finish(const Job& j, int status) {
        const double ms =
            std::chrono::duration<double, std::milli>(Clock::now() - j.t_submit).count();
        std::lock_guard<std::mutex> lk(mu);
        done[j.ticket] = Done{status, ms};
        t_last = Clock::now();
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

    // Copy results of a completed slot to the caller and release the slot.
    void retire(Slot& s, int status) {
        if (status == MC_OK) {
            std::memcpy(s.job.out_labels, s.h_buf + s.off_labels, (size_t)s.job.n * 4);
            if (s.job.out_top)
                std::memcpy(s.job.out_top, s.h_buf + s.off_top,
                            (size_t)s.job.n * s.job.opts.top_m * sizeof(mc_tophit));
        }
        inflight_bytes -= s.job.dev_need;
        s.busy = false;
        finish(s.job, status);
    }

    // Retire every slot whose work is complete; with `block`, wait for at least one.
    void poll(bool block) {
        for (;;) {
            bool any_busy = false, any_done = false;
            for (auto& s : slots) {
                if (!s.busy) continue;
                any_busy = true;
                hipError_t e = hipEventQuery(s.done);
                if (e == hipSuccess) {
                    retire(s, MC_OK);
                    any_done = true;
                } else if (e != hipErrorNotReady) {
                    retire(s, MC_ERR_HIP);
                    any_done = true;
                }
            }
            if (!block || any_done || !any_busy) return;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }

    bool any_busy() const {
        for (auto& s : slots)
            if (s.busy) return true;
        return false;
    }

    int grow(Slot& s, uint64_t dev, uint64_t host) {
        if (dev > s.d_cap) {
            (void)hipStreamSynchronize(s.stream);
            (void)hipFree(s.d_buf);
            s.d_buf = nullptr;
            s.d_cap = 0;
            if (hipMalloc((void**)&s.d_buf, dev) != hipSuccess) return MC_ERR_OOM;
            s.d_cap = dev;
        }
        if (host > s.h_cap) {
            (void)hipStreamSynchronize(s.stream);
            (void)hipHostFree(s.h_buf);
            s.h_buf = nullptr;
            s.h_cap = 0;
            if (hipHostMalloc((void**)&s.h_buf, host, hipHostMallocDefault) != hipSuccess)
                return MC_ERR_OOM;
            s.h_cap = host;
        }
        return MC_OK;
    }

    // Stage a batch into a free slot and queue copy-in, classify, copy-out.
    void launch(Slot& s, Job&& j) {
        const uint64_t seg = (j.opts.paired ? 2ull : 1ull) * j.n;   // offsets - 1
        const uint64_t base = j.offsets[0];
        const uint64_t rb = j.offsets[seg] - base;
        s.off_reads = 0;
        s.off_offsets = align256(rb);
        s.off_labels = s.off_offsets + align256((seg + 1) * 8);
        s.off_top = s.off_labels + align256((uint64_t)j.n * 4);
        const uint64_t total =
            s.off_top + (j.out_top ? align256((uint64_t)j.n * j.opts.top_m * sizeof(mc_tophit)) : 0);
        int rc = grow(s, total, total);
        s.job = std::move(j);
        s.busy = true;
        inflight_bytes += s.job.dev_need;
        if (rc != MC_OK) { retire(s, rc); return; }
        std::memcpy(s.h_buf + s.off_reads, s.job.reads + base, rb);
        uint64_t* ho = reinterpret_cast<uint64_t*>(s.h_buf + s.off_offsets);
        for (uint64_t i = 0; i <= seg; ++i) ho[i] = s.job.offsets[i] - base;
        hipError_t e = hipMemcpyAsync(s.d_buf, s.h_buf, s.off_labels, hipMemcpyHostToDevice,
                                      s.stream);
        if (e == hipSuccess) {
            rc = mc_classify_ex(db, s.d_buf + s.off_reads,
                                reinterpret_cast<const uint64_t*>(s.d_buf + s.off_offsets),
                                s.job.n, &s.job.opts,
                                reinterpret_cast<uint32_t*>(s.d_buf + s.off_labels),
                                s.job.out_top ? reinterpret_cast<mc_tophit*>(s.d_buf + s.off_top)
                                              : nullptr,
                                s.stream);
            if (rc != MC_OK) { (void)hipStreamSynchronize(s.stream); retire(s, rc); return; }
            e = hipMemcpyAsync(s.h_buf + s.off_labels, s.d_buf + s.off_labels,
                               total - s.off_labels, hipMemcpyDeviceToHost, s.stream);
        }
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) { (void)hipStreamSynchronize(s.stream); retire(s, MC_ERR_HIP); }
    }

    void run_add(Job& j) {
        int rc = mc_db_add_targets(db, j.genomes.data(), j.lengths.data(), j.taxa.data(),
                                   (uint32_t)j.lengths.size());
        if (rc == MC_OK && !j.parents.empty())
            rc = mc_db_set_taxonomy(db, j.parents.data(), (uint32_t)j.parents.size());
        finish(j, rc);
    }

    void loop() {
        (void)hipSetDevice(device);
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> lk(mu);
                while (queue.empty() && !stopping) {
                    if (any_busy()) {
                        lk.unlock();
                        poll(false);
                        std::this_thread::sleep_for(std::chrono::microseconds(20));
                        lk.lock();
                    } else {
                        cv_queue.wait(lk);
                    }
                }
                if (queue.empty() && stopping) break;
                j = std::move(queue.front());
                queue.pop_front();
            }
            if (j.is_add) {
                while (any_busy()) poll(true);   // batches before the addition finish first
                run_add(j);
                continue;
            }
            // admission: a free slot and room in the memory budget
            for (;;) {
                poll(false);
                Slot* free_slot = nullptr;
                for (auto& s : slots)
                    if (!s.busy) { free_slot = &s; break; }
                if (free_slot && (inflight_bytes + j.dev_need <= budget || !any_busy())) {
                    launch(*free_slot, std::move(j));
                    break;
                }
                poll(true);
            }
        }
        while (any_busy()) poll(true);
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
    s->slots.resize(s->n_slots);
    bool ok = true;
    for (auto& sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
    }
    (void)hipSetDevice(prev);
    if (!ok) {
        mc_server_destroy(s);
        mc::set_error(MC_ERR_HIP, "stream/event creation failed");
        return nullptr;
    }
    s->thr = std::thread([s] { s->loop(); });
    return s;
}

int mc_server_submit(mc_server* srv, const char* reads, const uint64_t* offsets,
                     uint32_t n_records, const mc_query_opts* opts, uint32_t* out_labels,
                     mc_tophit* out_top, uint64_t* ticket) {
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
    const uint64_t seg = (opts->paired ? 2ull : 1ull) * n_records;
    for (uint64_t i = 0; i < seg; ++i)
        if (offsets[i + 1] < offsets[i])
            return mc::set_error(MC_ERR_INVALID_ARG, "offsets decrease");
    j.bytes = offsets[seg] - offsets[0];
    j.dev_need = align256(j.bytes) + align256((seg + 1) * 8) + align256((uint64_t)n_records * 4) +
                 (out_top ? align256((uint64_t)n_records * opts->top_m * sizeof(mc_tophit)) : 0) +
                 (uint64_t)n_records * 4;   // overflow queue of the workspace
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
    j.genomes.assign(genomes, genomes + total);
    j.lengths.assign(lengths, lengths + n);
    j.taxa.assign(taxon_ids, taxon_ids + n);
    if (parents && n_nodes) j.parents.assign(parents, parents + n_nodes);
    j.t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    j.ticket = srv->next_ticket++;
    *ticket = j.ticket;
    srv->queue.push_back(std::move(j));
    srv->cv_queue.notify_one();
    return MC_OK;
}

int mc_server_wait(mc_server* srv, uint64_t ticket, double* latency_ms) {
    if (!srv) return mc::set_error(MC_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket == 0 || ticket >= srv->next_ticket)
        return mc::set_error(MC_ERR_INVALID_ARG, "unknown ticket");
    srv->cv_done.wait(lk, [&] { return srv->done.count(ticket) != 0; });
    Done d = srv->done[ticket];
    srv->done.erase(ticket);
    if (latency_ms) *latency_ms = d.ms;
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
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (auto& s : srv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        (void)hipFree(s.d_buf);
        (void)hipHostFree(s.h_buf);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    (void)hipSetDevice(prev);
    delete srv;
    return MC_OK;
}

}  // extern "C"
