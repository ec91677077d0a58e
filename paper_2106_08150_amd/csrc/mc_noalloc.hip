// Classification that allocates nothing (mc_classify_noalloc): for callers
// that cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation). Every device buffer of the
// classification beyond the caller's inputs and outputs (pass counters,
// routing data, record queues of the large-list and HBM-list passes, one
// region of the HBM-list pass) lives in one file-scope device array,
// `scratch`. Each GPU the library runs on holds its own copy of the array
// until the process ends; its device address is taken once per device, with
// that device current, and used for every launch on that device. Calls that
// overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/mc.h"
#include "mc_internal.hpp"

namespace {

constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

constexpr uint64_t kMaxRecords = MC_NOALLOC_MAX_RECORDS;
constexpr uint64_t kOffCounters = 0;
constexpr uint64_t kOffRoute = align256(kOffCounters + 4ull * mc::kNumQueryCounters);
constexpr uint64_t kOffQueue = align256(kOffRoute + 4ull * mc::kRouteMetaWords);
constexpr uint64_t kOffHuge = align256(kOffQueue + 4ull * 3 * kMaxRecords);
constexpr uint64_t kScratchBytes = kOffHuge + mc::kHugeRegionBytes;   // one HBM-list region
static_assert(kScratchBytes == MC_NOALLOC_SCRATCH_BYTES, "documented scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

int fail(int code, const char* fmt, unsigned long long a, unsigned long long b) {
    char msg[256];
    std::snprintf(msg, sizeof msg, fmt, a, b);
    return mc::set_error(code, msg);
}

// The scratch of `dev` (current device): its address from the runtime on the
// first call for that device.
int scratch_of(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MC_ERR_INVALID_ARG, "device %llu beyond the %llu supported",
                    (unsigned long long)dev, (unsigned long long)kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MC_ERR_HIP, "hipGetSymbolAddress of the scratch failed (error %llu, "
                        "device %llu)", (unsigned long long)e, (unsigned long long)dev);
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return MC_OK;
}

}  // namespace

extern "C" int mc_classify_noalloc(mc_db* db, const char* reads, const uint64_t* offsets,
                                   uint32_t n_records, const mc_query_opts* opts,
                                   uint32_t* out_labels, mc_tophit* out_top, void* stream) {
    if (!db) return mc::set_error(MC_ERR_INVALID_ARG, "db is NULL");
    if (n_records > kMaxRecords)
        return fail(MC_ERR_INVALID_ARG,
                    "%llu records exceed the %llu that mc_classify_noalloc's scratch holds",
                    n_records, kMaxRecords);
    const int dev = mc::db_device(db);
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return mc::set_error(MC_ERR_HIP, "no HIP device");
    if (prev != dev && hipSetDevice(dev) != hipSuccess)
        return mc::set_error(MC_ERR_HIP, "cannot select the database's device");
    unsigned char* base = nullptr;
    int rc = scratch_of(dev, &base);
    if (rc == MC_OK) {
        mc::ScratchView v;
        v.counters = reinterpret_cast<uint32_t*>(base + kOffCounters);
        v.route_meta = reinterpret_cast<uint32_t*>(base + kOffRoute);
        v.queue = reinterpret_cast<uint32_t*>(base + kOffQueue);
        v.queue_cap = kMaxRecords;
        v.huge = base + kOffHuge;
        v.huge_groups = 1;
        rc = mc::classify_into(db, reads, offsets, n_records, opts, out_labels, out_top, v,
                               static_cast<hipStream_t>(stream));
    }
    if (prev != dev) (void)hipSetDevice(prev);
    return rc;
}
