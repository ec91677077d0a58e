// Condensed query layout (Sec. 4.2, Sec. 5.1): after the build, the bucket
// table (one 8-byte slot per (feature, location) pair) is converted into a
// feature index (one 16-byte entry per feature) plus a value array holding,
// per feature with more than two locations, its locations in ascending order.
// A lookup then reads one index line and, for such features, one contiguous
// run, instead of every bucket line of the feature's chain.
//
// The conversion works on slices of 2^kCondSliceShift bucket-table buckets:
// all entries homed in a slice lie in its buckets or in the few buckets its
// chains run on into, so a workgroup gathers them, sorts them by (feature,
// location) in LDS and sees each feature's locations together. A count pass
// sizes the index and the value array; the write pass redoes the gather and
// sort, writes the runs at the slice's prefix of values and claims one index
// entry per feature with a per-bucket fill counter.
#include "mc_device.hpp"
#include "mc_internal.hpp"

namespace mc {

namespace {

constexpr int kCondThreads = 1024;
constexpr uint32_t kCondWaves = kCondThreads / kWave;

struct CondLds {
    unsigned long long key[kCondCap];   // feature << 32 | location, sorted
    uint16_t start[kCondCap + 1];       // first key of each distinct feature
    uint32_t wsum[kCondWaves];
    uint32_t n, nfeat, err;
    uint32_t end_bucket;                // offset of the first non-full bucket from b1 - 1
    unsigned long long vsum;
};

__device__ __forceinline__ bool bucket_full(const unsigned long long* table, uint64_t b) {
    return table[b * kSlots + (kSlots - 1)] != kEmpty;
}

// Exclusive prefix of one u32 per thread over the workgroup.
__device__ __forceinline__ uint32_t cond_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = shfl_idx(x, lane >= (uint32_t)d ? (int)lane - d : (int)lane);
        if (lane >= (uint32_t)d) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t base = 0;
    total = 0;
    for (uint32_t i = 0; i < kCondWaves; ++i) {
        const uint32_t y = wsum[i];
        if (i < w) base += y;
        total += y;
    }
    return base + x - v;
}

// Entries homed in slice z (buckets [b0, b1)) into L.key, sorted, and the
// first key of every distinct feature into L.start (L.start[nfeat] = n).
// Returns false (and sets L.err) if the slice holds more than kCondCap.
__device__ bool gather_slice(const CondArgs& c, uint32_t z, CondLds& L) {
    const uint32_t tid = threadIdx.x;
    const uint64_t b0 = (uint64_t)z << kCondSliceShift;
    const uint64_t b1 = b0 + (1ull << kCondSliceShift) < c.nb ? b0 + (1ull << kCondSliceShift)
                                                              : c.nb;
    if (tid == 0) {
        L.n = 0;
        L.err = 0;
        L.end_bucket = 0xFFFFFFFFu;
    }
    __syncthreads();
    // chains of features homed in the slice end at the first bucket that is
    // not full at or after b1 - 1 (buckets wrap around the table's end)
    // (chains are short: the first 64 buckets are tried first)
    for (uint64_t base = 0, width = kWave; base < c.nb; base += width, width = kCondThreads) {
        const uint64_t o = base + tid;
        if (tid < width && o < c.nb && !bucket_full(c.table, (b1 - 1 + o) % c.nb))
            atomicMin(&L.end_bucket, (uint32_t)o);
        __syncthreads();
        if (L.end_bucket != 0xFFFFFFFFu) break;
        __syncthreads();
    }
    const uint32_t end = L.end_bucket;
    __syncthreads();
    if (end == 0xFFFFFFFFu) return false;   // no bucket with a free slot: not a valid table
    // buckets [b0, b1 - 1 + end], each once
    uint64_t n_scan = (b1 - b0) + end;
    if (n_scan > c.nb) n_scan = c.nb;
    const uint64_t n_slots = n_scan * kSlots;
    for (uint64_t i = tid; i < n_slots; i += kCondThreads) {
        const uint64_t b = (b0 + i / kSlots) % c.nb;
        const unsigned long long e = c.table[b * kSlots + i % kSlots];
        if (!live_entry(e)) continue;
        const uint64_t h = home_bucket((uint32_t)(e >> 32), c.nb);
        if (h < b0 || h >= b1) continue;
        const uint32_t pos = atomicAdd(&L.n, 1u);
        if (pos < kCondCap) L.key[pos] = e;
        else L.err = 1;
    }
    __syncthreads();
    const bool bad = L.err != 0;
    const uint32_t n = L.n;
    __syncthreads();   // every thread has read them before the next slice resets them
    if (bad) return false;
    // bitonic sort of key[0, P), P the power of two >= n, padded with the largest key
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t i = n + tid; i < P; i += kCondThreads) L.key[i] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t x = tid; x < P / 2; x += kCondThreads) {
                const uint32_t i = (x / stride) * 2 * stride + (x % stride), j = i + stride;
                const bool asc = (i & size) == 0;
                const unsigned long long a = L.key[i], b = L.key[j];
                if ((a > b) == asc) {
                    L.key[i] = b;
                    L.key[j] = a;
                }
            }
            __syncthreads();
        }
    }
    // distinct features: a chunk of consecutive keys per thread
    const uint32_t per = (n + kCondThreads - 1) / kCondThreads;
    const uint32_t i0 = min(n, tid * per), i1 = min(n, i0 + per);
    uint32_t cnt = 0;
    for (uint32_t i = i0; i < i1; ++i)
        cnt += (i == 0 || (L.key[i] >> 32) != (L.key[i - 1] >> 32)) ? 1u : 0u;
    uint32_t total;
    uint32_t r = cond_scan(cnt, L.wsum, total);
    for (uint32_t i = i0; i < i1; ++i)
        if (i == 0 || (L.key[i] >> 32) != (L.key[i - 1] >> 32)) L.start[r++] = (uint16_t)i;
    if (tid == 0) {
        L.nfeat = total;
        L.start[total] = (uint16_t)n;
    }
    __syncthreads();
    return true;
}

// Count pass: distinct features and run values of every slice.
__global__ __launch_bounds__(kCondThreads) void k_condense_count(CondArgs c) {
    __shared__ CondLds L;
    for (uint32_t z = blockIdx.x; z < c.n_slices; z += gridDim.x) {
        if (!gather_slice(c, z, L)) {
            if (threadIdx.x == 0) atomicOr(&c.err[0], 1u);
            continue;
        }
        if (threadIdx.x == 0) L.vsum = 0;
        __syncthreads();
        unsigned long long v = 0;
        for (uint32_t f = threadIdx.x; f < L.nfeat; f += kCondThreads) {
            const uint32_t n = (uint32_t)L.start[f + 1] - L.start[f];
            if (n > kCondInline) v += n;
        }
        if (v) atomicAdd(&L.vsum, v);
        __syncthreads();
        if (threadIdx.x == 0) {
            c.slice_feats[z] = L.nfeat;
            c.slice_vals[z] = L.vsum;
        }
        __syncthreads();
    }
}

// Exclusive prefix of slice_vals in place (slice_vals[n_slices] = total) and
// the total of slice_feats, by one workgroup of 1024 threads.
__global__ __launch_bounds__(kCondThreads) void k_condense_scan(CondArgs c,
                                                                unsigned long long* total_feats) {
    __shared__ unsigned long long ws[kCondWaves], wf[kCondWaves];
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6, n = c.n_slices;
    const uint32_t per = (n + kCondThreads - 1) / kCondThreads;
    const uint32_t i0 = min(n, t * per), i1 = min(n, i0 + per);
    unsigned long long sv = 0, sf = 0;
    for (uint32_t i = i0; i < i1; ++i) {
        sv += c.slice_vals[i];
        sf += c.slice_feats[i];
    }
    unsigned long long x = sv;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int src = lane >= (uint32_t)d ? (int)lane - d : (int)lane;
        const uint32_t lo = shfl_idx((uint32_t)x, src), hi = shfl_idx((uint32_t)(x >> 32), src);
        if (lane >= (uint32_t)d) x += ((unsigned long long)hi << 32) | lo;
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const uint32_t lo = shfl_xor((uint32_t)sf, m), hi = shfl_xor((uint32_t)(sf >> 32), m);
        sf += ((unsigned long long)hi << 32) | lo;
    }
    if (lane == kWave - 1) ws[w] = x;
    if (lane == 0) wf[w] = sf;
    __syncthreads();
    unsigned long long base = 0, total = 0, tf = 0;
    for (uint32_t i = 0; i < kCondWaves; ++i) {
        if (i < w) base += ws[i];
        total += ws[i];
        tf += wf[i];
    }
    unsigned long long run = base + x - sv;
    for (uint32_t i = i0; i < i1; ++i) {
        const unsigned long long v = c.slice_vals[i];
        c.slice_vals[i] = run;
        run += v;
    }
    if (t == 0) {
        c.slice_vals[n] = total;
        *total_feats = tf;
    }
}

// Write pass: runs at the slice's value prefix (features in ascending order),
// one index entry per feature.
__global__ __launch_bounds__(kCondThreads) void k_condense_write(CondArgs c) {
    __shared__ CondLds L;
    for (uint32_t z = blockIdx.x; z < c.n_slices; z += gridDim.x) {
        if (!gather_slice(c, z, L)) continue;   // reported by the count pass
        // value offsets of the features' runs: a chunk of features per thread
        const uint32_t nf = L.nfeat;
        const uint32_t per = (nf + kCondThreads - 1) / kCondThreads;
        const uint32_t f0 = min(nf, threadIdx.x * per), f1 = min(nf, f0 + per);
        uint32_t own = 0;
        for (uint32_t f = f0; f < f1; ++f) {
            const uint32_t n = (uint32_t)L.start[f + 1] - L.start[f];
            if (n > kCondInline) own += n;
        }
        uint32_t total;
        uint64_t off = c.slice_vals[z] + cond_scan(own, L.wsum, total);
        for (uint32_t f = f0; f < f1; ++f) {
            const uint32_t s = L.start[f], n = (uint32_t)L.start[f + 1] - s;
            const uint32_t feat = (uint32_t)(L.key[s] >> 32);
            uint4 e;
            e.x = feat;
            e.y = n;
            if (n > kCondInline) {
                for (uint32_t i = 0; i < n; ++i) c.val[off + i] = (uint32_t)L.key[s + i];
                e.z = (uint32_t)off;
                e.w = (uint32_t)(off >> 32);
                off += n;
            } else {
                e.z = (uint32_t)L.key[s];
                e.w = n > 1 ? (uint32_t)L.key[s + 1] : 0u;
            }
            // claim an entry: the home bucket's next one, or the next bucket's
            uint64_t b = home_bucket(feat, c.nbc);
            bool placed = false;
            for (uint64_t d = 0; d < c.nbc && !placed; ++d) {
                if (c.fill[b] < kCondEntries) {
                    const uint32_t p = atomicAdd(&c.fill[b], 1u);
                    if (p < kCondEntries) {
                        reinterpret_cast<uint4*>(c.idx)[b * kCondEntries + p] = e;
                        placed = true;
                    }
                }
                b = b + 1 == c.nbc ? 0 : b + 1;
            }
            if (!placed) atomicOr(&c.err[1], 1u);
        }
        __syncthreads();
    }
}

// Test export: every (feature, location) of the condensed layout whose feature
// lies in [lo, hi].
__global__ __launch_bounds__(256) void k_condense_dump(const unsigned int* idx, uint64_t nbc,
                                                       const uint32_t* val, uint32_t lo,
                                                       uint32_t hi, unsigned long long* out,
                                                       uint64_t cap, unsigned long long* count) {
    const uint64_t n = nbc * kCondEntries;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 e = reinterpret_cast<const uint4*>(idx)[i];
        if (e.y == 0 || e.x < lo || e.x > hi) continue;
        const unsigned long long pos = atomicAdd(count, (unsigned long long)e.y);
        const unsigned long long f = (unsigned long long)e.x << 32;
        for (uint32_t k = 0; k < e.y; ++k) {
            uint32_t loc;
            if (e.y > kCondInline) loc = val[((uint64_t)e.w << 32 | e.z) + k];
            else loc = k == 0 ? e.z : e.w;
            if (pos + k < cap) out[pos + k] = f | loc;
        }
    }
}

// Pairs held by the condensed layout: the sum of its entries' counts, one
// atomic per wave.
__global__ __launch_bounds__(256) void k_condense_pairs(const unsigned int* idx, uint64_t nbc,
                                                        unsigned long long* total) {
    const uint64_t n = nbc * kCondEntries;
    unsigned long long sum = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        sum += reinterpret_cast<const uint4*>(idx)[i].y;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const uint32_t lo = shfl_xor((uint32_t)sum, m), hi = shfl_xor((uint32_t)(sum >> 32), m);
        sum += ((unsigned long long)hi << 32) | lo;
    }
    if (lane_id() == 0 && sum) atomicAdd(total, sum);
}

inline unsigned grid_cap(uint64_t items, unsigned max_blocks) {
    return (unsigned)(items < 1 ? 1 : items > max_blocks ? max_blocks : items);
}

}  // namespace

hipError_t launch_condense_count(const CondArgs& c, hipStream_t st) {
    hipLaunchKernelGGL(k_condense_count, dim3(grid_cap(c.n_slices, 8192)), dim3(kCondThreads), 0,
                       st, c);
    return hipGetLastError();
}

hipError_t launch_condense_scan(const CondArgs& c, unsigned long long* total_feats,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_condense_scan, dim3(1), dim3(kCondThreads), 0, st, c, total_feats);
    return hipGetLastError();
}

hipError_t launch_condense_write(const CondArgs& c, hipStream_t st) {
    hipLaunchKernelGGL(k_condense_write, dim3(grid_cap(c.n_slices, 8192)), dim3(kCondThreads), 0,
                       st, c);
    return hipGetLastError();
}

hipError_t launch_condense_pairs(const unsigned int* idx, uint64_t nbc, unsigned long long* total,
                                 hipStream_t st) {
    if (nbc == 0) return hipSuccess;
    const uint64_t n = nbc * kCondEntries;
    hipLaunchKernelGGL(k_condense_pairs, dim3(grid_cap((n + 255) / 256, 16384)), dim3(256), 0, st,
                       idx, nbc, total);
    return hipGetLastError();
}

hipError_t launch_condense_dump(const unsigned int* idx, uint64_t nbc, const uint32_t* val,
                                uint32_t lo, uint32_t hi, unsigned long long* out, uint64_t cap,
                                unsigned long long* count, hipStream_t st) {
    if (nbc == 0) return hipSuccess;
    const uint64_t n = nbc * kCondEntries;
    hipLaunchKernelGGL(k_condense_dump, dim3(grid_cap((n + 255) / 256, 16384)), dim3(256), 0, st,
                       idx, nbc, val, lo, hi, out, cap, count);
    return hipGetLastError();
}

}  // namespace mc
