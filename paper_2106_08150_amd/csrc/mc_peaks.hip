// Memory-system probes used as roofline denominators for the classifier's
// kernels: streaming copy, random 64-bit compare-and-swap, random 128-byte
// (and 64-byte) line reads, and the read-line-then-CAS pattern of a table
// insert, on a table of a given size. Not part of the classifier itself.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void k_init(unsigned long long* p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(256) void k_copy(const uint4* src, uint4* dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// One random 64-bit CAS per thread-iteration.
__global__ __launch_bounds__(256) void k_cas(unsigned long long* t, uint64_t n_slots,
                                             uint64_t n_ops, uint64_t seed,
                                             unsigned long long* sink) {
    unsigned long long acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t h = mix(i ^ seed);
        acc += atomicCAS(&t[__umul64hi(h, n_slots)], ~0ull, h | 1ull);
    }
    if (acc == 0x12345) sink[0] = acc;
}

// Groups of G lanes read one random line of G x 8 bytes.
template <int G>
__global__ __launch_bounds__(256) void k_lines(const unsigned long long* t, uint64_t n_lines,
                                               uint64_t n_ops, uint64_t seed,
                                               unsigned long long* sink) {
    const int gl = threadIdx.x % G;
    const uint64_t g0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const uint64_t gs = (uint64_t)gridDim.x * blockDim.x / G;
    unsigned long long acc = 0;
    for (uint64_t i = g0; i < n_ops; i += gs) {
        uint64_t line = __umul64hi(mix(i ^ seed), n_lines);
        acc ^= t[line * G + gl];
    }
    if (acc == 0x12345) sink[0] = acc;
}

// Insert pattern: 16 lanes read a random 128-byte line, the first empty slot
// is claimed with one CAS.
__global__ __launch_bounds__(256) void k_read_cas(unsigned long long* t, uint64_t n_lines,
                                                  uint64_t n_ops, uint64_t seed) {
    const int lane = threadIdx.x & 63, gl = lane & 15, g = lane >> 4;
    const uint64_t g0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 16;
    const uint64_t gs = (uint64_t)gridDim.x * blockDim.x / 16;
    for (uint64_t i0 = g0 - (g0 % 4); i0 < n_ops; i0 += gs) {   // wave-uniform trip count
        uint64_t i = i0 + (uint64_t)g;
        bool act = i < n_ops;
        uint64_t h = mix(i ^ seed);
        uint64_t line = __umul64hi(h, n_lines);
        unsigned long long v = act ? t[line * 16 + gl] : 0ull;
        uint64_t emp = __ballot(act && v == ~0ull);
        uint32_t gm = (uint32_t)(emp >> (16 * g)) & 0xFFFFu;
        if (act && gm && gl == __builtin_ctz(gm))
            atomicCAS(&t[line * 16 + gl], ~0ull, h | 1ull);
    }
}

unsigned grid_for(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

extern "C" {

// kind: 0 copy (rate = GB/s read+write), 1 random CAS (Gops/s), 2 random 128 B
// lines (Glines/s), 3 random 64 B lines (Glines/s), 4 line read + CAS
// (Ginserts/s). table_bytes is the working-set size; n_ops random operations
// per repetition. Returns 0 on success.
int mcp_measure(int kind, uint64_t table_bytes, uint64_t n_ops, int reps, double* rate,
                double* ms_per_rep) {
    if (table_bytes < 4096 || reps < 1 || !rate || !ms_per_rep) return -1;
    unsigned long long *t = nullptr, *t2 = nullptr, *sink = nullptr;
    uint64_t n_slots = table_bytes / 8;
    if (hipMalloc(&t, n_slots * 8) != hipSuccess) return -3;
    if (kind == 0 && hipMalloc(&t2, n_slots * 8) != hipSuccess) { (void)hipFree(t); return -3; }
    if (hipMalloc(&sink, 8) != hipSuccess) { (void)hipFree(t); (void)hipFree(t2); return -3; }
    hipLaunchKernelGGL(k_init, dim3(grid_for(n_slots)), dim3(256), 0, nullptr, t, n_slots, ~0ull);
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    float total = 0.f;
    for (int r = 0; r <= reps; ++r) {   // repetition 0 warms up
        if (kind == 1 || kind == 4)
            hipLaunchKernelGGL(k_init, dim3(grid_for(n_slots)), dim3(256), 0, nullptr, t,
                               n_slots, ~0ull);
        (void)hipEventRecord(a, nullptr);
        uint64_t seed = 0x51ed27ull * (uint64_t)(r + 1);
        switch (kind) {
            case 0:
                hipLaunchKernelGGL(k_copy, dim3(grid_for(n_slots / 2)), dim3(256), 0, nullptr,
                                   (const uint4*)t, (uint4*)t2, n_slots / 2);
                break;
            case 1:
                hipLaunchKernelGGL(k_cas, dim3(grid_for(n_ops)), dim3(256), 0, nullptr, t, n_slots,
                                   n_ops, seed, sink);
                break;
            case 2:
                hipLaunchKernelGGL((k_lines<16>), dim3(grid_for(n_ops * 16)), dim3(256), 0,
                                   nullptr, t, n_slots / 16, n_ops, seed, sink);
                break;
            case 3:
                hipLaunchKernelGGL((k_lines<8>), dim3(grid_for(n_ops * 8)), dim3(256), 0, nullptr,
                                   t, n_slots / 8, n_ops, seed, sink);
                break;
            case 4:
                hipLaunchKernelGGL(k_read_cas, dim3(grid_for(n_ops * 16)), dim3(256), 0, nullptr,
                                   t, n_slots / 16, n_ops, seed);
                break;
            default:
                break;
        }
        (void)hipEventRecord(b, nullptr);
        (void)hipEventSynchronize(b);
        float x = 0.f;
        (void)hipEventElapsedTime(&x, a, b);
        if (r > 0) total += x;
    }
    hipError_t e = hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(t);
    (void)hipFree(t2);
    (void)hipFree(sink);
    if (e != hipSuccess) return -6;
    double ms = total / reps;
    *ms_per_rep = ms;
    if (kind == 0) *rate = 2.0 * (double)(n_slots * 8) / (ms * 1e-3) / 1e9;
    else *rate = (double)n_ops / (ms * 1e-3) / 1e9;
    return 0;
}

}  // extern "C"
