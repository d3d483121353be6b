// Microbenchmarks of the memory system the RAMBO hot path is bound by:
// uniformly random row reads (a probe) and random 32-bit atomic ORs (an
// insertion) over buffers of HBM size. They give the empirical ceiling that
// the probe and build kernels are compared with. Built as libmicro.so, not
// part of the index library.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MICRO_API extern "C" __attribute__((visibility("default")))

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Each lane issues `iters` rounds of U independent random reads of ROWB
// bytes (ROWB/16 uint4 loads at consecutive addresses) and folds them into
// a value written once, so no load can be removed.
template <int ROWB, int U>
__global__ __launch_bounds__(256) void k_gather(const uint4 *__restrict__ buf, uint64_t n_rows, uint32_t iters,
                                                uint64_t seed, uint4 *sink) {
    constexpr int V = ROWB >= 16 ? ROWB / 16 : 1;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = mix64(seed ^ (gid * U + u + 1));
    uint4 acc = {0, 0, 0, 0};
    for (uint32_t it = 0; it < iters; it++) {
        uint4 v[U][V];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t row = __umul64hi(x[u], n_rows);
            const uint4 *p = buf + row * V;
#pragma unroll
            for (int k = 0; k < V; k++) v[u][k] = p[k];
            x[u] = mix64(x[u] + 0x9E3779B97F4A7C15ULL);
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int k = 0; k < V; k++) {
                acc.x ^= v[u][k].x; acc.y ^= v[u][k].y; acc.z ^= v[u][k].z; acc.w ^= v[u][k].w;
            }
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x12345678u) sink[gid & 1023] = acc;
}

// 4-byte rows: one dword per probe
template <int U>
__global__ __launch_bounds__(256) void k_gather4(const uint32_t *__restrict__ buf, uint64_t n_rows, uint32_t iters,
                                                 uint64_t seed, uint32_t *sink) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = mix64(seed ^ (gid * U + u + 1));
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; it++) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            v[u] = buf[__umul64hi(x[u], n_rows)];
            x[u] = mix64(x[u] + 0x9E3779B97F4A7C15ULL);
        }
#pragma unroll
        for (int u = 0; u < U; u++) acc ^= v[u];
    }
    if (acc == 0x12345678u) sink[gid & 1023] = acc;
}

// Rows of ROWB bytes read cooperatively, as the probe kernel reads rows wider
// than 16 bytes: ROWB/16 consecutive lanes each load one 16-byte piece of the
// same random row; U rows in flight per lane group.
template <int ROWB, int U>
__global__ __launch_bounds__(256) void k_gather_coop(const uint4 *__restrict__ buf, uint64_t n_rows, uint32_t iters,
                                                     uint64_t seed, uint4 *sink) {
    constexpr int LPR = ROWB / 16;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t grp = gid / LPR;
    const uint32_t piece = threadIdx.x % LPR;
    uint64_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = mix64(seed ^ (grp * U + u + 1));
    uint4 acc = {0, 0, 0, 0};
    for (uint32_t it = 0; it < iters; it++) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            v[u] = buf[__umul64hi(x[u], n_rows) * LPR + piece];
            x[u] = mix64(x[u] + 0x9E3779B97F4A7C15ULL);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            acc.x ^= v[u].x; acc.y ^= v[u].y; acc.z ^= v[u].z; acc.w ^= v[u].w;
        }
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x12345678u) sink[gid & 1023] = acc;
}

// random single-bit atomic ORs into 32-bit words
__global__ __launch_bounds__(256) void k_atomic_or(uint32_t *buf, uint64_t n_words, uint32_t iters, uint64_t seed) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x = mix64(seed ^ (gid + 1));
    for (uint32_t it = 0; it < iters; it++) {
        atomicOr(buf + __umul64hi(x, n_words), 1u << (x & 31));
        x = mix64(x + 0x9E3779B97F4A7C15ULL);
    }
}

// plain streaming copy of n16 16-byte words: the known-size reference for
// the hardware byte counters (it reads and writes exactly 16 * n16 bytes)
__global__ __launch_bounds__(256) void k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

MICRO_API double micro_copy(void *dst, const void *src, uint64_t bytes, uint32_t blocks) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
    hipEventRecord(a, 0);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, (uint4 *)dst, (const uint4 *)src, bytes / 16);
    hipEventRecord(b, 0);
    if (hipEventSynchronize(b) != hipSuccess) return -3;
    float ms = 0;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    return ms;
}

// Returns the kernel time in ms (events), or a negative value on error.
// kind: 0 = gather (one lane per row), 1 = atomic OR, 2 = cooperative gather
// (row_bytes/16 lanes per row). row_bytes: 4, 16, 64 or 128 (kind 0); 32, 64,
// 128 or 256 (kind 2).
MICRO_API double micro_run(int kind, void *buf, uint64_t bytes, int row_bytes, uint32_t blocks, uint32_t iters,
                           uint64_t seed, void *sink) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
    hipEventRecord(a, 0);
    if (kind == 1) {
        hipLaunchKernelGGL(k_atomic_or, dim3(blocks), dim3(256), 0, 0, (uint32_t *)buf, bytes / 4, iters, seed);
    } else if (kind == 2) {
        const uint64_t rows = bytes / (uint64_t)row_bytes;
        switch (row_bytes) {
        case 32: hipLaunchKernelGGL((k_gather_coop<32, 4>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        case 64: hipLaunchKernelGGL((k_gather_coop<64, 4>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        case 128: hipLaunchKernelGGL((k_gather_coop<128, 4>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        case 256: hipLaunchKernelGGL((k_gather_coop<256, 4>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        default: return -2;
        }
    } else {
        const uint64_t rows = bytes / (uint64_t)row_bytes;
        switch (row_bytes) {
        case 4: hipLaunchKernelGGL((k_gather4<8>), dim3(blocks), dim3(256), 0, 0, (const uint32_t *)buf, rows, iters, seed, (uint32_t *)sink); break;
        case 16: hipLaunchKernelGGL((k_gather<16, 8>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        case 64: hipLaunchKernelGGL((k_gather<64, 4>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        case 128: hipLaunchKernelGGL((k_gather<128, 2>), dim3(blocks), dim3(256), 0, 0, (const uint4 *)buf, rows, iters, seed, (uint4 *)sink); break;
        default: return -2;
        }
    }
    hipEventRecord(b, 0);
    if (hipEventSynchronize(b) != hipSuccess) return -3;
    float ms = 0;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return -4;
    return ms;
}

// loads (or atomics) each lane issues per call, for throughput accounting
// (kind 2: one row per row_bytes/16 lanes per load)
MICRO_API uint32_t micro_per_lane(int kind, int row_bytes) {
    if (kind == 1) return 1;
    if (kind == 2) return 4;
    switch (row_bytes) {
    case 4: return 8;
    case 16: return 8;
    case 64: return 4;
    case 128: return 2;
    default: return 0;
    }
}
