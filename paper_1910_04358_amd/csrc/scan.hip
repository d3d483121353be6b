// Device-wide exclusive prefix sum of uint64 counts, in three passes
// (per-block sums, scan of the block sums, per-block scan with the block's
// offset). The element count is read on the device, so the passes can be
// captured in a graph sized for a capacity.
#include "rambo_int.h"
#include "scan.h"

namespace rambo {

static constexpr uint32_t kScanThreads = 256, kScanPer = 4;
static constexpr uint64_t kScanChunk = kScanThreads * kScanPer;  // elements per block

// exclusive scan of one value per thread across the workgroup; returns the
// workgroup total in *total
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t x, uint64_t *total) {
    __shared__ uint64_t wsum[kScanThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(incl, d);
        if ((int)lane >= d) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (uint32_t w = 0; w < kScanThreads / 64; w++) {
        const uint64_t s = wsum[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint64_t *__restrict__ v, const uint64_t *n_ptr,
                                                             uint64_t *__restrict__ part) {
    const uint64_t n = *n_ptr;
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; k++) {
        const uint64_t i = base + k * kScanThreads + threadIdx.x;
        if (i < n) s += v[i];
    }
    uint64_t total;
    (void)block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// exclusive scan of the block sums (one workgroup, looping), off[n] = total
__global__ __launch_bounds__(kScanThreads) void k_scan_parts(uint64_t *__restrict__ part, const uint64_t *n_ptr,
                                                            uint64_t *__restrict__ off) {
    const uint64_t n = *n_ptr;
    const uint64_t nb = (n + kScanChunk - 1) / kScanChunk;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += kScanThreads) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t x = i < nb ? part[i] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(x, &total);
        if (i < nb) part[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) off[n] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint64_t *__restrict__ v, const uint64_t *n_ptr,
                                                            const uint64_t *__restrict__ part,
                                                            uint64_t *__restrict__ off) {
    const uint64_t n = *n_ptr;
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
    if (base >= n) return;
    // thread t owns elements base + t*kScanPer .. +kScanPer-1
    uint64_t x[kScanPer], s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; k++) {
        const uint64_t i = base + threadIdx.x * kScanPer + k;
        x[k] = i < n ? v[i] : 0;
        s += x[k];
    }
    uint64_t total;
    uint64_t run = part[blockIdx.x] + block_exclusive_scan(s, &total);
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; k++) {
        const uint64_t i = base + threadIdx.x * kScanPer + k;
        if (i < n) off[i] = run;
        run += x[k];
    }
}

uint64_t scan_parts_needed(uint64_t cap) { return (cap + kScanChunk - 1) / kScanChunk + 1; }

int launch_exclusive_scan(const uint64_t *v, const uint64_t *n_ptr, uint64_t cap, uint64_t *off, uint64_t *parts,
                          hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, (cap + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_reduce, dim3(blocks), dim3(kScanThreads), 0, s, v, n_ptr, parts);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanThreads), 0, s, parts, n_ptr, off);
    hipLaunchKernelGGL(k_scan_apply, dim3(blocks), dim3(kScanThreads), 0, s, v, n_ptr, parts, off);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

}  // namespace rambo
