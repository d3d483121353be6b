// Sharding by document (Section 5.3, Figure 3): documents are routed to G
// shards by a random hash tau of their id; each shard is an independent
// RAMBO over its documents with the same R, m, seeds and node-local B = b,
// its documents keeping the cells of their global ids, phi_r(global id).
// Stacked, the shards are the RAMBO built directly with the two-level
// partition b * tau(d) + phi_r(d) over G * b cells: a document's answer is
// its answer in its own shard, so the answer of a query is the shards'
// answers put back at the documents' global ids. Here: the routing kernel,
// shard creation, and the kernel that stacks a shard's answers into
// global-id bitsets. On one GPU every shard is a handle on the same device;
// across GPUs each would be a handle on its own GPU.
#include <algorithm>

#include "rambo_int.h"

namespace rambo {

static constexpr uint64_t kP61 = (1ULL << 61) - 1;

// tau(d) = ((a d + b) mod P) mod G (Carter-Wegman over the Mersenne prime P;
// a d + b < 2^125 fits 128 bits)
__global__ __launch_bounds__(256) void k_route(const uint64_t *__restrict__ ids, uint64_t n, uint32_t G, uint64_t a,
                                               uint64_t b, uint32_t *__restrict__ shard) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const unsigned __int128 v = (unsigned __int128)a * ids[i] + b;
        shard[i] = (uint32_t)((uint64_t)(v % kP61) % G);
    }
}

// One wave per query: every document set in the shard's answer row (local
// ids) sets the bit of its global id in the global row. Shards own disjoint
// documents but share the global rows' words, hence the atomic ORs.
__global__ __launch_bounds__(256) void k_stack(const uint64_t *__restrict__ slice, uint64_t n, uint32_t Wl,
                                               const uint64_t *__restrict__ gids, uint64_t *out, uint64_t Wg) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t q = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (q >= n) return;
    const uint64_t *row = slice + q * Wl;
    uint64_t *dst = out + q * Wg;
    for (uint32_t w = lane; w < Wl; w += 64) {
        uint64_t word = row[w];
        while (word) {
            const uint32_t bit = (uint32_t)__builtin_ctzll(word);
            word &= word - 1;
            const uint64_t g = gids[(uint64_t)w * 64 + bit];
            atomicOr((unsigned long long *)(dst + (g >> 6)), 1ULL << (g & 63));
        }
    }
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), sequential form
static uint64_t sm_next(uint64_t &s) {
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace rambo

using namespace rambo;

RAMBO_API int rambo_route(const uint64_t *doc_ids, uint64_t n, uint32_t G, uint64_t route_seed, uint32_t *shard,
                          void *stream) {
    if (G == 0) return fail(RAMBO_EINVAL, "rambo_route: G = 0");
    if (n == 0) return RAMBO_OK;
    if (!doc_ids || !shard) return fail(RAMBO_EINVAL, "rambo_route: null array");
    uint64_t s = route_seed;
    const uint64_t a = 1 + sm_next(s) % (kP61 - 1);
    const uint64_t b = sm_next(s) % kP61;
    int dev = 0, n_cu = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)n_cu * 16));
    hipLaunchKernelGGL(k_route, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, doc_ids, n, G, a, b, shard);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

RAMBO_API rambo_t *rambo_create_shard(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                                      const uint64_t *global_ids) {
    if (!global_ids) {
        fail(RAMBO_EINVAL, "rambo_create_shard: null global_ids");
        return nullptr;
    }
    return create_index(K, B, R, m, eta, seed, 0, global_ids);
}

RAMBO_API int rambo_shard_ids(const rambo_t *h, uint64_t *out) {
    if (!h || !out) return fail(RAMBO_EINVAL, "rambo_shard_ids: null argument");
    if (h->gids.empty()) return fail(RAMBO_EINVAL, "rambo_shard_ids: the index is not a shard");
    std::copy(h->gids.begin(), h->gids.end(), out);
    return RAMBO_OK;
}

RAMBO_API int rambo_stack_slice(rambo_t *h, const uint64_t *slice, uint64_t n, uint64_t *out, uint64_t out_words,
                                void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_stack_slice: null handle");
    if (h->gids.empty()) return fail(RAMBO_EINVAL, "rambo_stack_slice: the index is not a shard");
    if (n == 0) return RAMBO_OK;
    if (!slice || !out) return fail(RAMBO_EINVAL, "rambo_stack_slice: null array");
    if (h->gid_max >= out_words * 64)
        return fail(RAMBO_EINVAL, "rambo_stack_slice: global id %llu needs more than %llu words per row",
                    (unsigned long long)h->gid_max, (unsigned long long)out_words);
    const uint64_t blocks = (n + 3) / 4;  // four waves per workgroup, one per query
    if (blocks > 0x7FFFFFFFULL) return fail(RAMBO_EINVAL, "rambo_stack_slice: batch too large");
    hipLaunchKernelGGL(k_stack, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, slice, n, (uint32_t)h->W,
                       h->d_gids, out, out_words);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}
