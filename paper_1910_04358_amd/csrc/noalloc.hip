// Id-list queries that allocate nothing: rambo_query_seqs_ids_noalloc.
//
// rambo_query_seqs_ids keeps each read's answer size and the scan's scratch
// in per-handle device buffers that it allocates (and grows) on demand. This
// variant takes them from one fixed array of the library instead, so a call
// makes no allocation of any kind: the caller passes the inputs and outputs,
// the query runs in the plain form (one wave per read, which needs no other
// scratch), and the answer sizes, the count of reads without a term and the
// scan's block sums live in `noalloc_scratch`.
//
// Each device the library runs on holds its own copy of the array (module
// globals are per device), at an address known only on the device: host code
// must never pass the array's name to a kernel or a copy. Its address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and that pointer is what the kernels receive.
#include <mutex>

#include "rambo_int.h"
#include "scan.h"

namespace rambo {
namespace {

constexpr uint64_t kMaxReads = RAMBO_NOALLOC_MAX_READS;
// answer sizes (kMaxReads), the count of reads without a term (1), and the
// scan's block sums plus the element count (ceil(kMaxReads / 1024) + 2,
// with room to spare)
constexpr uint64_t kScratchWords = kMaxReads + 1 + kMaxReads / 1024 + 64;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint64_t noalloc_scratch[kScratchWords];

std::mutex g_mu[kMaxDevices];  // one caller at a time per device: they share its array
uint64_t *g_ptr[kMaxDevices] = {};

// Device address of `noalloc_scratch` on `dev`; looked up on first use, with
// dev current (and the caller's current device restored afterwards). Called
// with g_mu[dev] held.
int scratch_on(int dev, uint64_t **out) {
    if (!g_ptr[dev]) {
        int cur = 0;
        HIP_CHECK(hipGetDevice(&cur));
        if (cur != dev) HIP_CHECK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr)
            return fail(RAMBO_EDEVICE, "rambo_query_seqs_ids_noalloc: scratch lookup failed: %s", hipGetErrorString(e));
        g_ptr[dev] = static_cast<uint64_t *>(p);
    }
    *out = g_ptr[dev];
    return RAMBO_OK;
}

}  // namespace
}  // namespace rambo

using namespace rambo;

RAMBO_API int rambo_query_seqs_ids_noalloc(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                                           uint64_t *bits, uint32_t *ids, uint64_t *id_offsets, uint64_t ids_cap,
                                           void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: null handle");
    if (!id_offsets) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: null id_offsets");
    if (h->opaque)
        return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: the index holds opaque terms, not 31-mers");
    if (n > kMaxReads)
        return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: %llu reads exceed the limit of %llu per call",
                    (unsigned long long)n, (unsigned long long)kMaxReads);
    if (n > 0 && (!bits || !seqs || !offsets)) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: null array");
    if (h->device < 0 || h->device >= kMaxDevices)
        return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: device %d out of range", h->device);
    const hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        int st = launch_store_u64(id_offsets, 0, s);
        if (st == RAMBO_OK) HIP_CHECK(hipStreamSynchronize(s));
        return st;
    }
    std::lock_guard<std::mutex> g(g_mu[h->device]);
    uint64_t *base = nullptr;
    int st = scratch_on(h->device, &base);
    if (st != RAMBO_OK) return st;
    unsigned long long *counts = reinterpret_cast<unsigned long long *>(base);  // n + 1 words
    uint64_t *aux = base + n + 1;                                                // ids_aux_words(n) words
    if (n + 1 + ids_aux_words(n) > kScratchWords)
        return fail(RAMBO_EINVAL, "rambo_query_seqs_ids_noalloc: scratch too small for %llu reads",
                    (unsigned long long)n);
    // every read's answer size is written by the query; only the count of
    // reads without a term is cleared first (by a kernel, not a memset)
    st = launch_store_u64(base + n, 0, s);
    if (st == RAMBO_OK)
        st = launch_query_seqs_plain(h, seqs, offsets, n, bits, s, default_seg(h->RW), nullptr, counts);
    if (st != RAMBO_OK) return st;
    // the scan and compaction end with a wait on s, so nothing of this call
    // uses the array once it returns
    return launch_ids(h, bits, n, ids, id_offsets, ids_cap, s, counts, aux);
}
