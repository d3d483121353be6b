// Host-side internals of librambo: the handle, error reporting and the
// launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rambo.h"
#include "rambo_dev.h"

#define RAMBO_API extern "C" __attribute__((visibility("default")))

namespace rambo {

int fail(int status, const char *fmt, ...);  // records the message, returns status
int ok();                                     // clears nothing, returns RAMBO_OK

#define HIP_CHECK(expr)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::rambo::fail(RAMBO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

// Launch shape of the sequence-query kernels; what the autotuner searches.
struct Tune {
    int seg = 4;          // 32-bit words of a row one lane reads (1, 2 or 4)
    int tile = 1024;      // windows per work item (multiple of 64), batched form
    int waves_per_cu = 16; // resident waves per CU of the persistent grid
    int wpb = 4;          // waves per workgroup
    int grab = 1;         // work items taken per queue access
    int sched = 2;        // probe schedule of a read's windows (SCHED_*; 2 = scout)
};

struct BatchGraph;  // batched-form state for one set of buffers (batch.hip)

}  // namespace rambo

struct rambo_s {
    uint64_t K = 0, m = 0, seed = 0, W = 0;
    uint32_t B = 0, R = 0, eta = 0, RW = 0, log2RW = 0;
    int device = 0, n_cu = 0;
    uint64_t rows_bytes = 0;
    bool opaque = false;  // documents are sets of opaque 64-bit terms
    // a shard (Section 5.3): local document l stands for global document
    // gids[l], whose cells are phi_r(gids[l]); empty for an ordinary index
    std::vector<uint64_t> gids;
    uint64_t *d_gids = nullptr;
    uint64_t gid_max = 0;
    // id-list queries: per-read answer sizes and scan scratch (grown as
    // needed; one id-list query at a time per handle)
    unsigned long long *d_ids_counts = nullptr;
    uint64_t *d_ids_wm = nullptr;  // [ids_counts_cap][(W + 63) / 64] non-zero word marks
    uint64_t *d_ids_aux = nullptr;
    uint64_t ids_counts_cap = 0;
    std::mutex ids_mu;
    uint32_t *rows = nullptr;
    rambo::HashParams *d_hp = nullptr;
    uint4 *d_cells = nullptr;  // [K] phi_r(d) of every repetition, 16 bits each
    uint4 *d_cells0 = nullptr; // [K] the same records in repetition 0's cell grouping (bdoc order)
    uint32_t *d_boff = nullptr, *d_bdoc = nullptr;
    unsigned long long *d_invalid = nullptr;  // [2]: invalid inputs, queries without a term
    unsigned long long *d_emptyq = nullptr;   // = d_invalid + 1
    std::vector<uint64_t> pa, pb, Alo, Ahi, Clo, Chi;
    std::vector<uint32_t> phi;  // [R][K]
    int mode = RAMBO_MODE_PLAIN, resolve = RAMBO_RESOLVE_AUTO, early_exit = 1;
    unsigned long long *probe_counter = nullptr;
    unsigned long long *sparse_counter = nullptr;  // RAMBO+ tallies, 6 words (rambo_set_sparse_counter)
    bool tuned = false;
    rambo::Tune tune;
    hipStream_t aux = nullptr;  // internal stream (graph capture, sync helpers)
    std::mutex mu;              // guards the graph cache and tuner
    std::map<std::string, std::shared_ptr<rambo::BatchGraph>> graphs;
    std::shared_ptr<rambo::BatchGraph> last_graph;  // most recently launched
};

namespace rambo {

inline Index make_index(const rambo_s *h) {
    Index ix;
    ix.rows = h->rows;
    ix.hp = h->d_hp;
    ix.cells = h->d_cells;
    ix.boff = h->d_boff;
    ix.bdoc = h->d_bdoc;
    ix.cells0 = h->d_cells0;
    ix.m = h->m;
    ix.K = h->K;
    ix.B = h->B;
    ix.R = h->R;
    ix.eta = h->eta;
    ix.RW = h->RW;
    ix.log2RW = h->log2RW;
    ix.W = (uint32_t)h->W;
    ix.opaque = h->opaque ? 1u : 0u;
    return ix;
}

struct QueryOpts {
    int rmode;                    // RAMBO_RESOLVE_*
    int early_exit;
    unsigned long long *probes;   // may be null
    int sched;                    // probe schedule (SCHED_*)
    unsigned long long *counts;   // id-list mode: per-read answer sizes, zero answers not written; or null
    unsigned long long *emptyq;   // incremented once per query that has no term (no valid window)
    unsigned long long *rplus;    // RAMBO+ tallies (plain form, sweep/scout schedules), or null
    uint64_t *wm;                 // id-list mode: per read, (W + 63) / 64 words whose bit j of word k marks
                                  // bitset word 64 k + j non-zero (only non-zero words are then written); or null
};

// api.hip: create an index (gids: null, or K global document ids of a shard)
rambo_s *create_index(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed, uint32_t flags,
                      const uint64_t *gids);

// build.hip
int launch_build_kmers(rambo_s *h, const uint64_t *kmers, const uint64_t *koff, const uint64_t *doc_ids,
                       uint64_t n_docs, hipStream_t s);
int launch_build_seqs(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, const uint64_t *doc_ids,
                      uint64_t n_docs, hipStream_t s);
int launch_dump_bfu(rambo_s *h, uint32_t r, uint32_t b, uint64_t *d_out, hipStream_t s);
int launch_fold(rambo_s *h, const uint32_t *in, uint32_t *out, uint32_t RWi, uint32_t log2RWo, uint32_t half,
                hipStream_t s);
// Checksum of the row array (index files), synchronous on s.
int rows_checksum(rambo_s *h, uint64_t *out, hipStream_t s);

// query.hip
int launch_query_kmers(rambo_s *h, const uint64_t *kmers, uint64_t n, uint64_t *out, hipStream_t s);
int launch_query_termsets(rambo_s *h, const uint64_t *terms, const uint64_t *offs, uint64_t n, uint64_t *out,
                          hipStream_t s);
// With hdr (device), the batch is read from it on the device and n is only
// the capacity the grid is sized for. With counts, id-list mode (QueryOpts).
int launch_query_seqs_plain(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n,
                            uint64_t *out, hipStream_t s, int seg, const InputHdr *hdr = nullptr,
                            unsigned long long *counts = nullptr, uint64_t *wm = nullptr);
// Bitsets of an id-list mode query to id lists: counts holds the n answer
// sizes the query wrote, aux ids_aux_words(n) words of scan scratch.
uint64_t ids_aux_words(uint64_t n);
// counts has n + 1 words: the answer sizes, then the number of reads without
// a term (RAMBO_OK_EMPTYQ is returned if it is not zero).
// With wm (the query's non-zero word marks), only the marked words are read.
int launch_ids(rambo_s *h, const uint64_t *bits, uint64_t n, uint32_t *ids, uint64_t *id_off,
               uint64_t ids_cap, hipStream_t s, const unsigned long long *counts, uint64_t *aux,
               const uint64_t *wm = nullptr);
// *p = v on stream s (a one-thread kernel: no memset node in captured work)
int launch_store_u64(uint64_t *p, uint64_t v, hipStream_t s);

// batch.hip
int query_seqs_batched(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out,
                       hipStream_t s, unsigned long long *counts = nullptr, uint64_t *wm = nullptr);
void drop_graphs(rambo_s *h);

// Row split: a lane reads SEG words of a row, G = row_words / SEG lanes share
// one term. The instantiated (SEG, G) pairs:
#define RAMBO_SPLITS(X) \
    X(1, 1) X(2, 1) X(4, 1) X(1, 2) X(2, 2) X(4, 2) X(1, 4) X(2, 4) X(4, 4) X(1, 8) X(2, 8) X(4, 8) \
    X(1, 16) X(2, 16) X(4, 16) X(1, 32) X(2, 32) X(4, 32) X(1, 64) X(2, 64) X(4, 64)

#define RAMBO_SPLIT_CASE_(S_, G_) case (S_) * 1000 + (G_): { constexpr int SEG = (S_), G = (G_); RAMBO_SPLIT_BODY_; } break;

// Expands RAMBO_SPLIT_BODY_ (defined by the caller, using SEG and G) for the
// runtime pair (SEGV, GV).
#define RAMBO_DISPATCH_SPLIT(SEGV, GV)                                                              \
    switch ((SEGV) * 1000 + (GV)) {                                                                 \
        RAMBO_SPLITS(RAMBO_SPLIT_CASE_)                                                             \
    default:                                                                                        \
        return ::rambo::fail(RAMBO_EINVAL, "unsupported row split seg=%d lanes=%d", (int)(SEGV), (int)(GV)); \
    }

inline bool split_supported(int seg, int G) {
#define RAMBO_SPLIT_TEST_(S_, G_) if (seg == (S_) && G == (G_)) return true;
    RAMBO_SPLITS(RAMBO_SPLIT_TEST_)
#undef RAMBO_SPLIT_TEST_
    return false;
}

// largest power-of-two segment (<= 4 words) that divides a row
inline int default_seg(uint32_t RW) { return RW >= 4 ? 4 : (int)RW; }

}  // namespace rambo
