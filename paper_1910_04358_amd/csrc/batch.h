// Batched-form state shared by the query entry point and the serving loop.
#pragma once

#include <functional>

#include "rambo_int.h"

namespace rambo {

struct BatchBufs {
    uint32_t *rmask;           // [cap][R * RW] running AND per multi-tile read
    unsigned long long *done;  // [cap] per multi-tile read: finished tiles (low 32 bits) and
                               // finished tiles that held a valid window (high 32 bits)
    uint64_t *extra;           // [cap] tiles beyond the first, per read
    uint64_t *extra_off;       // [cap + 1] exclusive scan of extra
    uint32_t *order;           // [4][cap] reads by size class of their first tile
    unsigned long long *cls;   // reads of size class v at cls[16 v]
    unsigned long long *head;  // queue position
    uint32_t *smask;           // [cap][RW] repetition-0 AND over the scout windows (SCHED_PRESCOUT)
    uint32_t *live;            // [cap] bit 0: read not ended by the scout pass; bit 1: a scout
                               // window was valid (SCHED_PRESCOUT)
    uint64_t cap;
};

// Captured graphs for one batch description: prep (per-read tile counts and
// their scan; absent for the plain form) and the query kernel. The batch is
// read from the device header `in`, so the graphs serve any batch of up to
// cap reads placed anywhere the header points.
struct BatchGraph {
    uint64_t cap = 0;
    unsigned blocks = 0;  // workgroups of the persistent launch
    Tune tune;
    BatchBufs bb{};
    const InputHdr *in = nullptr;  // device
    uint64_t *parts = nullptr;     // scan scratch
    void *mem = nullptr;
    hipGraph_t graph_prep = nullptr, graph_main = nullptr;
    hipGraphExec_t exec_prep = nullptr, exec_main = nullptr;
    bool timed = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // before prep, before main, after main
    ~BatchGraph();
};

// Persistent batched form for batches described by in_dev (device; or, if
// null, by an owned header set once to *init), up to cap reads.
int make_batch_graph(rambo_s *h, const Tune &tu, const InputHdr *in_dev, const InputHdr *init, uint64_t cap,
                     uint64_t *out, std::shared_ptr<BatchGraph> &res, unsigned long long *counts = nullptr,
                     uint64_t *wm = nullptr);
// One-node graph of the plain kernel for batches described by in_dev.
int make_plain_graph(rambo_s *h, const InputHdr *in_dev, uint64_t cap, uint64_t *out,
                     std::shared_ptr<BatchGraph> &res);
// Enqueue the graphs on s with the timing events between them.
int launch_batch_graph(rambo_s *h, BatchGraph &bg, hipStream_t s);
bool tune_valid(const rambo_s *h, const Tune &t);
int autotune(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out, hipStream_t s);

}  // namespace rambo
