// Batched-form state shared by the query entry point and the serving loop.
#pragma once

#include <functional>

#include "rambo_int.h"

namespace rambo {

struct BatchBufs {
    uint32_t *rmask;           // [cap][R * RW] running AND per multi-tile read
    uint32_t *done;            // [cap] finished tiles per multi-tile read
    uint64_t *extra;           // [cap] tiles beyond the first, per read
    uint64_t *extra_off;       // [cap + 1] exclusive scan of extra
    unsigned long long *head;  // queue position
};

// Two captured graphs for one set of buffers: prep (per-read tile counts
// and their scan) and the persistent query kernel. The live batch size is
// read from d_n on the device, so the graphs serve any n <= cap.
struct BatchGraph {
    uint64_t cap = 0;
    unsigned blocks = 0;  // workgroups of the persistent launch
    Tune tune;
    BatchBufs bb{};
    uint64_t *d_n = nullptr;
    uint64_t *parts = nullptr;  // scan scratch
    void *mem = nullptr;
    hipGraph_t graph_prep = nullptr, graph_main = nullptr;
    hipGraphExec_t exec_prep = nullptr, exec_main = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // before prep, before main, after main
    ~BatchGraph();
};

// Capture the graphs for buffers (seqs, offs, out) of up to cap reads; if
// n_value is given, the live size is set to it once.
int make_batch_graph(rambo_s *h, const Tune &tu, const uint8_t *seqs, const uint64_t *offs, uint64_t cap,
                     uint64_t *out, const uint64_t *n_value, std::shared_ptr<BatchGraph> &res);
// Enqueue both graphs on s with the timing events between them.
int launch_batch_graph(rambo_s *h, BatchGraph &bg, hipStream_t s);
bool tune_valid(const rambo_s *h, const Tune &t);
int autotune(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out, hipStream_t s);

}  // namespace rambo
