// Device-wide exclusive scan of uint64 counts (scan.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rambo {

// Scratch words `parts` must hold for a capacity of cap elements.
uint64_t scan_parts_needed(uint64_t cap);

// off[i] = v[0] + ... + v[i-1] for i < n, off[n] = total, with n = *n_ptr
// (device) and n <= cap. Enqueued on s; capturable in a graph.
int launch_exclusive_scan(const uint64_t *v, const uint64_t *n_ptr, uint64_t cap, uint64_t *off, uint64_t *parts,
                          hipStream_t s);

}  // namespace rambo
