// Construction (Algorithm 1): every term of document d sets, in every
// repetition r and for every Bloom hash j, bit phi_r(d) of row
// (r, h_{r,j}(term)) -- one atomic OR of one bit per (term, r, j). Bits are
// only ever set, so the result is independent of order and of repeats
// (streaming insertion, Section 3.2, is the same kernel on new documents).
#include "rambo_int.h"

namespace rambo {

__device__ __forceinline__ void scatter_term(const Index &ix, uint64_t x, uint64_t d) {
    const uint4 cd = ix.cells[d];
#pragma unroll
    for (int r = 0; r < MAXR; r++) {
        if (r < (int)ix.R) {
            const uint32_t b = cell_at(cd, r);
            const uint32_t bit = 1u << (b & 31);
#pragma unroll
            for (int j = 0; j < MAXETA; j++) {
                if (j < (int)ix.eta) {
                    const uint64_t pos = bloom_pos(ix, (uint32_t)r * ix.eta + j, x);
                    atomicOr(ix.rows + (((uint64_t)r * ix.m + pos) << ix.log2RW) + (b >> 5), bit);
                }
            }
        }
    }
}

// largest k < n with off[k] <= p (off non-decreasing, off[0] <= p)
__device__ __forceinline__ uint64_t find_doc(const uint64_t *off, uint64_t n, uint64_t p) {
    uint64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (off[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Documents given as k-mer codes: kmers[koff[i] .. koff[i+1]) belong to doc_ids[i].
__global__ __launch_bounds__(256) void k_build_kmers(Index ix, const uint64_t *__restrict__ kmers,
                                                     const uint64_t *__restrict__ koff,
                                                     const uint64_t *__restrict__ doc_ids, uint64_t n_docs,
                                                     unsigned long long *invalid) {
    const uint64_t first = koff[0], last = koff[n_docs];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = first + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < last; i += stride) {
        const uint64_t k = find_doc(koff, n_docs, i);
        const uint64_t d = doc_ids[k], x = kmers[i];
        if (d >= ix.K || (!ix.opaque && (x >> 62))) {
            atomicAdd(invalid, 1ULL);
            continue;
        }
        scatter_term(ix, ix.opaque ? x : canonical(x), d);
    }
}

// Documents given as sequences: seqs[offs[i] .. offs[i+1]) is document
// doc_ids[i]; its terms are its valid 31-windows. A wave takes 64
// consecutive byte positions of the concatenation per step.
__global__ __launch_bounds__(256) void k_build_seqs(Index ix, const uint8_t *__restrict__ seqs,
                                                    const uint64_t *__restrict__ offs,
                                                    const uint64_t *__restrict__ doc_ids, uint64_t n_docs,
                                                    unsigned long long *invalid) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t first = offs[0], last = offs[n_docs];
    const uint64_t nchunks = last > first ? (last - first + 63) / 64 : 0;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t ch = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; ch < nchunks; ch += nwaves) {
        const uint64_t p0 = first + ch * 64, p = p0 + lane;
        uint64_t k = find_doc(offs, n_docs, p0);
        while (k + 1 < n_docs && offs[k + 1] <= p) k++;
        const uint64_t dend = offs[k + 1];
        const uint32_t c0 = p < last ? seqs[p] : 0u;
        const uint32_t c1 = (lane < 30 && p + 64 < last) ? seqs[p + 64] : 0u;
        const Window w = extract_windows(c0, c1, lane);
        if (w.valid && p + 31 <= dend) {
            const uint64_t d = doc_ids[k];
            if (d >= ix.K) atomicAdd(invalid, 1ULL);
            else scatter_term(ix, w.canon, d);
        }
    }
}

// BFU(r, b) as a plain m-bit filter: lane l of a wave reads row base + l.
__global__ __launch_bounds__(256) void k_dump_bfu(Index ix, uint32_t r, uint32_t b, uint64_t *out) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t words = (ix.m + 63) / 64;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < words; w += nwaves) {
        const uint64_t p = w * 64 + lane;
        uint32_t bit = 0;
        if (p < ix.m) bit = (ix.rows[(((uint64_t)r * ix.m + p) << ix.log2RW) + (b >> 5)] >> (b & 31)) & 1u;
        const uint64_t word = __ballot(bit);
        if (lane == 0) out[w] = word;
    }
}

static unsigned grid_for(const rambo_s *h, uint64_t work_waves, unsigned per_cu) {
    uint64_t cap = (uint64_t)h->n_cu * per_cu;
    uint64_t blocks = (work_waves + 3) / 4;
    if (blocks > cap) blocks = cap;
    return (unsigned)(blocks ? blocks : 1);
}

int launch_build_kmers(rambo_s *h, const uint64_t *kmers, const uint64_t *koff, const uint64_t *doc_ids,
                       uint64_t n_docs, hipStream_t s) {
    // the grid is persistent (grid-stride); the k-mer count is only known on the device
    const unsigned grid = (unsigned)h->n_cu * 16;
    hipLaunchKernelGGL(k_build_kmers, dim3(grid), dim3(256), 0, s, make_index(h), kmers, koff, doc_ids, n_docs,
                       h->d_invalid);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

int launch_build_seqs(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, const uint64_t *doc_ids,
                      uint64_t n_docs, hipStream_t s) {
    const unsigned grid = (unsigned)h->n_cu * 16;
    hipLaunchKernelGGL(k_build_seqs, dim3(grid), dim3(256), 0, s, make_index(h), seqs, offs, doc_ids, n_docs,
                       h->d_invalid);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

int launch_dump_bfu(rambo_s *h, uint32_t r, uint32_t b, uint64_t *d_out, hipStream_t s) {
    const uint64_t words = (h->m + 63) / 64;
    hipLaunchKernelGGL(k_dump_bfu, dim3(grid_for(h, words, 16)), dim3(256), 0, s, make_index(h), r, b, d_out);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

}  // namespace rambo

namespace rambo {

// Folding over (Section 5.3): BFU'(r, b) = BFU(r, b) OR BFU(r, b + B/2) for
// b < B/2. In the bit-sliced layout this is, per row, the OR of the row's low
// B/2 bits with its bits [B/2, B) shifted down by B/2. One thread per output
// word; rows of RWo words (RWo = power of two >= ceil(B/2 / 32)).
__global__ __launch_bounds__(256) void k_fold(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                              uint64_t rows, uint32_t RWi, uint32_t log2RWo, uint32_t half) {
    const uint64_t n = rows << log2RWo;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t RWo = 1u << log2RWo;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t row = i >> log2RWo;
        const uint32_t w = (uint32_t)(i & (RWo - 1));
        const uint32_t *r = in + row * RWi;
        const uint32_t b0 = w * 32;  // first output bit of this word
        uint32_t keep = 0;           // output bits b0 + k with b0 + k < half
        if (b0 < half) keep = (half - b0 >= 32) ? 0xFFFFFFFFu : ((1u << (half - b0)) - 1u);
        uint32_t v = 0;
        if (keep) {
            const uint32_t lo = (w < RWi) ? r[w] : 0u;
            const uint32_t hb = half + b0, q = hb >> 5, sh = hb & 31;
            uint32_t hi = (q < RWi) ? (r[q] >> sh) : 0u;
            if (sh && q + 1 < RWi) hi |= r[q + 1] << (32 - sh);
            v = (lo | hi) & keep;
        }
        out[i] = v;
    }
}

// Rows of at most 128 bits (B <= 128): one thread per row, which loads the
// row whole, folds it as one 128-bit value, v | (v >> B/2) on the low B/2
// bits, and stores the folded row whole -- one load and one store per row,
// coalesced across the wave.
template <int RWI>
__global__ __launch_bounds__(256) void k_fold_rows(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                   uint64_t rows, uint32_t RWo, uint32_t half) {
    typedef unsigned __int128 u128;
    const u128 keep = (((u128)1) << half) - 1;  // half <= 64
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t row = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; row < rows; row += stride) {
        u128 v;
        if constexpr (RWI == 4) {
            const uint4 a = reinterpret_cast<const uint4 *>(in)[row];
            v = (u128)a.x | ((u128)a.y << 32) | ((u128)a.z << 64) | ((u128)a.w << 96);
        } else if constexpr (RWI == 2) {
            const uint2 a = reinterpret_cast<const uint2 *>(in)[row];
            v = (u128)a.x | ((u128)a.y << 32);
        } else {
            v = in[row];
        }
        const u128 f = (v | (v >> half)) & keep;
        if (RWo == 2) {
            reinterpret_cast<uint2 *>(out)[row] = make_uint2((uint32_t)f, (uint32_t)(f >> 32));
        } else {
            out[row] = (uint32_t)f;
        }
    }
}

int launch_fold(rambo_s *h, const uint32_t *in, uint32_t *out, uint32_t RWi, uint32_t log2RWo, uint32_t half,
                hipStream_t s) {
    const uint64_t rows = (uint64_t)h->R * h->m;
    const dim3 grid((unsigned)h->n_cu * 32), block(256);
    const uint32_t RWo = 1u << log2RWo;  // (half <= 64 when RWi <= 4: RWo is 1 or 2)
    if (RWi == 4) hipLaunchKernelGGL(k_fold_rows<4>, grid, block, 0, s, in, out, rows, RWo, half);
    else if (RWi == 2) hipLaunchKernelGGL(k_fold_rows<2>, grid, block, 0, s, in, out, rows, RWo, half);
    else if (RWi == 1) hipLaunchKernelGGL(k_fold_rows<1>, grid, block, 0, s, in, out, rows, RWo, half);
    else hipLaunchKernelGGL(k_fold, grid, block, 0, s, in, out, rows, RWi, log2RWo, half);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

// ---------------------------------------------------------------------------
// Checksum of the row array (index files): the sum, mod 2^64, of the
// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014) applied to
// (word index << 32 | word) over every 32-bit word. Each term depends on a
// word's value and place, so a changed, moved or missing word changes the sum
// except with probability about 2^-64; the sum is independent of the order of
// accumulation, so the grid adds its partial sums with atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix_word(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_rows_checksum(const uint32_t *__restrict__ w, uint64_t n,
                                                       unsigned long long *sum) {
    uint64_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        acc += mix_word((i << 32) | w[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(sum, part[0] + part[1] + part[2] + part[3]);
}

int rows_checksum(rambo_s *h, uint64_t *out, hipStream_t s) {
    unsigned long long *d = nullptr;
    HIP_CHECK(hipMallocAsync((void **)&d, 8, s));
    int st = RAMBO_OK;
    if (hipMemsetAsync(d, 0, 8, s) != hipSuccess) st = fail(RAMBO_EDEVICE, "checksum: memset failed");
    if (st == RAMBO_OK) {
        hipLaunchKernelGGL(k_rows_checksum, dim3((unsigned)(h->n_cu * 8)), dim3(256), 0, s, h->rows,
                           h->rows_bytes / 4, d);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(out, d, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = fail(RAMBO_EDEVICE, "checksum: launch or copy failed");
    }
    (void)hipFreeAsync(d, s);
    (void)hipStreamSynchronize(s);
    return st;
}

}  // namespace rambo
