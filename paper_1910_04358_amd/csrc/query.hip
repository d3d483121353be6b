// Plain one-batch query kernels (Algorithm 2; Section 3.3.1 for sequences)
// and the bitset -> id-list compaction.
//
// Per term: R * eta row reads (one per Bloom hash and repetition), ANDed
// over j into the B-bit mask M_r of positive BFUs of repetition r. A
// sequence ANDs the masks of its terms across the lanes of its wave and
// stops at the first repetition whose mask is empty. The per-document AND
// over repetitions ("resolve") runs on the masks staged in LDS.
#include "rambo_int.h"
#include "scan.h"

namespace rambo {


// -------------------------------------------------------------------------
// single k-mer queries: 64 / G terms per wave, then one resolve per term
// -------------------------------------------------------------------------
template <int SEG, int G>
__global__ __launch_bounds__(256) void k_query_kmers(Index ix, const uint64_t *__restrict__ kmers, uint64_t n,
                                                     uint64_t *__restrict__ out, unsigned long long *invalid,
                                                     int rmode, int use_res) {
    constexpr int KPW = 64 / G;
    extern __shared__ uint64_t smem64[];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t mwords = ((KPW * ix.R * ix.RW) + 1) & ~1u;
    const uint32_t per_wave = mwords + (use_res ? 2 * ix.W : 0);
    uint32_t *M = reinterpret_cast<uint32_t *>(smem64) + wave * per_wave;
    uint64_t *res = use_res ? reinterpret_cast<uint64_t *>(M + mwords) : nullptr;

    const uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * KPW;
    if (base >= n) return;
    const uint32_t g = lane / G, seg = lane % G;
    const uint64_t q = base + g;

    Seg<SEG> acc[MAXR];
    set_ones(acc);
    if (q < n) {
        const uint64_t x = kmers[q];
        if (!ix.opaque && (x >> 62)) {
            if (seg == 0) atomicAdd(invalid, 1ULL);
#pragma unroll
            for (int r = 0; r < MAXR; r++)
#pragma unroll
                for (int s = 0; s < SEG; s++) acc[r].w[s] = 0;
        } else {
            probe_and<SEG>(ix, ix.opaque ? x : canonical(x), seg, acc);
        }
    }
    // stage every term's masks; alive = no repetition mask is empty
    uint64_t alive = ~0ULL;
    const uint64_t gm = (G >= 64) ? ~0ULL : ((1ULL << G) - 1);
#pragma unroll
    for (int r = 0; r < MAXR; r++) {
        if (r < (int)ix.R) {
            uint32_t o = 0;
#pragma unroll
            for (int s = 0; s < SEG; s++) {
                M[(g * ix.R + r) * ix.RW + seg * SEG + s] = acc[r].w[s];
                o |= acc[r].w[s];
            }
            const uint64_t bal = __ballot(o != 0);
            uint64_t a = 0;
#pragma unroll
            for (int t = 0; t < KPW; t++) a |= (uint64_t)(((bal >> (t * G)) & gm) != 0) << t;
            alive &= a;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const bool dense = rmode == RAMBO_RESOLVE_DENSE || res == nullptr || (rmode == RAMBO_RESOLVE_AUTO && ix.W <= 64);
    if (!dense) {
        for (int t = 0; t < KPW; t++) {
            const uint64_t row = base + t;
            if (row >= n) break;
            uint64_t *o = out + row * ix.W;
            if (!((alive >> t) & 1)) write_zeros(o, ix.W, lane);
            else resolve(ix, M + t * ix.R * ix.RW, res, o, lane, rmode);
        }
        return;
    }
    uint64_t live = alive;
    if (KPW < 64) live &= (1ULL << KPW) - 1;
    if (n - base < (uint64_t)KPW) live &= (1ULL << (n - base)) - 1;
    for (int t = 0; t < KPW; t++) {
        const uint64_t row = base + t;
        if (row >= n) break;
        if (!((live >> t) & 1)) write_zeros(out + row * ix.W, ix.W, lane);
    }
    if (!live) return;
    if constexpr (G == 1) {
        // One lane per term (B <= 128): transposed dense resolve. T[r][c] is
        // the 64-bit set of the wave's live terms whose repetition-r mask has
        // cell c; a document's terms are the AND over r of T[r][phi_r(d)],
        // and a 64 x 64 bit transpose turns the documents' term sets into
        // the terms' result words.
        uint64_t *T = reinterpret_cast<uint64_t *>(M);  // R * B words, fits the staging area
        const bool me_live = (live >> lane) & 1;
#pragma unroll
        for (int r = 0; r < MAXR; r++) {
            if (r < (int)ix.R) {
                uint64_t t0 = 0, t1 = 0;  // cells lane and 64 + lane
#pragma unroll
                for (int wi = 0; wi < SEG; wi++) {
                    for (uint32_t k = 0; k < 32; k++) {
                        const uint32_t c = (uint32_t)wi * 32 + k;
                        if (c >= ix.B) break;
                        const uint64_t tset = __ballot(me_live && ((acc[r].w[wi] >> k) & 1u));
                        if ((c & 63) == lane) {
                            if (c < 64) t0 = tset;
                            else t1 = tset;
                        }
                    }
                }
                if (lane < ix.B) T[r * ix.B + lane] = t0;
                if (64 + lane < ix.B) T[r * ix.B + 64 + lane] = t1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t w = 0; w < ix.W; w++) {
            const uint64_t d = (uint64_t)w * 64 + lane;
            uint64_t tm = 0;
            if (d < ix.K) {
                const uint4 cd = ix.cells[d];
                tm = ~0ULL;
#pragma unroll
                for (int r = 0; r < MAXR; r++)
                    if (r < (int)ix.R) tm &= T[r * ix.B + cell_at(cd, r)];
            }
            const uint64_t col = wave_transpose64(tm, lane);
            if (me_live) out[(base + lane) * ix.W + w] = col;
        }
        return;
    }
    // Dense resolve, word by word: the cells phi_r(d) of the word's 64
    // documents are loaded once and tested against every live term's masks.
    for (uint32_t w = 0; w < ix.W; w++) {
        const uint64_t d = (uint64_t)w * 64 + lane;
        const bool real = d < ix.K;
        const uint4 cd = real ? ix.cells[d] : make_uint4(0u, 0u, 0u, 0u);
        uint32_t ph[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; r++) ph[r] = cell_at(cd, r);
        uint64_t mine = 0, todo = live;
        while (todo) {
            const int t = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t *Mt = M + t * ix.R * ix.RW;
            uint32_t keep = real ? 1u : 0u;
#pragma unroll
            for (int r = 0; r < MAXR; r++)
                if (r < (int)ix.R) keep &= mask_bit(Mt + r * ix.RW, ph[r]);
            const uint64_t word = __ballot(keep);
            if (lane == (uint32_t)t) mine = word;
        }
        if ((live >> lane) & 1) out[(base + lane) * ix.W + w] = mine;
    }
}

// -------------------------------------------------------------------------
// sequence queries, plain form: one wave per read, 64 windows per step
// -------------------------------------------------------------------------
template <int SEG, int G, bool RPLUS>
__global__ __launch_bounds__(256) void k_query_seqs_plain(Index ix, const uint8_t *__restrict__ seqs,
                                                          const uint64_t *__restrict__ offs, uint64_t n,
                                                          const InputHdr *hdr, uint64_t *__restrict__ out,
                                                          QueryOpts opt, int use_res) {
    if (hdr) {  // batch described in device memory (graph replays)
        n = hdr->n;
        offs = hdr->offs;
        seqs = hdr->seqs;
    }
    extern __shared__ __align__(16) uint64_t smem64[];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const WaveLds L = wave_lds(ix.R * ix.RW, ix.W, use_res != 0, opt.sched == SCHED_SCOUT);
    uint32_t *M = reinterpret_cast<uint32_t *>(smem64) + wave * L.total;
    uint64_t *res = use_res ? reinterpret_cast<uint64_t *>(M + L.res) : nullptr;
    uint8_t *stage = opt.sched == SCHED_SCOUT ? reinterpret_cast<uint8_t *>(M + L.stage) : nullptr;

    const uint64_t read = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (read >= n) return;
    const uint64_t beg = offs[read];
    uint64_t end = offs[read + 1];
    if (end < beg) end = beg;
    const uint64_t nwin = end - beg >= 31 ? end - beg - 30 : 0;

    init_masks(ix, M, lane);
    const uint64_t issued = probe_windows<SEG, G, RPLUS>(ix, seqs, beg, end, 0, nwin, lane, M, opt.early_exit != 0,
                                                         opt.sched, stage, opt.rplus);
    if (opt.probes && lane == 0 && issued) atomicAdd(opt.probes, (unsigned long long)(issued * ix.eta));
    // every valid window is probed at least in repetition 0 unless a probe
    // has ended the read first, so nothing issued means no valid window
    if (issued == 0 && lane == 0) atomicAdd(opt.emptyq, 1ULL);
    uint64_t *o = out + read * ix.W;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    answer_read(ix, M, res, o, lane, opt.rmode, opt.counts, read, opt.wm);
}

// -------------------------------------------------------------------------
// term-set queries: one wave per set, 64 terms per step; repetition 0 over
// every term first, then the other repetitions (Section 3.3.1 order)
// -------------------------------------------------------------------------
template <int SEG, int G>
__global__ __launch_bounds__(256) void k_query_termsets(Index ix, const uint64_t *__restrict__ terms,
                                                        const uint64_t *__restrict__ offs, uint64_t n,
                                                        uint64_t *__restrict__ out, QueryOpts opt, int use_res,
                                                        unsigned long long *invalid) {
    extern __shared__ __align__(16) uint64_t smem64[];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const WaveLds L = wave_lds(ix.R * ix.RW, ix.W, use_res != 0, false);
    uint32_t *M = reinterpret_cast<uint32_t *>(smem64) + wave * L.total;
    uint64_t *res = use_res ? reinterpret_cast<uint64_t *>(M + L.res) : nullptr;

    const uint64_t q = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (q >= n) return;
    const uint64_t beg = offs[q];
    uint64_t end = offs[q + 1];
    if (end < beg) end = beg;
    const uint64_t len = end - beg;
    uint64_t *o = out + q * ix.W;
    if (len == 0 && lane == 0) atomicAdd(opt.emptyq, 1ULL);

    // a k-mer index takes 31-mer codes only: a set holding another value
    // answers no document
    bool bad = false;
    if (!ix.opaque)
        for (uint64_t w = 0; w < len && !bad; w += 64)
            bad = __ballot(w + lane < len && (terms[beg + w + lane] >> 62)) != 0;
    if (bad) {
        if (lane == 0) atomicAdd(invalid, 1ULL);
        write_zeros(o, ix.W, lane);
        return;
    }
    init_masks(ix, M, lane);
    uint64_t issued = 0;
    bool ended = false;
    for (int pass = 0; pass < 2 && !ended; pass++) {
        if (pass == 1 && ix.R == 1) break;
        for (uint64_t w = 0; w < len; w += 64) {
            const bool valid = w + lane < len;
            const uint64_t x = valid ? terms[beg + w + lane] : 0;
            Window wv;
            wv.canon = ix.opaque ? x : canonical(x);
            wv.valid = valid;
            const uint64_t nv = (uint64_t)__popcll(__ballot(valid));
            bool alive;
            if (pass == 0) {
                alive = probe_group<SEG, G, 0, 1>(ix, step_params(ix), wv, valid, lane, M);
                issued += nv;
            } else {
                alive = probe_group<SEG, G, 1, 4>(ix, step_params(ix), wv, valid, lane, M);
                issued += nv * (min(ix.R, 5u) - 1);
                if ((int)ix.R > 5 && (alive || !opt.early_exit)) {
                    alive &= probe_group<SEG, G, 5, MAXR - 5>(ix, step_params(ix), wv, valid, lane, M);
                    issued += nv * (ix.R - 5);
                }
            }
            if (opt.early_exit && !alive) {
                ended = true;
                break;
            }
        }
    }
    if (opt.probes && lane == 0 && issued) atomicAdd(opt.probes, (unsigned long long)(issued * ix.eta));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (masks_some_rep_empty(ix, M, lane)) {
        write_zeros(o, ix.W, lane);
        return;
    }
    resolve(ix, M, res, o, lane, opt.rmode);
}

static constexpr uint32_t kMaxLds = 64 * 1024;

int launch_query_kmers(rambo_s *h, const uint64_t *kmers, uint64_t n, uint64_t *out, hipStream_t s) {
    const Index ix = make_index(h);
    const int seg = default_seg(h->RW), G = (int)h->RW / seg;
    const int KPW = 64 / G, WPB = 4;
    const uint32_t mwords = ((KPW * h->R * h->RW) + 1) & ~1u;
    int use_res = 1;
    size_t lds = (size_t)WPB * (mwords + 2 * h->W) * 4;
    if (lds > kMaxLds) {
        use_res = 0;
        lds = (size_t)WPB * mwords * 4;
    }
    const uint64_t waves = (n + KPW - 1) / KPW;
    const uint64_t blocks = (waves + WPB - 1) / WPB;
    if (blocks > 0x7FFFFFFFULL) return fail(RAMBO_EINVAL, "rambo_query_kmers: batch too large");
#define RAMBO_SPLIT_BODY_                                                                                  \
    hipLaunchKernelGGL((k_query_kmers<SEG, G>), dim3((unsigned)blocks), dim3(64 * WPB), lds, s, ix, kmers, n, out, \
                       h->d_invalid, h->resolve, use_res)
    RAMBO_DISPATCH_SPLIT(seg, G)
#undef RAMBO_SPLIT_BODY_
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

int launch_query_seqs_plain(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out,
                            hipStream_t s, int seg, const InputHdr *hdr, unsigned long long *counts, uint64_t *wm) {
    // with hdr, the batch is read on the device and n is only its capacity
    const Index ix = make_index(h);
    const int G = (int)h->RW / seg;
    const int WPB = 4;
    const int sched = h->tune.sched;  // (this form scouts inside its kernel)
    const bool stage = sched == SCHED_SCOUT;
    const int use_res = seq_lds_result(h->W) ? 1 : 0;
    const size_t lds = (size_t)WPB * wave_lds(h->R * h->RW, h->W, use_res != 0, stage).total * 4;
    const uint64_t blocks = (n + WPB - 1) / WPB;
    if (blocks > 0x7FFFFFFFULL) return fail(RAMBO_EINVAL, "rambo_query_seqs: batch too large");
    // id-list mode counts queries without a term in the word after the n
    // answer sizes (the caller zeroes it), bitset mode in the handle
    QueryOpts opt{h->resolve, h->early_exit, h->probe_counter, sched, counts, counts ? counts + n : h->d_emptyq,
                  h->sparse_counter, counts ? wm : nullptr};
    // the RAMBO+ tallies have a kernel of their own (measurement only)
#define RAMBO_SPLIT_BODY_                                                                                  \
    if (opt.rplus)                                                                                         \
        hipLaunchKernelGGL((k_query_seqs_plain<SEG, G, true>), dim3((unsigned)blocks), dim3(64 * WPB), lds, s, ix,  \
                           seqs, offs, n, hdr, out, opt, use_res);                                          \
    else                                                                                                   \
        hipLaunchKernelGGL((k_query_seqs_plain<SEG, G, false>), dim3((unsigned)blocks), dim3(64 * WPB), lds, s, ix, \
                           seqs, offs, n, hdr, out, opt, use_res)
    RAMBO_DISPATCH_SPLIT(seg, G)
#undef RAMBO_SPLIT_BODY_
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

int launch_query_termsets(rambo_s *h, const uint64_t *terms, const uint64_t *offs, uint64_t n, uint64_t *out,
                          hipStream_t s) {
    const Index ix = make_index(h);
    const int seg = default_seg(h->RW), G = (int)h->RW / seg;
    const int WPB = 4;
    int use_res = 1;
    size_t lds = (size_t)WPB * wave_lds(h->R * h->RW, h->W, true, false).total * 4;
    if (lds > kMaxLds) {
        use_res = 0;
        lds = (size_t)WPB * wave_lds(h->R * h->RW, h->W, false, false).total * 4;
    }
    const uint64_t blocks = (n + WPB - 1) / WPB;
    if (blocks > 0x7FFFFFFFULL) return fail(RAMBO_EINVAL, "rambo_query_term_sets: batch too large");
    QueryOpts opt{h->resolve, h->early_exit, h->probe_counter, SCHED_SWEEP, nullptr, h->d_emptyq};
#define RAMBO_SPLIT_BODY_                                                                                  \
    hipLaunchKernelGGL((k_query_termsets<SEG, G>), dim3((unsigned)blocks), dim3(64 * WPB), lds, s, ix, terms, offs, \
                       n, out, opt, use_res, h->d_invalid)
    RAMBO_DISPATCH_SPLIT(seg, G)
#undef RAMBO_SPLIT_BODY_
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

// -------------------------------------------------------------------------
// bitsets -> ascending id lists
// -------------------------------------------------------------------------
// One wave per 64 reads: the reads with ids (a few per cent in id-list
// workloads) are found with one ballot and compacted one after the other by
// the whole wave; empty answers cost nothing more. A row is read 64 words at
// a time (one coalesced load), eight such loads in flight together; each
// 64-word chunk is placed by a prefix sum of its words' id counts. The total
// (off[n]) is checked here: over cap, nothing is written and the host reports
// the shortfall after the pass.
__global__ __launch_bounds__(256) void k_compact(const uint64_t *__restrict__ bits, uint64_t n, uint32_t W,
                                                 const uint64_t *__restrict__ off, uint32_t *__restrict__ ids,
                                                 uint64_t cap) {
    constexpr uint32_t U = 8;  // chunks in flight
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t i0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64;
    if (i0 >= n || off[n] > cap) return;
    const uint64_t mine = i0 + lane;
    uint64_t todo = __ballot(mine < n && off[mine + 1] != off[mine]);
    while (todo) {
        const uint64_t i = i0 + (uint64_t)__builtin_ctzll(todo);
        todo &= todo - 1;
        const uint64_t *row = bits + i * W;
        uint64_t base = off[i];
        for (uint32_t c0 = 0; c0 < W; c0 += 64 * U) {
            uint64_t word[U];
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint32_t w = c0 + 64 * u + lane;
                word[u] = w < W ? row[w] : 0;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint32_t w = c0 + 64 * u + lane;
                const uint32_t pc = (uint32_t)__popcll(word[u]);
                uint32_t incl = pc;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t v = __shfl_up(incl, d);
                    if ((int)lane >= d) incl += v;
                }
                uint64_t pos = base + incl - pc;
                uint64_t x = word[u];
                while (x) {
                    ids[pos++] = w * 64 + (uint32_t)__builtin_ctzll(x);
                    x &= x - 1;
                }
                base += __shfl(incl, 63);
            }
        }
    }
}

// As k_compact, reading only the words the query marked non-zero in wm
// ((W + 63) / 64 words per read): per mark word, the lanes take its 64
// bitset words, load the marked ones, and number their ids by a prefix sum,
// mark words in order, so each read's ids come out ascending.
__global__ __launch_bounds__(256) void k_compact_marked(const uint64_t *__restrict__ bits,
                                                        const uint64_t *__restrict__ wm, uint64_t n, uint32_t W,
                                                        const uint64_t *__restrict__ off, uint32_t *__restrict__ ids,
                                                        uint64_t cap) {
    const uint32_t lane = threadIdx.x & 63, WM = (W + 63) / 64;
    const uint64_t i0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64;
    if (i0 >= n || off[n] > cap) return;
    const uint64_t mine = i0 + lane;
    uint64_t todo = __ballot(mine < n && off[mine + 1] != off[mine]);
    while (todo) {
        const uint64_t i = i0 + (uint64_t)__builtin_ctzll(todo);
        todo &= todo - 1;
        const uint64_t *row = bits + i * W, *marks = wm + i * WM;
        uint64_t base = off[i];
        for (uint32_t m0 = 0; m0 < WM; m0 += 64) {
            const uint64_t mw = m0 + lane < WM ? marks[m0 + lane] : 0;
            uint64_t src = __ballot(mw != 0);
            while (src) {
                const uint32_t j = (uint32_t)__builtin_ctzll(src);
                src &= src - 1;
                // (readlane returns a signed int: widen through uint32_t)
                const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(mw >> 32), (int)j) << 32) |
                                   (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mw, (int)j);
                const uint32_t w = (m0 + j) * 64 + lane;
                const uint64_t v = (((m >> lane) & 1) && w < W) ? row[w] : 0;
                const uint32_t pc = (uint32_t)__popcll(v);
                uint32_t incl = pc;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t t = __shfl_up(incl, d);
                    if ((int)lane >= d) incl += t;
                }
                uint64_t pos = base + incl - pc;
                uint64_t x = v;
                while (x) {
                    ids[pos++] = w * 64 + (uint32_t)__builtin_ctzll(x);
                    x &= x - 1;
                }
                base += __shfl(incl, 63);
            }
        }
    }
}

__global__ void k_store_u64(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0) *p = v;
}

uint64_t ids_aux_words(uint64_t n) { return scan_parts_needed(n) + 1; }

int launch_ids(rambo_s *h, const uint64_t *bits, uint64_t n, uint32_t *ids, uint64_t *id_off, uint64_t ids_cap,
               hipStream_t s, const unsigned long long *counts, uint64_t *aux, const uint64_t *wm) {
    const uint32_t W = (uint32_t)h->W;
    uint64_t total = 0;
    if (n == 0) {
        HIP_CHECK(hipMemsetAsync(id_off, 0, 8, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return RAMBO_OK;
    }
    uint64_t *parts = aux, *d_n = aux + scan_parts_needed(n);
    hipLaunchKernelGGL(k_store_u64, dim3(1), dim3(64), 0, s, d_n, n);
    HIP_CHECK(hipGetLastError());
    int sst = launch_exclusive_scan(reinterpret_cast<const uint64_t *>(counts), d_n, n, id_off, parts, s);
    if (sst != RAMBO_OK) return sst;
    // the compaction checks the total against ids_cap itself: no round trip
    // to the host before it
    if (ids) {
        const uint64_t waves = (n + 63) / 64;
        if (wm)
            hipLaunchKernelGGL(k_compact_marked, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, bits, wm, n, W,
                               id_off, ids, ids_cap);
        else
            hipLaunchKernelGGL(k_compact, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, bits, n, W, id_off,
                               ids, ids_cap);
        HIP_CHECK(hipGetLastError());
    }
    unsigned long long noterm = 0;
    hipError_t e = hipMemcpyAsync(&total, id_off + n, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && counts) e = hipMemcpyAsync(&noterm, counts + n, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(RAMBO_EDEVICE, "rambo_query_seqs_ids: %s", hipGetErrorString(e));
    if (total > ids_cap)
        return fail(RAMBO_ETRUNC, "rambo_query_seqs_ids: %llu ids do not fit %llu", (unsigned long long)total,
                    (unsigned long long)ids_cap);
    if (total > 0 && !ids) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids: null ids");
    return noterm ? RAMBO_OK_EMPTYQ : RAMBO_OK;
}

int launch_store_u64(uint64_t *p, uint64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_store_u64, dim3(1), dim3(64), 0, s, p, v);
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

}  // namespace rambo
