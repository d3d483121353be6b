// Batched sequence queries: a scout pass over every read (scout schedule),
// then one persistent launch over a work queue of (read, tile of windows)
// items of the reads still alive, replayed from captured HIP graphs, with a
// launch shape chosen by an autotuner.
//
// Most reads end on their scout windows (Section 3.3.1: once a term has
// emptied the running intersection, no later term can bring a document
// back); the scout pass answers them and leaves them out of the queue.
// The queue runs longest work first (see the order below). A read that fits
// one tile is finished by the wave that took it, from its LDS masks. Longer
// reads are spread over many waves; their tiles AND into a per-read mask in
// global memory (AND is associative and commutative, so the order does not
// matter), a tile whose read is already dead skips its probes, and the wave
// that finishes a read's last tile resolves it.
//
// The batch size lives in device memory, so one captured graph serves any
// batch up to its capacity (the serving loop's slots rely on this).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <type_traits>

#include "batch.h"
#include "scan.h"

namespace rambo {

// Queue order of the persistent kernel, longest work first so that the last
// items to start are short. Class c holds the reads whose first tile has
// [c, c+1) quarters of a tile of windows (class 3 up to a full tile, which
// includes every multi-tile read). Order: class 3 first tiles, then every
// extra tile (tiles 1.. of multi-tile reads; after their read's first tile,
// which may empty the read's masks and let them skip), then classes 2, 1, 0.
// (the four class counters are 128 bytes apart: their atomics use different
// cache lines)
__global__ void k_batch_reset(BatchBufs bb) {
    if (threadIdx.x == 0) *bb.head = 0;
    if (threadIdx.x < 4) bb.cls[16 * threadIdx.x] = 0;
}

// With a scout pass before it (prescout), reads that pass ended are
// answered already and left out of the queue, and a multi-tile read's
// running mask starts from its scout AND in repetition 0.
// Each thread takes kPrepReads reads (256 apart), so a workgroup makes one
// atomic per size class for 256 x kPrepReads reads: same-address atomics
// serialise, and one per 256 reads made the pass over 10^6 reads wait on them
// (52 -> 23 us with 4); small batches keep one read per thread (100,000
// reads: 9 us with 1, 19 us with 4, where fewer workgroups wait longer).
template <uint32_t kPrepReads>
__global__ __launch_bounds__(256) void k_batch_prep(const InputHdr *in, uint32_t mw, uint32_t rw, uint32_t tile,
                                                    BatchBufs bb, int prescout) {
    const uint64_t n = in->n;
    const uint64_t *__restrict__ offs = in->offs;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool real[kPrepReads];
    uint32_t cls[kPrepReads];
#pragma unroll
    for (uint32_t k = 0; k < kPrepReads; k++) {
        const uint64_t i = ((uint64_t)blockIdx.x * kPrepReads + k) * blockDim.x + threadIdx.x;
        real[k] = i < n;
        cls[k] = 0;
        if (real[k] && prescout && !(bb.live[i] & 1u)) {
            bb.extra[i] = 0;
            real[k] = false;
        } else if (real[k]) {
            const uint64_t beg = offs[i], end = offs[i + 1];
            const uint64_t nw = n_windows(beg, end > beg ? end : beg);
            const uint64_t tiles = nw ? (nw + tile - 1) / tile : 1;
            bb.extra[i] = tiles - 1;
            if (tiles > 1) {
                bb.done[i] = 0;
                for (uint32_t w = 0; w < mw; w++)
                    bb.rmask[i * mw + w] = (prescout && w < rw) ? bb.smask[i * rw + w] : 0xFFFFFFFFu;
            }
            cls[k] = (uint32_t)min<uint64_t>(3, min<uint64_t>(nw, tile) * 4 / tile);
        }
    }
    // slots in the class lists, in read order: ranks within the wave
    // (ballots), offsets of the earlier (read group, wave) pairs of the
    // workgroup (LDS), one atomic per class and workgroup
    __shared__ uint32_t wcount[kPrepReads][4][4];  // [read group][wave][class]
    __shared__ unsigned long long bbase[4];
    uint64_t mine[kPrepReads];
#pragma unroll
    for (uint32_t k = 0; k < kPrepReads; k++) {
        mine[k] = 0;
        for (uint32_t v = 0; v < 4; v++) {
            const uint64_t mask = __ballot(real[k] && cls[k] == v);
            if (cls[k] == v) mine[k] = mask;
            if (lane == 0) wcount[k][wave][v] = (uint32_t)__popcll(mask);
        }
    }
    __syncthreads();
    const uint32_t waves = blockDim.x >> 6;
    if (threadIdx.x < 4) {
        const uint32_t v = threadIdx.x;
        uint32_t tot = 0;
        for (uint32_t k = 0; k < kPrepReads; k++)
            for (uint32_t w = 0; w < waves; w++) tot += wcount[k][w][v];
        bbase[v] = tot ? atomicAdd(bb.cls + 16 * v, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kPrepReads; k++) {
        if (!real[k]) continue;
        const uint32_t c = cls[k];
        uint64_t slot = bbase[c] + __popcll(mine[k] & ((1ULL << lane) - 1));
        for (uint32_t kk = 0; kk < k; kk++)
            for (uint32_t w = 0; w < waves; w++) slot += wcount[kk][w][c];
        for (uint32_t w = 0; w < wave; w++) slot += wcount[k][w][c];
        const uint64_t i = ((uint64_t)blockIdx.x * kPrepReads + k) * blockDim.x + threadIdx.x;
        bb.order[(uint64_t)c * bb.cap + slot] = (uint32_t)i;
    }
}

// lanes per read in the scout pass
__host__ __device__ constexpr int scout_group(int G, bool narrow) {
    return (narrow && G >= 8) ? G : (16 * G < 64 ? 16 * G : 64);
}

// The scout pass's window arithmetic within one read (a read holds fewer
// than 2^32 bytes): windows, scout windows and scout positions as in
// n_windows, scout_count and scout_pos over the whole read, in 32 bits.
__device__ __forceinline__ uint32_t windows32(uint64_t beg, uint64_t end) {
    return end >= beg + 31 ? (uint32_t)(end - beg - 30) : 0u;
}
__device__ __forceinline__ uint32_t scout_count32(uint32_t nw) {
    return nw ? (nw + 30) / 31 + ((nw - 1) % 31 != 0 ? 1u : 0u) : 0u;
}
__device__ __forceinline__ uint32_t scout_pos32(uint32_t nw, uint32_t k) { return min(31u * k, nw - 1); }

// Scout pass of the batched form (SCHED_SCOUT), before the queue is
// built: repetition 0 on every read's scout windows (every 31st window and
// the last, which together cover every base of the read). A group of GS
// lanes takes one read at a time, GS / G windows per round (G lanes split a
// row, as in the main kernel), and ANDs the rounds' rows by lane exchanges.
// The AND is stored in smask[i], the starting repetition-0 mask of the read's
// items, and live[i] says whether it is non-empty. With early exit an empty
// AND ends the read here (Section 3.3.1): its answer (a zero bitset, or a
// zero answer size in id-list mode) is written now and the read never enters
// the queue.
//
// Most reads end after a round or two, so the pass is a chain of short
// dependent steps (offsets, window bytes, rows) per read. Each group walks
// its own reads (every stride-th one) independently of the other groups of
// its wave -- a group whose read ended starts the next at once -- and loads
// one round ahead: while a round's rows are in flight, the group also loads
// the bytes of its read's next round and of its next read's first round, and
// the offsets two reads ahead. A round then costs one memory round trip,
// whichever way the read goes. The grid is what fits on the device at once.
// NARROW (id-list mode, where an ended read costs no output) gives rows split
// over 8 or more lanes one window per round (a group of G lanes per read)
// instead of 8: the read ends at its first empty window, with no probes of
// the windows after it, and a wave holds as many rows in flight as with wider
// groups, as it walks 8 reads at once; with bitsets the wider groups write the
// zero bitsets faster.
// In id-list mode with split rows a wave keeps only 8 reads' rounds in
// flight and the pass waits on their round trips: 8 waves per SIMD instead of
// the 7 its 71 VGPRs allow (two values spilled to scratch) make it 12 % faster
// (K=101,000: 0.44 -> 0.39 ms).
template <int SEG, int G, int NARROW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((NARROW && G >= 8) ? 8 : 1))) void k_batch_scout(Index ix, const InputHdr *in, uint64_t *__restrict__ out,
                                                     BatchBufs bb, QueryOpts opt) {
    constexpr int GS = scout_group(G, NARROW != 0);  // lanes per read
    constexpr int SLOTS = GS / G;                   // windows per round
    const uint8_t *__restrict__ seqs = in->seqs;
    const uint64_t *__restrict__ offs = in->offs;
    const uint64_t n = in->n;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t sub = lane % GS, seg = sub % G, slot = sub / G;
    const uint64_t gmask = (GS >= 64) ? ~0ULL : (((1ULL << GS) - 1) << (lane - sub));  // the group's lanes
    constexpr uint32_t GPB = 256 / GS;  // groups per workgroup
    const uint64_t stride = (uint64_t)gridDim.x * GPB;
    __shared__ unsigned long long blk_issued;
    if (threadIdx.x == 0) blk_issued = 0;
    __syncthreads();
    uint64_t issued = 0;

    // the group's current read i, with the offsets of the next two at hand
    uint64_t i = (uint64_t)blockIdx.x * GPB + threadIdx.x / GS;
    // (offsets read as global memory, as the window bytes are: a generic
    // load would also count against the scalar-load counter, and each wait
    // for the hash parameters would wait for it; a read with end < beg has no
    // window, which n_windows gives without clamping)
    typedef const uint64_t __attribute__((address_space(1))) *goffs;
    auto bounds = [&](uint64_t r, uint64_t &b, uint64_t &e) {
        b = e = 0;
        if (r < n) {
            b = ((goffs)offs)[r];
            e = ((goffs)offs)[r + 1];
        }
    };
    uint64_t beg, end, nbeg, nend, nnbeg = 0, nnend = 0;
    bounds(i, beg, end);
    bounds(i + stride, nbeg, nend);
    bool need_offs = true;  // the offsets of read i + 2 stride are still to load
    uint32_t nw = windows32(beg, end), ns = scout_count32(nw);
    uint32_t k0 = 0;  // first scout window of the current round
    // A window's bytes are loaded and decoded by the P lanes that split its
    // rows (P = 1: each lane takes a whole window).
    constexpr int P = G >= 8 ? 8 : G;
    using Bytes = std::conditional_t<(P > 1), WinPart<P>, WinBytes>;
    auto load_win = [&](Bytes &b, const uint8_t *p) {
        if constexpr (P > 1) load_window_part<P>(b, p, seg % P);
        else load_window_bytes(b, p);
    };
    auto decode_win = [&](const Bytes &b) -> Window {
        if constexpr (P > 1) return decode_window_parts<P>(b, seg % P);
        else return decode_window(b);
    };
    Bytes cur{}, next_round{}, next_read{};
    bool next_read_loaded = false;
    if (i < n && slot < ns) load_win(cur, seqs + beg + scout_pos32(nw, slot));
    // repetition 0's hash functions (eta <= 2), held for the whole pass
    const HashRec h0 = hash_rec(ix.hp->h, 0), h1 = hash_rec(ix.hp->h, ix.eta >= 2 ? 1 : 0);
    Seg<SEG> acc;
#pragma unroll
    for (int s = 0; s < SEG; s++) acc.w[s] = 0xFFFFFFFFu;
    bool saw = false;  // some scout window of the read was valid (uniform over the group)
    // Every load a round issues has completed when the round ends (explicit
    // wait at its end): the loads ahead are issued first, then the round's
    // rows, and the wait for the rows covers them all. The compiler's waits
    // inside the loop then never hold a load ahead back.
    __builtin_amdgcn_s_waitcnt(0);
    for (;;) {
        const bool have = i < n;
        if (__ballot(have) == 0) break;
        // loads ahead: the offsets two reads on, the bytes of this read's
        // next round and of the next read's first round
        const bool more = have && k0 + SLOTS < ns;
        if (need_offs) {
            bounds(i + 2 * stride, nnbeg, nnend);
            need_offs = false;
        }
        if (more && k0 + SLOTS + slot < ns) load_win(next_round, seqs + beg + scout_pos32(nw, k0 + SLOTS + slot));
        if (!next_read_loaded && i + stride < n) {
            const uint32_t w2 = windows32(nbeg, nend);
            if (slot < scout_count32(w2)) load_win(next_read, seqs + nbeg + scout_pos32(w2, slot));
            next_read_loaded = true;
        }
        // this round (every lane decodes: the lanes of a window exchange parts)
        Window wv = decode_win(cur);
        wv.valid = wv.valid && have && k0 + slot < ns;
        Seg<SEG> cm[1];
#pragma unroll
        for (int s = 0; s < SEG; s++) cm[0].w[s] = 0xFFFFFFFFu;
        if (wv.valid) {
            if (ix.eta <= 2) {
                // both rows in flight together (with one hash function the
                // same row twice)
                const Seg<SEG> a = load_seg<SEG>(row_ptr(ix, 0, bloom_pos(h0, ix.m, wv.canon)) + seg * SEG);
                const Seg<SEG> b = load_seg<SEG>(row_ptr(ix, 0, bloom_pos(h1, ix.m, wv.canon)) + seg * SEG);
#pragma unroll
                for (int s = 0; s < SEG; s++) cm[0].w[s] = a.w[s] & b.w[s];
            } else {
                probe_reps<SEG, 0, 1>(ix, ix.hp->h, wv.canon, seg, cm);
            }
        }
        const uint64_t vb = __ballot(wv.valid && seg == 0);
        issued += (uint64_t)__popcll(vb);
        saw |= (vb & gmask) != 0;
        uint32_t o = 0;
#pragma unroll
        for (int s = 0; s < SEG; s++) {
            uint32_t v = cm[0].w[s];
#pragma unroll
            for (int d = G; d < GS; d <<= 1) v &= (uint32_t)__shfl_xor((int)v, d);
            acc.w[s] &= v;
            o |= acc.w[s];
        }
        const bool live = !opt.early_exit || (__ballot(o != 0) & gmask) != 0;
        if (have && live && more) {
            k0 += SLOTS;
            cur = next_round;
        } else if (have) {
            // read i is done: its scout AND, and the answer of an ended read
            if (slot == 0)
#pragma unroll
                for (int s = 0; s < SEG; s++) bb.smask[i * ix.RW + seg * SEG + s] = acc.w[s];
            if (sub == 0) bb.live[i] = (live ? 1u : 0u) | (saw ? 2u : 0u);
            if (!live) {
                if (opt.counts) {
                    if (sub == 0) opt.counts[i] = 0;
                } else {
                    for (uint32_t w = sub; w < ix.W; w += GS) out[i * ix.W + w] = 0;
                }
            }
            // on to the next read
            i += stride;
            beg = nbeg;
            end = nend;
            nbeg = nnbeg;
            nend = nnend;
            need_offs = true;
            nw = windows32(beg, end);
            ns = scout_count32(nw);
            k0 = 0;
            cur = next_read;
            next_read_loaded = false;
#pragma unroll
            for (int s = 0; s < SEG; s++) acc.w[s] = 0xFFFFFFFFu;
            saw = false;
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    // one counter update per workgroup (same-address atomics serialise)
    if (opt.probes) {
        if (lane == 0 && issued) atomicAdd(&blk_issued, (unsigned long long)issued);
        __syncthreads();
        if (threadIdx.x == 0 && blk_issued) atomicAdd(opt.probes, blk_issued * ix.eta);
    }
}

// largest i < n with off[i] <= u, by a 64-way search (one load per lane per round)
__device__ __forceinline__ uint64_t find_read(const uint64_t *off, uint64_t n, uint64_t u, uint32_t lane) {
    uint64_t lo = 0, hi = n;  // invariant: off[lo] <= u, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint64_t step = (hi - lo + 63) / 64;
        const uint64_t idx = lo + (uint64_t)lane * step;
        const bool pred = idx < hi && off[idx] <= u;
        const uint32_t k = (uint32_t)__popcll(__ballot(pred)) - 1;  // pred holds on a prefix of lanes
        lo = lo + (uint64_t)k * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// a wave-uniform value, kept in scalar registers
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t load_coherent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// some repetition of the read's global running mask is already empty
__device__ __forceinline__ bool read_dead(const Index &ix, const uint32_t *rm, uint32_t lane) {
    bool dead = false;
    for (uint32_t r = 0; r < ix.R; r++) {
        uint32_t o = 0;
        for (uint32_t w = lane; w < ix.RW; w += 64) o |= load_coherent(rm + r * ix.RW + w);
        dead |= __ballot(o != 0) == 0;
    }
    return dead;
}

// Rows split over G > 1 lanes: the compiler's default would take 172 VGPRs
// (2 waves per SIMD); 3 waves fit without spilling.
template <int SEG, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(G == 1 ? 1 : 3))) void k_batch_main(Index ix, const InputHdr *in, uint64_t *__restrict__ out,
                                                    BatchBufs bb, QueryOpts opt, int use_res, uint32_t tile,
                                                    uint32_t grab) {
    const uint8_t *__restrict__ seqs = in->seqs;
    const uint64_t *__restrict__ offs = in->offs;
    extern __shared__ __align__(16) uint64_t smem64[];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t mw = ix.R * ix.RW;
    // (no staging area: this form scouts in a pass of its own)
    const WaveLds L = wave_lds(mw, ix.W, use_res != 0, false);
    uint32_t *M = reinterpret_cast<uint32_t *>(smem64) + wave * L.total;
    uint64_t *res = use_res ? reinterpret_cast<uint64_t *>(M + L.res) : nullptr;
    uint8_t *stage = nullptr;

    const uint64_t n = in->n;
    const uint64_t n_extra = bb.extra_off[n];
    const uint64_t c3 = uniform64(bb.cls[48]), c2 = uniform64(bb.cls[32]), c1 = uniform64(bb.cls[16]);
    const uint64_t total = c3 + c2 + c1 + uniform64(bb.cls[0]) + n_extra;  // queued reads and extra tiles
    uint64_t issued = 0;
    for (;;) {
        uint64_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(bb.head, (unsigned long long)grab);
        t0 = uniform64(__shfl(t0, 0));
        if (t0 >= total) break;
        const uint64_t t1 = min(total, t0 + grab);
        for (uint64_t t = t0; t < t1; t++) {
            uint64_t i, c = 0;
            if (t >= c3 && t < c3 + n_extra) {
                const uint64_t u = t - c3;
                i = uniform64(find_read(bb.extra_off, n, u, lane));
                c = uniform64(1 + (u - bb.extra_off[i]));
            } else {
                uint64_t u = t, v = 3;
                if (u >= c3) {
                    u -= c3 + n_extra;
                    v = 2;
                    if (u >= c2) { u -= c2; v = 1; }
                    if (v == 1 && u >= c1) { u -= c1; v = 0; }
                }
                i = uniform64(bb.order[v * bb.cap + u]);
            }
            const uint64_t beg = uniform64(offs[i]);
            uint64_t end = uniform64(offs[i + 1]);
            if (end < beg) end = beg;
            const uint64_t nwin = n_windows(beg, end);
            const uint64_t ntiles = nwin ? (nwin + tile - 1) / tile : 1;
            uint32_t *rm = bb.rmask + i * mw;
            uint64_t *o = out + i * ix.W;

            // another tile of the read may have emptied its masks already
            const bool skip = ntiles > 1 && opt.early_exit && read_dead(ix, rm, lane);
            init_masks(ix, M, lane);
            if (opt.sched == SCHED_PRESCOUT && ntiles == 1)
                for (uint32_t w = lane; w < ix.RW; w += 64) M[w] = bb.smask[i * ix.RW + w];
            uint64_t got = 0;  // probes this item issued (0: no valid window in it)
            if (!skip) {
                const uint64_t w_hi = min(nwin, (c + 1) * (uint64_t)tile);
                got = probe_windows<SEG, G>(ix, seqs, beg, end, c * (uint64_t)tile, w_hi, lane, M,
                                            opt.early_exit != 0, opt.sched, stage);
                issued += got;
            }
            // a scout window of the read was valid (it was probed by the scout pass)
            const bool scout_saw = opt.sched == SCHED_PRESCOUT && (bb.live[i] & 2u);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (ntiles == 1) {
                // the whole read was in this tile: resolve from its masks
                if (got == 0 && !scout_saw && lane == 0) atomicAdd(opt.emptyq, 1ULL);
                answer_read(ix, M, res, o, lane, opt.rmode, opt.counts, i, opt.wm);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            // Publish this tile's masks, then count the tile done. Every
            // access to rm and done is an agent-scope atomic read-modify-write,
            // performed at the device's point of coherence (one for all XCDs),
            // and a returning RMW's old value comes back only once the RMW has
            // been performed there. The ANDs return their old values, the
            // wave folds them into one value (a ballot over every lane's
            // results) and the count's operand is made to depend on it, so
            // the count is issued only after each of this tile's ANDs has
            // been performed. The last tile issues its mask reads only after
            // its own count has returned, i.e. after every other tile's count
            // and hence after every other tile's ANDs. (A release fence at
            // agent scope would also order them, but on a multi-XCD device it
            // writes back the XCD's whole L2, which made small tiles 4.5x
            // slower; nothing here needs it, as no plain store is published.)
            uint32_t olds = 0;
            if (!skip) {
                for (uint32_t w = lane; w < mw; w += 64) {
                    const uint32_t v = M[w];
                    if (v != 0xFFFFFFFFu)
                        olds |= __hip_atomic_fetch_and(rm + w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            // (a skipped tile belongs to a read whose answer is empty anyway:
            // it counts as holding a valid window)
            const unsigned long long inc = 1ull + ((got > 0 || skip) ? (1ull << 32) : 0ull);
            const uint32_t zero = opaque_zero(__ballot(olds != 0));
            unsigned long long prev = 0;
            if (lane == 0)
                prev = __hip_atomic_fetch_add(bb.done + i, inc + zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            prev = uniform64(__shfl(prev, 0));
            if ((prev & 0xFFFFFFFFull) + 1 == ntiles) {
                if ((prev >> 32) + (inc >> 32) == 0 && !scout_saw && lane == 0) atomicAdd(opt.emptyq, 1ULL);
                // last tile of read i: read the masks with atomic RMWs too,
                // at the same point of coherence as the ANDs
                for (uint32_t w = lane; w < mw; w += 64)
                    M[w] = __hip_atomic_fetch_or(rm + w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                answer_read(ix, M, res, o, lane, opt.rmode, opt.counts, i, opt.wm);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    if (opt.probes && lane == 0 && issued) atomicAdd(opt.probes, (unsigned long long)(issued * ix.eta));
}


static int enqueue_prep(rambo_s *h, const Tune &tu, BatchGraph &bg, uint64_t *out, unsigned long long *counts,
                        hipStream_t s) {
    const uint32_t mw = h->R * h->RW;
    const bool pre = tu.sched == SCHED_SCOUT;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, bg.bb);
    HIP_CHECK(hipGetLastError());
    if (pre) {
        const Index ix = make_index(h);
        const int G = (int)h->RW / tu.seg;
        // a grid of what fits on the device at once strides over the reads
        const bool narrow = counts != nullptr;
        const uint64_t GS = (uint64_t)scout_group(G, narrow);
        int fit = 0;
#define RAMBO_SPLIT_BODY_                                                                                    \
    HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                  \
        &fit, narrow ? k_batch_scout<SEG, G, 1> : k_batch_scout<SEG, G, 0>, 256, 0))
        RAMBO_DISPATCH_SPLIT(tu.seg, G)
#undef RAMBO_SPLIT_BODY_
        const uint64_t blocks = std::max<uint64_t>(
            1, std::min<uint64_t>((bg.cap * GS + 255) / 256, (uint64_t)std::max(1, fit) * h->n_cu));
        QueryOpts opt{h->resolve, h->early_exit, h->probe_counter, tu.sched, counts,
                      counts ? counts + bg.cap : h->d_emptyq};
#define RAMBO_SPLIT_BODY_                                                                                   \
    if (narrow)                                                                                             \
        hipLaunchKernelGGL((k_batch_scout<SEG, G, 1>), dim3((unsigned)blocks), dim3(256), 0, s, ix, bg.in, out,   \
                           bg.bb, opt);                                                                      \
    else                                                                                                     \
        hipLaunchKernelGGL((k_batch_scout<SEG, G, 0>), dim3((unsigned)blocks), dim3(256), 0, s, ix, bg.in, out,   \
                           bg.bb, opt)
        RAMBO_DISPATCH_SPLIT(tu.seg, G)
#undef RAMBO_SPLIT_BODY_
        HIP_CHECK(hipGetLastError());
    }
    // four reads per thread once one per thread would take over eight
    // workgroups per compute unit
    if ((bg.cap + 255) / 256 > 8 * (uint64_t)h->n_cu)
        hipLaunchKernelGGL(k_batch_prep<4>, dim3((unsigned)((bg.cap + 1023) / 1024)), dim3(256), 0, s, bg.in, mw,
                           h->RW, (uint32_t)tu.tile, bg.bb, pre ? 1 : 0);
    else
        hipLaunchKernelGGL(k_batch_prep<1>, dim3((unsigned)((bg.cap + 255) / 256)), dim3(256), 0, s, bg.in, mw,
                           h->RW, (uint32_t)tu.tile, bg.bb, pre ? 1 : 0);
    HIP_CHECK(hipGetLastError());
    // the header's first field is n
    return launch_exclusive_scan(bg.bb.extra, &bg.in->n, bg.cap, bg.bb.extra_off, bg.parts, s);
}

static int enqueue_main(rambo_s *h, const Tune &tu, BatchGraph &bg, uint64_t *out, hipStream_t s,
                        unsigned long long *counts, uint64_t *wm) {
    const Index ix = make_index(h);
    const uint32_t mw = h->R * h->RW;
    const int G = (int)h->RW / tu.seg;
    const int use_res = seq_lds_result(h->W) ? 1 : 0;
    const size_t lds = (size_t)tu.wpb * wave_lds(mw, h->W, use_res != 0, false).total * 4;
    // the scout schedule has run its scout windows in the scout pass already
    const int ksched = tu.sched == SCHED_SCOUT ? SCHED_PRESCOUT : tu.sched;
    QueryOpts opt{h->resolve, h->early_exit, h->probe_counter, ksched, counts, counts ? counts + bg.cap : h->d_emptyq,
                  nullptr, counts ? wm : nullptr};
    // a persistent grid must be resident: never more workgroups than fit
#define RAMBO_SPLIT_BODY_                                                                                  \
    {                                                                                                      \
        int fit = 0;                                                                                       \
        HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, k_batch_main<SEG, G>, 64 * tu.wpb, lds)); \
        const int per_cu = std::max(1, std::min(fit, tu.waves_per_cu / tu.wpb));                         \
        bg.blocks = (unsigned)(h->n_cu * per_cu);                                                          \
        hipLaunchKernelGGL((k_batch_main<SEG, G>), dim3(bg.blocks), dim3(64 * tu.wpb), lds, s, ix, bg.in, out,  \
                           bg.bb, opt, use_res, (uint32_t)tu.tile, (uint32_t)tu.grab);                     \
    }
    RAMBO_DISPATCH_SPLIT(tu.seg, G)
#undef RAMBO_SPLIT_BODY_
    HIP_CHECK(hipGetLastError());
    return RAMBO_OK;
}

BatchGraph::~BatchGraph() {
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (exec_prep) (void)hipGraphExecDestroy(exec_prep);
    if (exec_main) (void)hipGraphExecDestroy(exec_main);
    if (graph_prep) (void)hipGraphDestroy(graph_prep);
    if (graph_main) (void)hipGraphDestroy(graph_main);
    if (mem) (void)hipFree(mem);
}

static int capture(rambo_s *h, hipGraph_t *g, hipGraphExec_t *exec, const std::function<int(hipStream_t)> &body) {
    HIP_CHECK(hipStreamBeginCapture(h->aux, hipStreamCaptureModeThreadLocal));
    int st = body(h->aux);
    hipGraph_t gg = nullptr;
    hipError_t e = hipStreamEndCapture(h->aux, &gg);
    if (st != RAMBO_OK) {
        if (gg) (void)hipGraphDestroy(gg);
        return st;
    }
    if (e != hipSuccess) return fail(RAMBO_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    *g = gg;
    HIP_CHECK(hipGraphInstantiate(exec, gg, nullptr, nullptr, 0));
    return RAMBO_OK;
}

// Graph state and, without an external header, an owned one set to *init.
static int alloc_graph_state(rambo_s *h, BatchGraph &bg, uint64_t cap, bool batch_bufs, const InputHdr *in_dev,
                             const InputHdr *init) {
    const size_t mw = (size_t)h->R * h->RW;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t b_mask = 0, b_done = 0, b_extra = 0, b_off = 0, b_parts = 0, b_order = 0, b_smask = 0, b_live = 0;
    if (batch_bufs) {
        b_smask = al(cap * h->RW * 4);
        b_live = al(cap * 4);
        b_mask = al(cap * mw * 4);
        b_done = al(cap * 8);
        b_extra = al(cap * 8);
        b_off = al((cap + 1) * 8);
        b_parts = al(scan_parts_needed(cap) * 8);
        b_order = al(4 * cap * 4);
    }
    HIP_CHECK(hipMalloc(&bg.mem, b_mask + b_done + b_extra + b_off + b_parts + b_order + b_smask + b_live + 640 + 256));
    char *p = (char *)bg.mem;
    bg.bb.smask = b_smask ? (uint32_t *)p : nullptr; p += b_smask;
    bg.bb.live = b_live ? (uint32_t *)p : nullptr; p += b_live;
    bg.parts = (uint64_t *)p; p += b_parts;
    bg.bb.rmask = (uint32_t *)p; p += b_mask;
    bg.bb.done = (unsigned long long *)p; p += b_done;
    bg.bb.extra = (uint64_t *)p; p += b_extra;
    bg.bb.extra_off = (uint64_t *)p; p += b_off;
    bg.bb.order = (uint32_t *)p; p += b_order;
    bg.bb.head = (unsigned long long *)p;  // its own 128-byte line (every wave's queue atomic)
    bg.bb.cls = bg.bb.head + 16;           // class v at cls[16 v]: the next four lines
    p += 640;
    bg.bb.cap = cap;
    if (in_dev) {
        bg.in = in_dev;
    } else {
        InputHdr *own = (InputHdr *)p;
        HIP_CHECK(hipMemcpy(own, init, sizeof(InputHdr), hipMemcpyHostToDevice));
        bg.in = own;
    }
    // graphs of the query entry point are timed (rambo_last_batch_ms); the
    // server's are not (three fewer operations per batch)
    bg.timed = in_dev == nullptr;
    if (bg.timed)
        for (auto &e : bg.ev) HIP_CHECK(hipEventCreate(&e));
    return RAMBO_OK;
}

int make_batch_graph(rambo_s *h, const Tune &tu, const InputHdr *in_dev, const InputHdr *init, uint64_t cap,
                     uint64_t *out, std::shared_ptr<BatchGraph> &res, unsigned long long *counts, uint64_t *wm) {
    auto bg = std::make_shared<BatchGraph>();
    bg->cap = cap;
    bg->tune = tu;
    int st = alloc_graph_state(h, *bg, cap, true, in_dev, init);
    if (st == RAMBO_OK)
        st = capture(h, &bg->graph_prep, &bg->exec_prep,
                     [&](hipStream_t s) { return enqueue_prep(h, tu, *bg, out, counts, s); });
    if (st == RAMBO_OK)
        st = capture(h, &bg->graph_main, &bg->exec_main,
                     [&](hipStream_t s) { return enqueue_main(h, tu, *bg, out, s, counts, wm); });
    if (st != RAMBO_OK) return st;
    res = bg;
    return RAMBO_OK;
}

int make_plain_graph(rambo_s *h, const InputHdr *in_dev, uint64_t cap, uint64_t *out,
                     std::shared_ptr<BatchGraph> &res) {
    auto bg = std::make_shared<BatchGraph>();
    bg->cap = cap;
    int st = alloc_graph_state(h, *bg, cap, false, in_dev, nullptr);
    if (st == RAMBO_OK)
        st = capture(h, &bg->graph_main, &bg->exec_main, [&](hipStream_t s) {
            return launch_query_seqs_plain(h, nullptr, nullptr, cap, out, s, default_seg(h->RW), bg->in);
        });
    if (st != RAMBO_OK) return st;
    res = bg;
    return RAMBO_OK;
}

int launch_batch_graph(rambo_s *h, BatchGraph &bg, hipStream_t s) {
    (void)h;
    if (bg.timed) HIP_CHECK(hipEventRecord(bg.ev[0], s));
    if (bg.exec_prep) HIP_CHECK(hipGraphLaunch(bg.exec_prep, s));
    if (bg.timed) HIP_CHECK(hipEventRecord(bg.ev[1], s));
    HIP_CHECK(hipGraphLaunch(bg.exec_main, s));
    if (bg.timed) HIP_CHECK(hipEventRecord(bg.ev[2], s));
    return RAMBO_OK;
}

static std::string graph_key(const Tune &tu, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out,
                             const unsigned long long *counts, const uint64_t *wm) {
    char buf[320];
    snprintf(buf, sizeof buf, "%p/%p/%llu/%p/%p/%p/%d.%d.%d.%d.%d.%d", (const void *)seqs, (const void *)offs,
             (unsigned long long)n, (void *)out, (const void *)counts, (const void *)wm, tu.seg, tu.tile,
             tu.waves_per_cu, tu.wpb, tu.grab, tu.sched);
    return buf;
}

static int run_graph(rambo_s *h, const Tune &tu, const uint8_t *seqs, const uint64_t *offs, uint64_t n,
                     uint64_t *out, hipStream_t s, unsigned long long *counts = nullptr, uint64_t *wm = nullptr) {
    std::shared_ptr<BatchGraph> bg;
    std::lock_guard<std::mutex> g(h->mu);
    const std::string key = graph_key(tu, seqs, offs, n, out, counts, wm);
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        bg = it->second;
    } else {
        if (h->graphs.size() >= 16) h->graphs.clear();
        const InputHdr init{n, offs, seqs, 0};
        int st = make_batch_graph(h, tu, nullptr, &init, n, out, bg, counts, wm);
        if (st != RAMBO_OK) return st;
        h->graphs[key] = bg;
    }
    int st = launch_batch_graph(h, *bg, s);
    if (st == RAMBO_OK) h->last_graph = bg;
    return st;
}

void drop_graphs(rambo_s *h) {
    h->graphs.clear();
    h->last_graph.reset();
}

// ---------------------------------------------------------------------------
// autotuner: coordinate search over the launch shape on the caller's batch
// (every candidate computes the same bits), cached per index shape.
// ---------------------------------------------------------------------------
bool tune_valid(const rambo_s *h, const Tune &t) {
    return (t.seg == 1 || t.seg == 2 || t.seg == 4) && (int)h->RW % t.seg == 0 &&
           split_supported(t.seg, (int)h->RW / t.seg) && t.tile >= 64 && t.tile % 64 == 0 && t.tile <= (1 << 20) &&
           t.waves_per_cu >= 1 && t.waves_per_cu <= 64 && (t.wpb == 1 || t.wpb == 2 || t.wpb == 4) && t.grab >= 1 &&
           t.grab <= 64 && t.sched >= 0 && t.sched <= 2;
}

static std::string tune_key(const rambo_s *h) {
    hipDeviceProp_t prop;
    const char *arch = "gpu";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    char buf[256];
    snprintf(buf, sizeof buf, "%s K=%llu B=%u R=%u eta=%u m=%llu ee=%d", arch, (unsigned long long)h->K, h->B, h->R,
             h->eta, (unsigned long long)h->m, h->early_exit);
    std::string s = buf;
    for (auto &c : s)
        if (c == ':' || c == '|') c = '_';
    return s;
}

static bool tune_cache_load(rambo_s *h) {
    const char *path = getenv("RAMBO_TUNE_CACHE");
    if (!path) return false;
    std::ifstream f(path);
    std::string line, key = tune_key(h);
    while (std::getline(f, line)) {
        const size_t bar = line.find('|');
        if (bar == std::string::npos || line.substr(0, bar) != key) continue;
        Tune t;
        if (sscanf(line.c_str() + bar + 1, "%d %d %d %d %d %d", &t.seg, &t.tile, &t.waves_per_cu, &t.wpb, &t.grab,
                   &t.sched) == 6 &&
            tune_valid(h, t)) {
            h->tune = t;
            return true;
        }
    }
    return false;
}

static void tune_cache_store(const rambo_s *h) {
    const char *path = getenv("RAMBO_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << tune_key(h) << "|" << h->tune.seg << " " << h->tune.tile << " " << h->tune.waves_per_cu << " "
      << h->tune.wpb << " " << h->tune.grab << " " << h->tune.sched << "\n";
}

static int time_candidate(rambo_s *h, const Tune &tu, const uint8_t *seqs, const uint64_t *offs, uint64_t n,
                          uint64_t *out, hipStream_t s, float &best_ms) {
    hipEvent_t a, b;
    HIP_CHECK(hipEventCreate(&a));
    HIP_CHECK(hipEventCreate(&b));
    int st = run_graph(h, tu, seqs, offs, n, out, s);  // warm-up (and graph build)
    if (st == RAMBO_OK) st = run_graph(h, tu, seqs, offs, n, out, s);
    float best = 1e30f;
    for (int rep = 0; rep < 5 && st == RAMBO_OK; rep++) {
        (void)hipEventRecord(a, s);
        st = run_graph(h, tu, seqs, offs, n, out, s);
        (void)hipEventRecord(b, s);
        if (hipEventSynchronize(b) != hipSuccess) st = fail(RAMBO_EDEVICE, "autotune: run failed");
        float ms = 0;
        if (st == RAMBO_OK) {
            (void)hipEventElapsedTime(&ms, a, b);
            best = std::min(best, ms);
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    best_ms = best;
    return st;
}

int autotune(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out, hipStream_t s) {
    Tune best = h->tune;
    best.seg = default_seg(h->RW);
    float best_ms = 0;
    int st = time_candidate(h, best, seqs, offs, n, out, s, best_ms);
    if (st != RAMBO_OK) return st;
    const char *vb = getenv("RAMBO_TUNE_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    if (verbose)
        fprintf(stderr, "rambo autotune: seg=%d tile=%d waves/CU=%d wpb=%d grab=%d sched=%d -> %.3f ms (start)\n",
                best.seg, best.tile, best.waves_per_cu, best.wpb, best.grab, best.sched, best_ms);
    auto consider = [&](Tune t) -> int {
        if (!tune_valid(h, t)) return RAMBO_OK;
        float ms = 0;
        int st2 = time_candidate(h, t, seqs, offs, n, out, s, ms);
        if (st2 != RAMBO_OK) return st2;
        if (verbose)
            fprintf(stderr, "rambo autotune: seg=%d tile=%d waves/CU=%d wpb=%d grab=%d sched=%d -> %.3f ms\n", t.seg,
                    t.tile, t.waves_per_cu, t.wpb, t.grab, t.sched, ms);
        if (ms < best_ms * 0.98f) {
            best = t;
            best_ms = ms;
        }
        return RAMBO_OK;
    };
    // two rounds of coordinate search (the second revisits every axis from
    // the first round's shape); a candidate must beat the best by 2 %
    for (int round = 0; round < 2; round++) {
        for (int tile : {128, 256, 512, 1024, 2048, 4096}) {
            Tune t = best; t.tile = tile;
            if (t.tile != best.tile && (st = consider(t))) return st;
        }
        for (int wpc : {8, 12, 16, 20, 24, 32}) {
            Tune t = best; t.waves_per_cu = wpc;
            if (t.waves_per_cu != best.waves_per_cu && (st = consider(t))) return st;
        }
        for (int seg : {1, 2, 4}) { Tune t = best; t.seg = seg; if (t.seg != best.seg && (st = consider(t))) return st; }
        for (int grab : {1, 2, 4, 16}) {
            Tune t = best; t.grab = grab;
            if (t.grab != best.grab && (st = consider(t))) return st;
        }
        for (int wpb : {1, 2, 4}) { Tune t = best; t.wpb = wpb; if (t.wpb != best.wpb && (st = consider(t))) return st; }
        for (int sched : {0, 1, 2}) {
            Tune t = best; t.sched = sched;
            if (sched != best.sched && (st = consider(t))) return st;
        }
    }
    std::lock_guard<std::mutex> g(h->mu);
    h->tune = best;
    drop_graphs(h);  // keep only graphs of the chosen shape
    return RAMBO_OK;
}

int query_seqs_batched(rambo_s *h, const uint8_t *seqs, const uint64_t *offs, uint64_t n, uint64_t *out,
                       hipStream_t s, unsigned long long *counts, uint64_t *wm) {
    if (!h->tuned) {
        h->tune.seg = default_seg(h->RW);
        const char *mode = getenv("RAMBO_TUNE");
        const bool off = mode && !strcmp(mode, "off");
        if (!off && !tune_cache_load(h)) {
            int st = autotune(h, seqs, offs, n, out, s);
            if (st != RAMBO_OK) return st;
            tune_cache_store(h);
        }
        h->tuned = true;
    }
    Tune tu;
    {
        std::lock_guard<std::mutex> g(h->mu);
        tu = h->tune;
    }
    return run_graph(h, tu, seqs, offs, n, out, s, counts, wm);
}

}  // namespace rambo

using namespace rambo;

RAMBO_API int rambo_autotune(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n, uint64_t *out,
                             void *stream) {
    if (!h || !seqs || !offsets || !out || n == 0) return fail(RAMBO_EINVAL, "rambo_autotune: bad argument");
    int st = autotune(h, seqs, offsets, n, out, (hipStream_t)stream);
    if (st == RAMBO_OK) h->tuned = true;
    return st;
}

RAMBO_API int rambo_last_batch_ms(rambo_t *h, float *graph_ms, float *kernel_ms) {
    if (!h || !graph_ms || !kernel_ms) return fail(RAMBO_EINVAL, "rambo_last_batch_ms: null argument");
    std::shared_ptr<BatchGraph> bg;
    {
        std::lock_guard<std::mutex> g(h->mu);
        bg = h->last_graph;
    }
    if (!bg || !bg->timed) return fail(RAMBO_EINVAL, "rambo_last_batch_ms: no batched launch yet");
    HIP_CHECK(hipEventSynchronize(bg->ev[2]));
    HIP_CHECK(hipEventElapsedTime(graph_ms, bg->ev[0], bg->ev[2]));
    HIP_CHECK(hipEventElapsedTime(kernel_ms, bg->ev[1], bg->ev[2]));
    return RAMBO_OK;
}

RAMBO_API int rambo_get_tune(const rambo_t *h, rambo_tune_t *t) {
    if (!h || !t) return fail(RAMBO_EINVAL, "rambo_get_tune: null argument");
    t->seg = h->tune.seg;
    t->tile = h->tune.tile;
    t->waves_per_cu = h->tune.waves_per_cu;
    t->wpb = h->tune.wpb;
    t->grab = h->tune.grab;
    t->sched = h->tune.sched;
    t->tuned = h->tuned ? 1 : 0;
    return RAMBO_OK;
}

RAMBO_API int rambo_set_tune(rambo_t *h, const rambo_tune_t *t) {
    if (!h || !t) return fail(RAMBO_EINVAL, "rambo_set_tune: null argument");
    Tune tu;
    tu.seg = t->seg;
    tu.tile = t->tile;
    tu.waves_per_cu = t->waves_per_cu;
    tu.wpb = t->wpb;
    tu.grab = t->grab;
    tu.sched = t->sched;
    if (!tune_valid(h, tu)) return fail(RAMBO_EINVAL, "rambo_set_tune: launch shape out of range");
    std::lock_guard<std::mutex> g(h->mu);
    h->tune = tu;
    h->tuned = true;
    drop_graphs(h);
    return RAMBO_OK;
}
