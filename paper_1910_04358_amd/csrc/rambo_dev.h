// Device-side building blocks of the RAMBO hot path for gfx950 (wave64).
//
// Index layout in HBM ("bit-sliced"): rows[r][p][RW] uint32, r < R, p < m.
// Row (r, p) holds bit p of every BFU of repetition r: BFU(r, b) is bit
// (b & 31) of word (b >> 5). A Bloom probe of all B BFUs of a repetition at
// position p (Section 3.3: test every BFU of the table) is therefore ONE
// contiguous row read of RW * 4 bytes, and an insertion (Algorithm 1) is one
// atomic OR of a single bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rambo {

constexpr int MAXR = 8;
constexpr int MAXETA = 16;
constexpr uint64_t MASK62 = (1ULL << 62) - 1;

// Bloom hash parameters h_{r,j} (A = ahi:alo, C = chi:clo), index
// r * eta + j; one 32-byte record per hash function (one scalar load).
struct HashRec {
    uint64_t alo, ahi, clo, chi;
};
struct HashParams {
    HashRec h[MAXR * MAXETA];
};

// Everything a kernel needs to address the index (passed by value).
struct Index {
    uint32_t *rows;          // [R][m][RW]
    const HashParams *hp;    // device
    const uint4 *cells;      // [K]      phi_r(d) at 16-bit slot r of record d
    const uint32_t *boff;    // [R][B+1] cell offsets into bdoc
    const uint32_t *bdoc;    // [R][K]   documents grouped by cell, ascending
    const uint4 *cells0;     // [K]      the cell record of bdoc[k] for k < K (repetition 0's grouping)
    uint64_t m;
    uint64_t K;
    uint32_t B, R, eta, RW;  // RW = 32-bit words per row (power of two)
    uint32_t log2RW, W;      // W = result words per query
    uint32_t opaque;         // terms are opaque 64-bit values (no k-mer encoding)
};

// phi_r(d) from document d's cell record
__device__ __forceinline__ uint32_t cell_at(const uint4 &c, int r) {
    const uint32_t w = r < 2 ? c.x : r < 4 ? c.y : r < 6 ? c.z : c.w;
    return (r & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// A batch of reads described in device memory, so that one captured graph
// can serve batches of any size and placement: read i is
// seqs[offs[i] .. offs[i+1]), i < n. n comes first (scans read it alone).
struct InputHdr {
    uint64_t n;
    const uint64_t *offs;
    const uint8_t *seqs;
    uint64_t pad;
};

// Per-wave LDS area of the sequence query kernels, in 32-bit words: the
// running masks (R * RW words, rounded to 16 bytes), the candidate bitset
// (W 64-bit words, rounded to 16 bytes) when use_res, and the byte staging
// area of the scout schedule when stage. Host and device use this one layout.
constexpr uint32_t kStageWords = 528;  // 2112 bytes: 64 windows 31 apart, +30, +alignment
struct WaveLds {
    uint32_t masks, res, stage, total;  // word offsets and size
};
// Whether a sequence-query kernel keeps the candidate resolve's bitset in
// LDS: only for small W. Its 2 W words per wave would otherwise limit the
// waves a compute unit holds (K = 101,000: 12.6 KB per wave, 8 waves per
// CU); without it the candidate resolve writes the output row directly,
// which is slower than the LDS bitset where LDS is plentiful.
__host__ __device__ inline bool seq_lds_result(uint64_t W) { return W <= 512; }

__host__ __device__ inline WaveLds wave_lds(uint32_t mask_words, uint64_t W, bool use_res, bool stage) {
    WaveLds l;
    l.masks = 0;
    l.res = (mask_words + 3u) & ~3u;
    const uint32_t resw = use_res ? (uint32_t)((2 * W + 3) & ~3ull) : 0u;
    l.stage = l.res + resw;
    l.total = l.stage + (stage ? kStageWords : 0u);
    return l;
}

// ---------------------------------------------------------------------------
// Hashing: h_{r,j}(x) = floor(m * hi64((A x + C) mod 2^128) / 2^64)
// (multiply-add-shift, strongly universal for 62-bit keys; range reduced by
// a multiply-high, which is the plain top-bits shift when m = 2^t).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t bloom_pos(const HashRec &p, uint64_t m, uint64_t x) {
    const uint64_t alo = p.alo, ahi = p.ahi, clo = p.clo, chi = p.chi;
    const uint64_t lo = alo * x;
    uint64_t hi = __umul64hi(alo, x) + ahi * x;
    const uint64_t lo2 = lo + clo;
    hi += chi + (lo2 < lo ? 1 : 0);
    return __umul64hi(hi, m);
}

// Hash function i of the table at hp, read through the constant address
// space: the table does not change while a kernel runs, so the loads are
// scalar loads whatever the kernel stores (through a generic pointer, a
// kernel that also stores to global memory gets vector loads, and each
// would wait for the row loads issued before it).
__device__ __forceinline__ HashRec hash_rec(const HashRec *hp, uint32_t i) {
    typedef const HashRec __attribute__((address_space(4))) *ConstHash;
    const ConstHash c = (ConstHash)hp + i;
    HashRec r;
    r.alo = c->alo;
    r.ahi = c->ahi;
    r.clo = c->clo;
    r.chi = c->chi;
    return r;
}

__device__ __forceinline__ uint64_t bloom_pos(const Index &ix, uint32_t i, uint64_t x) {
    return bloom_pos(hash_rec(ix.hp->h, i), ix.m, x);
}

// ---------------------------------------------------------------------------
// k-mer codes: A=0 C=1 G=2 T=3, first base most significant (62 bits).
// ---------------------------------------------------------------------------
// Reverse the 31 two-bit groups of s (base i at group i -> group 30 - i).
__device__ __forceinline__ uint64_t reverse_groups31(uint64_t s) {
    uint64_t v = __builtin_bitreverse64(s);
    v = ((v >> 1) & 0x5555555555555555ULL) | ((v & 0x5555555555555555ULL) << 1);
    return v >> 2;
}

__device__ __forceinline__ uint64_t canonical(uint64_t x) {
    // x = sum c_i 4^(30-i); groups reversed give sum c_i 4^i, whose
    // complement is the reverse complement sum (3 - c_i) 4^i.
    const uint64_t rc = (~reverse_groups31(x)) & MASK62;
    return x < rc ? x : rc;
}

__device__ __forceinline__ uint32_t base_code(uint32_t c) { return ((c >> 1) & 3u) ^ ((c >> 2) & 1u); }

__device__ __forceinline__ bool base_ok(uint32_t c) {
    const uint32_t l = c | 0x20u;
    return l == 'a' || l == 'c' || l == 'g' || l == 't';
}

// Morton spread: bit i of the low 32 bits goes to bit 2i.
__device__ __forceinline__ uint64_t spread32(uint64_t v) {
    v &= 0xFFFFFFFFULL;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFULL;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFULL;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0FULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

// Bits [l, l + 31) of the 128-bit value (hi:lo).
__device__ __forceinline__ uint32_t window31(uint64_t lo, uint64_t hi, uint32_t l) {
    const uint64_t w = l ? ((lo >> l) | (hi << (64 - l))) : lo;
    return (uint32_t)w & 0x7FFFFFFFu;
}

struct Window {
    uint64_t canon;
    bool valid;
};

// Wave-cooperative extraction of 64 consecutive windows. Lane l passes the
// byte at position p0 + l (c0) and, for l < 30, the byte at p0 + 64 + l (c1);
// bytes outside the sequence are passed as 0. Lane l receives the canonical
// code of the window starting at p0 + l and whether all its 31 bytes are
// bases. Three ballots per plane build the 2-bit code planes of the 94
// bytes; each lane then cuts its window out of the planes. Must be called
// by all 64 lanes.
__device__ __forceinline__ Window extract_windows(uint32_t c0, uint32_t c1, uint32_t lane) {
    const uint32_t k0 = base_code(c0), k1 = base_code(c1);
    const uint64_t L0 = __ballot(k0 & 1u), L1 = __ballot(k1 & 1u);
    const uint64_t H0 = __ballot(k0 >> 1), H1 = __ballot(k1 >> 1);
    const uint64_t I0 = __ballot(!base_ok(c0)), I1 = __ballot(!base_ok(c1));
    Window w;
    w.valid = window31(I0, I1, lane) == 0;
    // s = sum c_i 4^i over the window's bases i = 0..30
    const uint64_t s = spread32(window31(L0, L1, lane)) | (spread32(window31(H0, H1, lane)) << 1);
    const uint64_t rc = (~s) & MASK62;
    const uint64_t fwd = reverse_groups31(s);
    w.canon = fwd < rc ? fwd : rc;
    return w;
}

// ---------------------------------------------------------------------------
// Row segments: a lane reads SEG consecutive words of a row.
// ---------------------------------------------------------------------------
template <int SEG>
struct Seg {
    uint32_t w[SEG];
};

template <int SEG>
__device__ __forceinline__ Seg<SEG> load_seg(const uint32_t *p) {
    Seg<SEG> s;
    if constexpr (SEG == 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        s.w[0] = v.x; s.w[1] = v.y; s.w[2] = v.z; s.w[3] = v.w;
    } else if constexpr (SEG == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        s.w[0] = v.x; s.w[1] = v.y;
    } else {
        s.w[0] = *p;
    }
    return s;
}

__device__ __forceinline__ const uint32_t *row_ptr(const Index &ix, uint32_t r, uint64_t pos) {
    return ix.rows + (((uint64_t)r * ix.m + pos) << ix.log2RW);
}

template <int SEG>
__device__ __forceinline__ void set_ones(Seg<SEG> (&acc)[MAXR]) {
#pragma unroll
    for (int r = 0; r < MAXR; r++)
#pragma unroll
        for (int s = 0; s < SEG; s++) acc[r].w[s] = 0xFFFFFFFFu;
}

// 64 x 64 bit-matrix transpose across a wave: lane i holds row i on entry
// and column i on exit (bit j of lane i's input = bit i of lane j's output).
// Six butterfly stages, each swapping the off-diagonal blocks of one size.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, uint32_t lane) {
    const uint64_t masks[6] = {0x00000000FFFFFFFFULL, 0x0000FFFF0000FFFFULL, 0x00FF00FF00FF00FFULL,
                               0x0F0F0F0F0F0F0F0FULL, 0x3333333333333333ULL, 0x5555555555555555ULL};
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const uint32_t s = 32u >> k;
        const uint64_t m = masks[k];
        const uint64_t y = __shfl_xor(x, (int)s);
        x = (lane & s) ? ((x & ~m) | ((y & ~m) >> s)) : ((x & m) | ((y & m) << s));
    }
    return x;
}

// AND across the k-mer groups of a wave: lanes l and l ^ off (off >= G) hold
// the same row segment of different terms.
// With one lane per term (G = 1) the AND of all 64 lanes, by lane moves
// inside each row of 16 (DPP: lane ^ 1, lane ^ 2, the mirrored half-row, the
// mirrored row) and the four rows' lanes read into scalar registers: no LDS
// round trips in the chain, and the result (the same for every lane) kept
// in a scalar register frees vector registers for loads in flight. Must be
// called by all 64 lanes.
template <int G>
__device__ __forceinline__ uint32_t and_across_groups(uint32_t v) {
    if constexpr (G == 1) {
        v &= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        v &= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        v &= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
        v &= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
        return __builtin_amdgcn_readlane(v, 0) & __builtin_amdgcn_readlane(v, 16) & __builtin_amdgcn_readlane(v, 32) &
               __builtin_amdgcn_readlane(v, 48);
    } else {
#pragma unroll
        for (int off = G; off < 64; off <<= 1) v &= __shfl_xor(v, off);
        return v;
    }
}

template <int SEG, int G>
__device__ __forceinline__ void reduce_groups(Seg<SEG> (&acc)[MAXR], uint32_t R) {
#pragma unroll
    for (int r = 0; r < MAXR; r++)
        if (r < (int)R)
#pragma unroll
            for (int s = 0; s < SEG; s++) acc[r].w[s] = and_across_groups<G>(acc[r].w[s]);
}

// After reduce_groups: is the mask of some repetition empty? (wave-uniform)
template <int SEG, int G>
__device__ __forceinline__ bool some_rep_empty(const Seg<SEG> (&acc)[MAXR], uint32_t R) {
    const uint64_t group0 = (G >= 64) ? ~0ULL : ((1ULL << G) - 1);
    bool empty = false;
#pragma unroll
    for (int r = 0; r < MAXR; r++) {
        if (r < (int)R) {
            uint32_t o = 0;
#pragma unroll
            for (int s = 0; s < SEG; s++) o |= acc[r].w[s];
            empty |= (__ballot(o != 0) & group0) == 0;
        }
    }
    return empty;
}

// Rows of term x in repetitions FIRST .. FIRST+COUNT-1 (those below R), with
// ETA hash functions each: all loads issued before any is used (so a wave
// keeps COUNT * ETA row reads in flight), then ANDed into cm -- per
// repetition the Bloom test of all B BFUs at once (Section 2.1, Section 3.3).
// This lane's segment seg of each row.
// cm[OFF + k] receives repetition FIRST + k.
template <int SEG, int FIRST, int COUNT, int ETA, int OFF, int N>
__device__ __forceinline__ void probe_reps_eta(const Index &ix, const HashRec *hp, uint64_t x, uint32_t seg,
                                               Seg<SEG> (&cm)[N]) {
    static_assert(OFF + COUNT <= N, "repetition group past the masks");
    Seg<SEG> v[COUNT][ETA];
#pragma unroll
    for (int k = 0; k < COUNT; k++) {
        if (FIRST + k < (int)ix.R) {
#pragma unroll
            for (int j = 0; j < ETA; j++) {
                const uint64_t pos = bloom_pos(hash_rec(hp, (FIRST + k) * ETA + j), ix.m, x);
                v[k][j] = load_seg<SEG>(row_ptr(ix, FIRST + k, pos) + seg * SEG);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < COUNT; k++)
        if (FIRST + k < (int)ix.R)
#pragma unroll
            for (int j = 0; j < ETA; j++)
#pragma unroll
                for (int s = 0; s < SEG; s++) cm[OFF + k].w[s] &= v[k][j].w[s];
}

// As probe_reps_eta for any eta (up to MAXETA): one row at a time.
template <int SEG, int FIRST, int COUNT, int OFF, int N>
__device__ __forceinline__ void probe_reps_any(const Index &ix, const HashRec *hp, uint64_t x, uint32_t seg,
                                               Seg<SEG> (&cm)[N]) {
#pragma unroll
    for (int k = 0; k < COUNT; k++) {
        if (FIRST + k < (int)ix.R) {
#pragma unroll 1
            for (int j = 0; j < (int)ix.eta; j++) {
                const uint64_t pos = bloom_pos(hash_rec(hp, (FIRST + k) * ix.eta + j), ix.m, x);
                const Seg<SEG> v = load_seg<SEG>(row_ptr(ix, FIRST + k, pos) + seg * SEG);
#pragma unroll
                for (int s = 0; s < SEG; s++) cm[OFF + k].w[s] &= v.w[s];
            }
        }
    }
}

template <int SEG, int FIRST, int COUNT, int OFF = 0, int N>
__device__ __forceinline__ void probe_reps(const Index &ix, const HashRec *hp, uint64_t x, uint32_t seg,
                                           Seg<SEG> (&cm)[N]) {
    switch (ix.eta) {
    case 1: probe_reps_eta<SEG, FIRST, COUNT, 1, OFF, N>(ix, hp, x, seg, cm); break;
    case 2: probe_reps_eta<SEG, FIRST, COUNT, 2, OFF, N>(ix, hp, x, seg, cm); break;
    case 3: probe_reps_eta<SEG, FIRST, COUNT, 3, OFF, N>(ix, hp, x, seg, cm); break;
    default: probe_reps_any<SEG, FIRST, COUNT, OFF, N>(ix, hp, x, seg, cm); break;
    }
}

// Rows of U terms (this lane's segment seg) in repetition r, ETA hashes each:
// all U * ETA loads are issued before any is used. A term with !v[u] loads
// row 0 instead (in range, its value unused) so that no branch separates the
// loads; the result for it is not ANDed.
template <int SEG, int U, int ETA>
__device__ __forceinline__ void probe_terms_eta(const Index &ix, const HashRec *hp, int r, const uint64_t (&x)[U],
                                                const bool (&v)[U], uint32_t seg, Seg<SEG> &cm) {
    Seg<SEG> rows[U][ETA];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int j = 0; j < ETA; j++) {
            const uint64_t pos = v[u] ? bloom_pos(hash_rec(hp, r * ETA + j), ix.m, x[u]) : 0;
            rows[u][j] = load_seg<SEG>(row_ptr(ix, r, pos) + seg * SEG);
        }
#pragma unroll
    for (int u = 0; u < U; u++)
        if (v[u])
#pragma unroll
            for (int j = 0; j < ETA; j++)
#pragma unroll
                for (int s = 0; s < SEG; s++) cm.w[s] &= rows[u][j].w[s];
}

// The hash parameter table, re-derived at every step of a probe loop: the
// compiler then reloads a group's parameters (one scalar load per hash) at
// each step instead of hoisting every repetition's parameters out of the
// loop, which would hold them all in scalar registers at once and spill.
__device__ __forceinline__ const HashRec *step_params(const Index &ix) {
    uint32_t z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return ix.hp->h + z;
}

// Probe term x in every BFU of every repetition: per repetition r, the AND
// over j of rows (r, h_{r,j}(x)) -- the Bloom test of all B BFUs at once
// (Section 2.1, Section 3.3). This lane's segment `seg` of each masked row
// is ANDed into acc[r]; the rows of four repetitions are read together.
template <int SEG>
__device__ __forceinline__ void probe_and(const Index &ix, uint64_t x, uint32_t seg, Seg<SEG> (&acc)[MAXR]) {
    probe_reps<SEG, 0, 4, 0>(ix, ix.hp->h, x, seg, acc);
    if (ix.R > 4) probe_reps<SEG, 4, MAXR - 4, 4>(ix, ix.hp->h, x, seg, acc);
}

// AND a repetition's step mask across the wave into its running mask Mr
// (RW words in the wave's LDS area; lane l of a term group owns words
// (l mod G) * SEG ..); returns whether the running mask is still non-empty
// (wave-uniform).
template <int SEG, int G>
__device__ __forceinline__ bool fold_rep(const Seg<SEG> &cm, uint32_t *Mr, uint32_t lane) {
    const uint64_t group0 = (G >= 64) ? ~0ULL : ((1ULL << G) - 1);
    const uint32_t base = (lane % G) * SEG;
    uint32_t o = 0;
#pragma unroll
    for (int s = 0; s < SEG; s++) {
        uint32_t prev = Mr[base + s];
        if constexpr (G == 1) prev = __builtin_amdgcn_readfirstlane(prev);
        const uint32_t v = and_across_groups<G>(cm.w[s]) & prev;
        if (lane < (uint32_t)G) Mr[base + s] = v;
        o |= v;
    }
    if constexpr (G == 1) return o != 0;  // uniform already
    else return (__ballot(o != 0) & group0) != 0;
}

// Running masks of all repetitions (the wave's LDS area M, R * RW words) to
// all ones: nothing excluded yet.
__device__ __forceinline__ void init_masks(const Index &ix, uint32_t *M, uint32_t lane) {
    for (uint32_t w = lane; w < ix.R * ix.RW; w += 64) M[w] = 0xFFFFFFFFu;
}

// Some repetition's running mask in M is empty (wave-uniform): the read's
// answer is empty.
__device__ __forceinline__ bool masks_some_rep_empty(const Index &ix, const uint32_t *M, uint32_t lane) {
    bool empty = false;
    for (uint32_t r = 0; r < ix.R; r++) {
        uint32_t o = 0;
        for (uint32_t w = lane; w < ix.RW; w += 64) o |= M[r * ix.RW + w];
        empty |= __ballot(o != 0) == 0;
    }
    return empty;
}

// Probe repetitions FIRST .. FIRST+COUNT-1 (those below R) with all their
// loads in flight together and AND them into the running masks; returns
// whether every one of those running masks is still non-empty.
template <int SEG, int G, int FIRST, int COUNT>
__device__ __forceinline__ bool probe_group(const Index &ix, const HashRec *hp, const Window &wv, bool valid,
                                            uint32_t lane, uint32_t *M) {
    static_assert(FIRST + COUNT <= MAXR, "repetition group past MAXR");
    Seg<SEG> cm[COUNT];
#pragma unroll
    for (int k = 0; k < COUNT; k++)
#pragma unroll
        for (int s = 0; s < SEG; s++) cm[k].w[s] = 0xFFFFFFFFu;
    if constexpr (G == 1) {
        if (valid) probe_reps<SEG, FIRST, COUNT>(ix, hp, wv.canon, 0, cm);
    } else {
        // the lanes of a term group split the row: the group's term comes
        // from the lane that extracted it (64/G terms per sub-step, G
        // sub-steps per step)
        constexpr int KPW = 64 / G;
        constexpr int U = (G >= 4) ? 4 : G;  // sub-steps whose loads go together
        // (a group of which only repetition FIRST is below R, e.g. the last
        // one of R = 6, probes as a group of one)
        if ((COUNT == 1 || (int)ix.R == FIRST + 1) && (ix.eta == 1 || ix.eta == 2)) {
            // one repetition, the rows of U sub-steps in flight together
#pragma unroll 1
            for (int s0 = 0; s0 < G; s0 += U) {
                uint64_t xs[U];
                bool vs[U];
                bool any = false;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int src = (s0 + u) * KPW + (int)(lane / G);
                    xs[u] = __shfl(wv.canon, src);
                    vs[u] = __shfl((int)valid, src) != 0;
                    any |= vs[u];
                }
                if (__ballot(any) == 0) continue;  // no term in these sub-steps
                if (ix.eta == 2) probe_terms_eta<SEG, U, 2>(ix, hp, FIRST, xs, vs, lane % G, cm[0]);
                else probe_terms_eta<SEG, U, 1>(ix, hp, FIRST, xs, vs, lane % G, cm[0]);
            }
        } else {
#pragma unroll 1
            for (int sub = 0; sub < G; sub++) {
                const int src = sub * KPW + (int)(lane / G);
                const uint64_t x = __shfl(wv.canon, src);
                const int v = __shfl((int)valid, src);
                if (v) probe_reps<SEG, FIRST, COUNT>(ix, hp, x, lane % G, cm);
            }
        }
    }
    bool alive = true;
#pragma unroll
    for (int k = 0; k < COUNT; k++)
        if (FIRST + k < (int)ix.R) alive &= fold_rep<SEG, G>(cm[k], M + (FIRST + k) * ix.RW, lane);
    return alive;
}

// Zero, as a value the compiler cannot see through: it depends on x, so an
// operation that takes it as an operand is issued only once x is available
// (when x comes from the results of loads or atomics, once they have
// returned).
__device__ __forceinline__ uint32_t opaque_zero(uint64_t x) {
    uint32_t z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z) : "s"(x));
    return z;
}

// bit b of the B-bit mask M (LDS)
__device__ __forceinline__ uint32_t mask_bit(const uint32_t *M, uint32_t b) {
    return (M[b >> 5] >> (b & 31)) & 1u;
}

// RAMBO+ (Section 5.1, query time speedup): in repetition r only the BFUs
// that hold documents returned by the earlier repetitions need a test. For a
// step about to probe repetitions 1..R-1 of its nv valid windows (eta rows
// each), count how much of each probed row a probe restricted to those BFUs
// could leave unread: the candidates of repetition r are the documents whose
// cells are set in the running masks of repetitions 0..r-1; a 16-byte row
// segment (128 cells) or a 128-byte line (1,024 cells) holding none of their
// repetition-r cells would not be read. Adds, over repetitions r >= 1:
// rplus[0] probes, [1] probes whose row holds no candidate cell, [2]
// untouched 16-byte segments, [3] segments probed, [4] untouched 128-byte
// lines, [5] lines probed. Measurement only (every candidate's cell record is
// read once per step); called by all lanes.
__device__ __forceinline__ void rplus_tally(const Index &ix, const uint32_t *M, uint32_t lane, uint64_t nv,
                                            unsigned long long *rplus) {
    uint64_t segs[MAXR];  // per repetition, bit s: segment s holds a candidate cell
#pragma unroll
    for (int r = 0; r < MAXR; r++) segs[r] = 0;
    for (uint32_t c0 = 0; c0 < ix.B; c0 += 64) {
        const uint32_t b = c0 + lane;
        uint64_t todo = __ballot(b < ix.B && mask_bit(M, b));
        while (todo) {
            const uint32_t cb = c0 + (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t beg = ix.boff[cb], len = ix.boff[cb + 1] - beg;
            for (uint32_t k = lane; k < len; k += 64) {
                const uint4 cd = ix.cells[ix.bdoc[beg + k]];
                bool alive = true;
#pragma unroll
                for (int r = 1; r < MAXR; r++) {
                    if (r < (int)ix.R && alive) {
                        const uint32_t c = cell_at(cd, r);
                        segs[r] |= 1ULL << (c >> 7);
                        alive = mask_bit(M + r * ix.RW, c) != 0;
                    }
                }
            }
        }
    }
    const uint32_t nseg = ix.RW >= 4 ? ix.RW / 4 : 1, nline = ix.RW >= 32 ? ix.RW / 32 : 1;
    uint64_t c[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 1; r < MAXR; r++) {
        if (r < (int)ix.R) {
            uint64_t s = segs[r];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s |= __shfl_xor(s, off);
            uint32_t lines = 0;
            for (uint32_t l = 0; l < nline; l++) lines += ((s >> (8 * l)) & 0xFFull) != 0;
            const uint64_t pr = nv * ix.eta;
            c[0] += pr;
            c[1] += s == 0 ? pr : 0;
            c[2] += pr * (nseg - (uint32_t)__popcll(s));
            c[3] += pr * nseg;
            c[4] += pr * (nline - lines);
            c[5] += pr * nline;
        }
    }
    if (lane == 0)
        for (int k = 0; k < 6; k++)
            if (c[k]) atomicAdd(rplus + k, (unsigned long long)c[k]);
}

// Probe schedules of a read's windows (all give the same running masks)
enum : int {
    SCHED_STEP = 0,   // per step of 64 windows: repetition 0, then the others
    SCHED_SWEEP = 1,  // repetition 0 over every step of the span, then the others
    SCHED_SCOUT = 2,  // as SWEEP, after repetition 0 on every 31st window
    // (internal) the batched form's SCHED_SCOUT: a pass of its own has probed
    // the scout windows of every read before the work queue was built
    SCHED_PRESCOUT = 3,
};

// windows of 31 bases in the bytes [beg, end)
__device__ __forceinline__ uint64_t n_windows(uint64_t beg, uint64_t end) {
    return end >= beg + 31 ? end - beg - 30 : 0;
}

// Scout windows of a span [w_lo, w_hi): w_lo, w_lo + 31, ... and the last
// window. Windows 31 apart cover every base of the span, so a read holding
// a base no indexed document has there (a sequencing error, a random read)
// mostly ends on them.
__device__ __forceinline__ uint64_t scout_count(uint64_t w_lo, uint64_t w_hi) {
    const uint64_t span = w_hi - w_lo;  // > 0
    return (span + 30) / 31 + ((span - 1) % 31 != 0 ? 1 : 0);
}
__device__ __forceinline__ uint64_t scout_pos(uint64_t w_lo, uint64_t w_hi, uint64_t i) {
    return min(w_lo + 31 * i, w_hi - 1);
}
__device__ __forceinline__ bool is_scout(uint64_t w_lo, uint64_t w_hi, uint64_t w) {
    // (offsets within one read fit 32 bits)
    return (uint32_t)(w - w_lo) % 31u == 0 || w == w_hi - 1;
}

// Bytes [lo, hi) of seqs (inside one read) to the wave's LDS staging area,
// keeping the global 16-byte alignment: byte lo lands at buf[addr(lo) & 15].
// Whole 16-byte blocks inside [lo, hi) are copied with one load each, the
// blocks at the two ends byte by byte (nothing outside the read is read).
__device__ __forceinline__ void stage_bytes(const uint8_t *__restrict__ seqs, uint64_t lo, uint64_t hi, uint8_t *buf,
                                            uint32_t lane) {
    const uint8_t *first = seqs + lo, *last = seqs + hi;
    const uint8_t *base = reinterpret_cast<const uint8_t *>(reinterpret_cast<uintptr_t>(first) & ~(uintptr_t)15);
    const uint64_t nb = (uint64_t)(last - base + 15) / 16;
    for (uint64_t k = lane; k < nb; k += 64) {
        const uint8_t *a = base + 16 * k;
        uint8_t *dst = buf + 16 * k;
        if (a >= first && a + 16 <= last) {
            *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(a);
        } else {
            for (int i = 0; i < 16; i++)
                if (a + i >= first && a + i < last) dst[i] = a[i];
        }
    }
}

// Four bytes at a time (byte k of w in bits 8k..8k+7): the 2-bit code of
// each byte (base_code, in the byte's low bits); which bytes are not a base
// (non-zero bytes of the result: a byte is a base iff, made lowercase, it is
// the letter its own code stands for, looked up by byte permute in "acgt");
// and the four codes packed first-byte-most-significant into 8 bits (the
// products of the multiply land in distinct bit ranges below bit 24, so no
// carry reaches the top byte).
__device__ __forceinline__ uint32_t codes4(uint32_t w) { return ((w >> 1) & 0x03030303u) ^ ((w >> 2) & 0x01010101u); }
__device__ __forceinline__ uint32_t nonbases4(uint32_t w, uint32_t c) {
    return (w | 0x20202020u) ^ __builtin_amdgcn_perm(0u, 0x74676361u, c);
}
__device__ __forceinline__ uint32_t pack4(uint32_t c) { return (c * 0x40100401u) >> 24; }

// The 31 bytes of a window held in registers, loaded ahead of their use:
// bytes 0-15 in a, 16-27 in b, 28-29 in c and 30 in d, each part loaded by
// one instruction and left as loaded (so that nothing waits for the loads
// before the bytes are decoded). The bytes are read as global memory (a
// generic access would also count against the wave's LDS and scalar-load
// counter, and every wait for those would wait for these loads too).
struct WinBytes {
    uint4 a;
    uint3 b;
    uint32_t c, d;
};
__device__ __forceinline__ void load_window_bytes(WinBytes &wb, const uint8_t *p) {
    typedef const uint8_t __attribute__((address_space(1))) *gbytes;
    const gbytes g = (gbytes)p;
    __builtin_memcpy(&wb.a, g, 16);
    __builtin_memcpy(&wb.b, g + 16, 12);
    uint16_t c;
    __builtin_memcpy(&c, g + 28, 2);
    wb.c = c;
    wb.d = g[30];
}

// The window held in wb, encoded and made canonical, four bytes at a time:
// 32 codes (the last from the zero byte past the window, dropped by the
// final shift) and the non-bases of the 31 bytes.
__device__ __forceinline__ Window decode_window(const WinBytes &wb) {
    const uint32_t v[8] = {wb.a.x, wb.a.y, wb.a.z, wb.a.w, wb.b.x, wb.b.y, wb.b.z, wb.c | (wb.d << 16)};
    uint64_t x = 0;
    uint32_t bad = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const uint32_t c = codes4(v[k]);
        bad |= nonbases4(v[k], c) & (k == 7 ? 0x00FFFFFFu : 0xFFFFFFFFu);
        x = (x << 8) | pack4(c);
    }
    Window w;
    w.valid = bad == 0;
    w.canon = canonical(x >> 2);
    return w;
}

// A window's bytes split over P lanes (P = 2, 4 or 8, lanes q = 0 .. P-1 of
// an aligned block): lane q holds window bytes qL .. qL+L-1 (L = 32 / P; the
// last lane the L-1 bytes up to byte 30, loaded from one byte earlier so that
// nothing past the window is read).
template <int P>
struct WinPart {
    uint32_t w[32 / P / 4];
};
template <int P>
__device__ __forceinline__ void load_window_part(WinPart<P> &wp, const uint8_t *p, uint32_t q) {
    constexpr int L = 32 / P;
    typedef const uint8_t __attribute__((address_space(1))) *gbytes;
    const gbytes g = (gbytes)p + q * L - (q == P - 1 ? 1 : 0);
    __builtin_memcpy(wp.w, g, L);
}

// The window whose parts the P lanes of each aligned block hold, encoded and
// made canonical (every lane of the block gets it). Lane q encodes its bytes,
// the block ORs the codes (invalid bytes flagged in bit 63) by lane exchanges.
// Must be called by all 64 lanes.
template <int P>
__device__ __forceinline__ Window decode_window_parts(const WinPart<P> &wp, uint32_t q) {
    constexpr int L = 32 / P, NW = L / 4;
    const uint32_t last = q == P - 1 ? 1u : 0u;
    // the last lane's bytes start one byte into its words
    uint32_t v[NW];
#pragma unroll
    for (int k = 0; k < NW; k++)
        v[k] = __builtin_amdgcn_alignbyte(k + 1 < NW ? wp.w[k + 1] : 0u, wp.w[k], last);
    // four bytes at a time; the last lane's top byte is past the window
    uint64_t y = 0;
    uint32_t bad = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
        const uint32_t c = codes4(v[k]);
        bad |= nonbases4(v[k], c) & (k == NW - 1 && last ? 0x00FFFFFFu : 0xFFFFFFFFu);
        y = (y << 8) | pack4(c);
    }
    y >>= 2 * last;
    // bytes qL .. qL+n-1 (n = L - last) go to 4^(30 - j): shift the last one
    // to 4^(30 - (qL + n - 1))
    uint64_t part = (y << (2 * (31 - (q * L + L - last)))) | ((uint64_t)(bad != 0) << 63);
#pragma unroll
    for (int d = 1; d < P; d <<= 1) part |= __shfl_xor(part, d);
    Window w;
    w.valid = (part >> 63) == 0;
    w.canon = canonical(part & MASK62);
    return w;
}

// The window of 31 bytes at p (LDS), encoded and made canonical.
__device__ __forceinline__ Window window_at(const uint8_t *p) {
    uint64_t x = 0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 31; i++) {
        const uint32_t c = p[i];
        ok = ok && base_ok(c);
        x = (x << 2) | base_code(c);
    }
    Window w;
    w.valid = ok;
    w.canon = canonical(x & MASK62);
    return w;
}

// The bytes lane needs for the 64 windows of step w (window indices relative
// to the read start beg): base beg+w+lane, and base beg+w+64+lane for the
// lanes whose windows run past the step.
struct StepBytes {
    uint32_t c0, c1;
};
__device__ __forceinline__ StepBytes load_bytes(const uint8_t *__restrict__ seqs, uint64_t beg, uint64_t end,
                                                uint64_t w, uint32_t lane) {
    const uint64_t p = beg + w + lane;
    return {p < end ? (uint32_t)seqs[p] : 0u, (lane < 30 && p + 64 < end) ? (uint32_t)seqs[p + 64] : 0u};
}

// Repetitions 1..R-1 (R <= 5) of a work item's steps when a lane holds a
// whole row (G = 1), two steps in flight: the rows of step w + 64 are issued
// before those of step w are ANDed into the running masks, so a lane keeps up
// to two steps' loads in flight (2 x 4 x ETA rows). The two row sets are
// used alternately (no register copies, which would wait for the loads). A
// step past the item issues its loads at row 0 of repetition 0 (in range,
// unused). Returns the probes issued (with early exit, the step in flight
// when the read ends counts too).
template <int SEG, int ETA>
__device__ __forceinline__ void issue_rows_g1(const Index &ix, const HashRec *hp, uint64_t x, bool valid,
                                              Seg<SEG> (&r)[4][ETA]) {
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int j = 0; j < ETA; j++) {
            const bool use = valid && 1 + k < (int)ix.R;
            const uint64_t pos = use ? bloom_pos(hash_rec(hp, (1 + k) * ETA + j), ix.m, x) : 0;
            r[k][j] = load_seg<SEG>(row_ptr(ix, use ? 1 + k : 0, pos));
        }
}

template <int SEG, int ETA>
__device__ __forceinline__ uint64_t sweep_rest_g1(const Index &ix, const uint8_t *__restrict__ seqs, uint64_t beg,
                                                  uint64_t end, uint64_t w_lo, uint64_t w_hi, uint32_t lane,
                                                  uint32_t *M, bool early_exit) {
    const uint32_t reps = ix.R - 1;
    uint64_t issued = 0;
    Seg<SEG> ra[4][ETA], rb[4][ETA];
    bool va = false, vb = false;
    StepBytes nb = load_bytes(seqs, beg, end, w_lo, lane);
    // extract step w (its bytes in nb), load the next step's bytes, issue step w's rows
    auto stage = [&](uint64_t w, Seg<SEG>(&r)[4][ETA], bool &v) {
        const Window wv = extract_windows(nb.c0, nb.c1, lane);
        v = wv.valid && (w + lane < w_hi);
        nb = load_bytes(seqs, beg, end, w + 64, lane);
        issue_rows_g1<SEG, ETA>(ix, step_params(ix), wv.canon, v, r);
    };
    // AND a step's rows into the running masks; false once one is empty
    auto finish = [&](const Seg<SEG>(&r)[4][ETA], bool v) -> bool {
        bool alive = true;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (1 + k < (int)ix.R) {
                Seg<SEG> cm;
#pragma unroll
                for (int t = 0; t < SEG; t++) cm.w[t] = 0xFFFFFFFFu;
                if (v)
#pragma unroll
                    for (int j = 0; j < ETA; j++)
#pragma unroll
                        for (int t = 0; t < SEG; t++) cm.w[t] &= r[k][j].w[t];
                alive &= fold_rep<SEG, 1>(cm, M + (1 + k) * ix.RW, lane);
            }
        }
        return alive;
    };
    stage(w_lo, ra, va);
    for (uint64_t w = w_lo;;) {
        stage(w + 64, rb, vb);
        issued += (uint64_t)__popcll(__ballot(va)) * reps;
        if (!finish(ra, va) && early_exit) return issued + (uint64_t)__popcll(__ballot(vb)) * reps;
        w += 64;
        if (w >= w_hi) return issued;
        stage(w + 64, ra, va);
        issued += (uint64_t)__popcll(__ballot(vb)) * reps;
        if (!finish(rb, vb) && early_exit) return issued + (uint64_t)__popcll(__ballot(va)) * reps;
        w += 64;
        if (w >= w_hi) return issued;
    }
}

// Probe windows [w_lo, w_hi) of the read held in seqs[beg, end) into the
// running masks in M, 64 windows per step; the step's masks are ANDed across
// the wave (G lanes share a term). With early exit the probing stops once a
// running mask is empty: the read's answer is then empty whatever the other
// rows hold (Section 3.3.1). Under SCHED_STEP each step probes repetition 0
// and then, if the read is still alive, the others. SCHED_SWEEP follows the
// repetition-major order of that section over the whole span: repetition 0
// over every step first, then the others over every step; a read whose answer
// is empty (a random read, a read with a sequencing error) mostly ends within
// repetition 0, without the other repetitions' rows for the windows before
// its first mismatch. SCHED_SCOUT (with a staging area) first probes
// repetition 0 on the span's scout windows, staged through LDS, then sweeps
// as SCHED_SWEEP with those windows skipped in repetition 0; SCHED_PRESCOUT
// sweeps the same way, skipping the scout windows of the whole read, which
// the scout pass has probed and ANDed into M already. The next step's bytes
// are loaded while the current step probes. Returns the number of (window,
// repetition) probes the wave issued.
// With RPLUS, the sweep and scout schedules also tally, before each step of
// the other repetitions, what a RAMBO+ probe could skip (rplus_tally).
template <int SEG, int G, bool RPLUS = false>
__device__ __forceinline__ uint64_t probe_windows(const Index &ix, const uint8_t *__restrict__ seqs, uint64_t beg,
                                                  uint64_t end, uint64_t w_lo, uint64_t w_hi, uint32_t lane,
                                                  uint32_t *M, bool early_exit, int sched, uint8_t *stage,
                                                  unsigned long long *rplus = nullptr) {
    uint64_t issued = 0;
    const bool scout = sched == SCHED_SCOUT && stage != nullptr && w_lo < w_hi;
    // Repetition 0 skips the scout windows: those of this span after the
    // scout pass above, or (SCHED_PRESCOUT) those of the whole read, which a
    // pass of their own has probed and ANDed into the masks already.
    const bool skip0 = scout || sched == SCHED_PRESCOUT;
    const uint64_t sk_lo = scout ? w_lo : 0, sk_hi = scout ? w_hi : n_windows(beg, end);
    if (scout) {
        const uint64_t ns = scout_count(w_lo, w_hi);
        for (uint64_t i0 = 0; i0 < ns; i0 += 64) {
            const uint64_t i1 = min(ns, i0 + 64);
            const uint64_t p0 = scout_pos(w_lo, w_hi, i0);
            const uint64_t b_lo = beg + p0, b_hi = beg + scout_pos(w_lo, w_hi, i1 - 1) + 31;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // earlier reads of the area are done
            __builtin_amdgcn_wave_barrier();
            stage_bytes(seqs, b_lo, b_hi, stage, lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            Window wv;
            wv.canon = 0;
            wv.valid = false;
            if (i0 + lane < i1) {
                const uint32_t q = (uint32_t)(reinterpret_cast<uintptr_t>(seqs + b_lo) & 15) +
                                   (uint32_t)(scout_pos(w_lo, w_hi, i0 + lane) - p0);
                wv = window_at(stage + q);
            }
            const bool alive = probe_group<SEG, G, 0, 1>(ix, step_params(ix), wv, wv.valid, lane, M);
            issued += (uint64_t)__popcll(__ballot(wv.valid));
            if (early_exit && !alive) return issued;
        }
    }
    if ((sched == SCHED_SWEEP || skip0) && ix.R > 1) {
        if (G == 1 && ix.eta <= 2) {
            // one lane per term: repetition 0 over U0 steps at a time, their
            // rows in flight together (a lane holds U0 terms), the next
            // group's bytes loaded meanwhile
            constexpr int U0 = 4;
            StepBytes nb[U0];
#pragma unroll
            for (int u = 0; u < U0; u++) nb[u] = load_bytes(seqs, beg, end, w_lo + 64 * u, lane);
            for (uint64_t w = w_lo; w < w_hi; w += 64 * U0) {
                uint64_t xs[U0];
                bool vs[U0];
                uint64_t nv = 0;
#pragma unroll
                for (int u = 0; u < U0; u++) {
                    const uint64_t wu = w + 64 * u;
                    const Window wv = extract_windows(nb[u].c0, nb[u].c1, lane);
                    vs[u] = wv.valid && (wu + lane < w_hi) && !(skip0 && is_scout(sk_lo, sk_hi, wu + lane));
                    xs[u] = wv.canon;
                    nv += (uint64_t)__popcll(__ballot(vs[u]));
                }
                if (w + 64 * U0 < w_hi)
#pragma unroll
                    for (int u = 0; u < U0; u++) nb[u] = load_bytes(seqs, beg, end, w + 64 * (U0 + u), lane);
                Seg<SEG> cm;
#pragma unroll
                for (int t = 0; t < SEG; t++) cm.w[t] = 0xFFFFFFFFu;
                if (ix.eta == 2) probe_terms_eta<SEG, U0, 2>(ix, step_params(ix), 0, xs, vs, 0, cm);
                else probe_terms_eta<SEG, U0, 1>(ix, step_params(ix), 0, xs, vs, 0, cm);
                const bool alive = fold_rep<SEG, G>(cm, M, lane);
                issued += nv;
                if (early_exit && !alive) return issued;
            }
        } else {
            StepBytes next = load_bytes(seqs, beg, end, w_lo, lane);
            for (uint64_t w = w_lo; w < w_hi; w += 64) {
                const StepBytes cur = next;
                if (w + 64 < w_hi) next = load_bytes(seqs, beg, end, w + 64, lane);
                const Window wv = extract_windows(cur.c0, cur.c1, lane);
                const bool valid = wv.valid && (w + lane < w_hi) && !(skip0 && is_scout(sk_lo, sk_hi, w + lane));
                const bool alive = probe_group<SEG, G, 0, 1>(ix, step_params(ix), wv, valid, lane, M);
                issued += (uint64_t)__popcll(__ballot(valid));
                if (early_exit && !alive) return issued;
            }
        }
        if constexpr (G == 1 && !RPLUS) {
            if (ix.R <= 5 && ix.eta == 2) return issued + sweep_rest_g1<SEG, 2>(ix, seqs, beg, end, w_lo, w_hi, lane, M, early_exit);
            if (ix.R <= 5 && ix.eta == 1) return issued + sweep_rest_g1<SEG, 1>(ix, seqs, beg, end, w_lo, w_hi, lane, M, early_exit);
        }
        StepBytes next = load_bytes(seqs, beg, end, w_lo, lane);
        for (uint64_t w = w_lo; w < w_hi; w += 64) {
            const StepBytes cur = next;
            if (w + 64 < w_hi) next = load_bytes(seqs, beg, end, w + 64, lane);
            const Window wv = extract_windows(cur.c0, cur.c1, lane);
            const bool valid = wv.valid && (w + lane < w_hi);
            const uint64_t nv = (uint64_t)__popcll(__ballot(valid));
            if constexpr (RPLUS) rplus_tally(ix, M, lane, nv, rplus);
            bool alive = probe_group<SEG, G, 1, 4>(ix, step_params(ix), wv, valid, lane, M);
            issued += nv * (min(ix.R, 5u) - 1);
            if ((int)ix.R > 5 && (alive || !early_exit)) {
                alive &= probe_group<SEG, G, 5, MAXR - 5>(ix, step_params(ix), wv, valid, lane, M);
                issued += nv * (ix.R - 5);
            }
            if (early_exit && !alive) return issued;
        }
        return issued;
    }
    StepBytes next = load_bytes(seqs, beg, end, w_lo, lane);
    for (uint64_t w = w_lo; w < w_hi; w += 64) {
        const StepBytes cur = next;
        if (w + 64 < w_hi) next = load_bytes(seqs, beg, end, w + 64, lane);
        const Window wv = extract_windows(cur.c0, cur.c1, lane);
        const bool valid = wv.valid && (w + lane < w_hi);
        // (with one repetition a scout pass has probed its windows already)
        const bool valid0 = valid && !(skip0 && is_scout(sk_lo, sk_hi, w + lane));
        bool alive = probe_group<SEG, G, 0, 1>(ix, step_params(ix), wv, valid0, lane, M);
        issued += (uint64_t)__popcll(__ballot(valid0));
        const uint64_t nv = (uint64_t)__popcll(__ballot(valid));
        if (alive || !early_exit) {
            alive &= probe_group<SEG, G, 1, 4>(ix, step_params(ix), wv, valid, lane, M);
            issued += nv * (min(ix.R, 5u) - 1);
            if ((int)ix.R > 5 && (alive || !early_exit)) {
                alive &= probe_group<SEG, G, 5, MAXR - 5>(ix, step_params(ix), wv, valid, lane, M);
                issued += nv * (ix.R - 5);
            }
        }
        if (early_exit && !alive) return issued;
    }
    return issued;
}

// ---------------------------------------------------------------------------
// Resolve (Section 3.3 / Algorithm 2 with bitmaps, Section 5.1): given the
// per-repetition masks M_r of positive BFUs (staged in LDS, R * RW words),
// document d is reported iff bit phi_r(d) of M_r is set for every r.
// ---------------------------------------------------------------------------
// the bits of row word wi that are real cells (b < B); padding bits above B
// can be set in all-ones masks and must not be read as cells
__device__ __forceinline__ uint32_t cell_mask(const Index &ix, uint32_t wi) {
    const uint32_t lo = wi * 32;
    if (lo + 32 <= ix.B) return 0xFFFFFFFFu;
    if (lo >= ix.B) return 0u;
    return (1u << (ix.B - lo)) - 1u;
}


// Document d's cells are all set in the masks M (repetitions FIRST..R-1).
template <int FIRST>
__device__ __forceinline__ bool doc_kept(const Index &ix, const uint32_t *M, const uint4 &cd) {
    bool keep = true;
#pragma unroll
    for (int r = FIRST; r < MAXR; r++)
        if (r < (int)ix.R) keep = keep && mask_bit(M + r * ix.RW, cell_at(cd, r));
    return keep;
}

// Dense: every document tests its R cells; lane l handles document 64 w + l
// and a ballot forms result word w. Eight words' cell records are loaded
// together.
// With wm (id-list mode), only the non-zero words are written, and wm[k]
// marks which of words 64 k .. 64 k + 63 those are.
__device__ __forceinline__ uint64_t resolve_dense(const Index &ix, const uint32_t *M, uint64_t *out, uint32_t lane,
                                                  uint64_t *wm) {
    constexpr uint32_t U = 8;
    uint64_t pc = 0;  // this lane's documents kept
    for (uint32_t w0 = 0; w0 < ix.W; w0 += 64) {
        uint64_t mine = 0;
        const uint32_t nw = min(64u, ix.W - w0);
        for (uint32_t t = 0; t < nw; t += U) {
            uint4 cd[U];
            bool real[U];
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint64_t d = (uint64_t)(w0 + t + u) * 64 + lane;
                real[u] = t + u < nw && d < ix.K;
                cd[u] = real[u] ? ix.cells[d] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint64_t word = __ballot(real[u] && doc_kept<0>(ix, M, cd[u]));
                if (lane == t + u) mine = word;
            }
        }
        if (wm) {
            const uint64_t nz = __ballot(lane < nw && mine != 0);
            if (lane == 0) wm[w0 >> 6] = nz;
        }
        if (lane < nw) {
            if (!wm || mine) out[w0 + lane] = mine;
            pc += (uint64_t)__popcll(mine);
        }
    }
    return pc;
}

// Candidate: only documents of positive repetition-0 cells can survive the
// intersection (Algorithm 2); each is tested in repetitions 1..R-1 and set in
// an LDS bitset `res` (W words), which is then written out. The candidates
// are spread over the lanes: per 64 cells, lane l takes cell c0 + l (its
// range of bdoc), a prefix sum over the lanes numbers the candidates, and
// each lane then tests candidates k = lane, lane + 64, ... -- the cell range
// loads, the document ids and their cell records each take one round trip
// for up to 128 candidates.
__device__ __forceinline__ uint64_t resolve_candidates(const Index &ix, const uint32_t *M, uint64_t *res,
                                                       uint64_t *out, uint32_t lane, uint64_t *wm) {
    for (uint32_t w = lane; w < ix.W; w += 64) res[w] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t c0 = 0; c0 < ix.B; c0 += 64) {
        const uint32_t b = c0 + lane;
        const bool set = b < ix.B && mask_bit(M, b);
        if (__ballot(set) == 0) continue;
        uint32_t beg = 0, len = 0;
        if (set) {
            beg = ix.boff[b];
            len = ix.boff[b + 1] - beg;
        }
        uint32_t incl = len;  // inclusive prefix sum of len over the lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(incl, off);
            if ((int)lane >= off) incl += t;
        }
        const uint32_t total = __shfl(incl, 63);
        const uint32_t excl = incl - len;
        // a candidate's id and its cell record are loaded together (the
        // records are also kept in repetition 0's grouping): one round trip
        // per 64 * U candidates
        constexpr int U = 4;
        for (uint32_t k0 = 0; k0 < total; k0 += 64 * U) {
            uint32_t pos[U];
            bool has[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t k = k0 + (uint32_t)u * 64 + lane;
                has[u] = k < total;
                // owner: the number of lanes whose inclusive sum is <= k (its
                // range holds candidate k; all lanes take part in the search)
                uint32_t lo = 0;
#pragma unroll
                for (uint32_t st = 32; st; st >>= 1)
                    if (__shfl(incl, (int)(lo + st - 1)) <= k) lo += st;
                const uint32_t ob = __shfl(beg, (int)lo), oe = __shfl(excl, (int)lo);
                pos[u] = has[u] ? ob + (k - oe) : 0u;
            }
            uint32_t d[U];
            uint4 cd[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                d[u] = has[u] ? ix.bdoc[pos[u]] : 0u;
                cd[u] = has[u] ? ix.cells0[pos[u]] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                if (has[u] && doc_kept<1>(ix, M, cd[u]))
                    atomicOr((unsigned long long *)&res[d[u] >> 6], 1ULL << (d[u] & 63));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t pc = 0;
    for (uint32_t w0 = 0; w0 < ix.W; w0 += 64) {
        const uint32_t w = w0 + lane;
        const uint64_t v = w < ix.W ? res[w] : 0;
        if (wm) {
            const uint64_t nz = __ballot(v != 0);
            if (lane == 0) wm[w0 >> 6] = nz;
        }
        if (w < ix.W && (!wm || v)) out[w] = v;
        pc += (uint64_t)__popcll(v);
    }
    return pc;
}

// As resolve_candidates, with the answer written straight into the output
// row instead of an LDS bitset (which would take W words of LDS per wave and
// limit the waves a compute unit holds): the row is zeroed, and once those
// stores have completed each kept candidate sets its bit with an atomic OR
// (the documents of distinct cells are distinct, so each bit is set once).
// Returns this lane's number of documents kept.
__device__ __forceinline__ uint64_t resolve_candidates_out(const Index &ix, const uint32_t *M, uint64_t *out,
                                                           uint32_t lane, uint64_t *wm) {
    for (uint32_t w = lane; w < ix.W; w += 64) out[w] = 0;
    if (wm)
        for (uint32_t k = lane; k < (ix.W + 63) / 64; k += 64) wm[k] = 0;
    // every lane's zeros are performed (acknowledged by L2) before any OR
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    uint64_t kept = 0;
    for (uint32_t c0 = 0; c0 < ix.B; c0 += 64) {
        const uint32_t b = c0 + lane;
        const bool set = b < ix.B && mask_bit(M, b);
        if (__ballot(set) == 0) continue;
        uint32_t beg = 0, len = 0;
        if (set) {
            beg = ix.boff[b];
            len = ix.boff[b + 1] - beg;
        }
        uint32_t incl = len;  // inclusive prefix sum of len over the lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(incl, off);
            if ((int)lane >= off) incl += t;
        }
        const uint32_t total = __shfl(incl, 63);
        const uint32_t excl = incl - len;
        constexpr int U = 4;  // candidates per lane per round trip
        for (uint32_t k0 = 0; k0 < total; k0 += 64 * U) {
            uint32_t pos[U];
            bool has[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t k = k0 + (uint32_t)u * 64 + lane;
                has[u] = k < total;
                uint32_t lo = 0;  // owner lane of candidate k (all lanes search)
#pragma unroll
                for (uint32_t st = 32; st; st >>= 1)
                    if (__shfl(incl, (int)(lo + st - 1)) <= k) lo += st;
                const uint32_t ob = __shfl(beg, (int)lo), oe = __shfl(excl, (int)lo);
                pos[u] = has[u] ? ob + (k - oe) : 0u;
            }
            uint32_t d[U];
            uint4 cd[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                d[u] = has[u] ? ix.bdoc[pos[u]] : 0u;
                cd[u] = has[u] ? ix.cells0[pos[u]] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                if (has[u] && doc_kept<1>(ix, M, cd[u])) {
                    atomicOr((unsigned long long *)&out[d[u] >> 6], 1ULL << (d[u] & 63));
                    if (wm) atomicOr((unsigned long long *)&wm[d[u] >> 12], 1ULL << ((d[u] >> 6) & 63));
                    kept++;
                }
        }
    }
    return kept;
}

// Number of candidates of the repetition-0 cells set in M, estimated from the
// number of cells (documents spread evenly over the B cells).
__device__ __forceinline__ uint64_t estimate_candidates(const Index &ix, const uint32_t *M0) {
    uint64_t cells = 0;
    for (uint32_t wi = 0; wi < ix.RW; wi++) cells += __popc(M0[wi] & cell_mask(ix, wi));
    return cells * ((ix.K + ix.B - 1) / ix.B);
}

// resolve: 0 auto, 1 dense, 2 candidate (with res, an LDS bitset of W words,
// the candidates collect there; without, straight in the output row).
// Returns the number of documents reported (wave-uniform).
__device__ __forceinline__ uint64_t resolve(const Index &ix, const uint32_t *M, uint64_t *res, uint64_t *out,
                                            uint32_t lane, int mode, uint64_t *wm = nullptr) {
    bool cand = false;
    if (mode == 2) cand = true;
    else if (mode == 0) cand = estimate_candidates(ix, M) * (ix.R - 1) * 2 < ix.K * ix.R;
    uint64_t pc = !cand              ? resolve_dense(ix, M, out, lane, wm)
                  : res != nullptr ? resolve_candidates(ix, M, res, out, lane, wm)
                                   : resolve_candidates_out(ix, M, out, lane, wm);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off);
    return pc;
}


__device__ __forceinline__ void write_zeros(uint64_t *out, uint32_t W, uint32_t lane) {
    for (uint32_t w = lane; w < W; w += 64) out[w] = 0;
}

// Answer of a read whose masks are final: with counts (id-list mode) an
// empty answer writes only its count (the bitset row is left as it is) and
// a non-empty one its bitset and count, and with wm as well (per read,
// (W + 63) / 64 words) only the bitset's non-zero words and their marks;
// otherwise the bitset row always.
__device__ __forceinline__ void answer_read(const Index &ix, const uint32_t *M, uint64_t *res, uint64_t *o,
                                            uint32_t lane, int mode, unsigned long long *counts, uint64_t i,
                                            uint64_t *wm = nullptr) {
    if (masks_some_rep_empty(ix, M, lane)) {
        if (counts) {
            if (lane == 0) counts[i] = 0;
        } else {
            write_zeros(o, ix.W, lane);
        }
        return;
    }
    uint64_t *wrow = (counts && wm) ? wm + i * ((ix.W + 63) / 64) : nullptr;
    const uint64_t pc = resolve(ix, M, res, o, lane, mode, wrow);
    if (counts && lane == 0) counts[i] = pc;
}

}  // namespace rambo
