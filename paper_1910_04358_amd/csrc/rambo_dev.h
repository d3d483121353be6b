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
constexpr int MAXETA = 8;
constexpr uint64_t MASK62 = (1ULL << 62) - 1;

// Bloom hash parameters h_{r,j}, index r * eta + j.
struct HashParams {
    uint64_t Alo[MAXR * MAXETA], Ahi[MAXR * MAXETA], Clo[MAXR * MAXETA], Chi[MAXR * MAXETA];
};

// Everything a kernel needs to address the index (passed by value).
struct Index {
    uint32_t *rows;          // [R][m][RW]
    const HashParams *hp;    // device
    const uint16_t *phi;     // [R][K]   phi_r(d)
    const uint32_t *boff;    // [R][B+1] cell offsets into bdoc
    const uint32_t *bdoc;    // [R][K]   documents grouped by cell, ascending
    uint64_t m;
    uint64_t K;
    uint32_t B, R, eta, RW;  // RW = 32-bit words per row (power of two)
    uint32_t log2RW, W;      // W = result words per query
};

// A batch of reads described in device memory, so that one captured graph
// can serve batches of any size and placement: read i is
// seqs[offs[i] .. offs[i+1]), i < n. n comes first (scans read it alone).
struct InputHdr {
    uint64_t n;
    const uint64_t *offs;
    const uint8_t *seqs;
    uint64_t pad;
};

// ---------------------------------------------------------------------------
// Hashing: h_{r,j}(x) = floor(m * hi64((A x + C) mod 2^128) / 2^64)
// (multiply-add-shift, strongly universal for 62-bit keys; range reduced by
// a multiply-high, which is the plain top-bits shift when m = 2^t).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t bloom_pos(const Index &ix, uint32_t i, uint64_t x) {
    const uint64_t alo = ix.hp->Alo[i], ahi = ix.hp->Ahi[i];
    const uint64_t clo = ix.hp->Clo[i], chi = ix.hp->Chi[i];
    const uint64_t lo = alo * x;
    uint64_t hi = __umul64hi(alo, x) + ahi * x;
    const uint64_t lo2 = lo + clo;
    hi += chi + (lo2 < lo ? 1 : 0);
    return __umul64hi(hi, ix.m);
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

// Probe term x in every BFU of every repetition: per repetition r, the AND
// over j of rows (r, h_{r,j}(x)) -- the Bloom test of all B BFUs at once
// (Section 2.1, Section 3.3). This lane's segment `seg` of each masked row
// is ANDed into acc[r].
template <int SEG>
__device__ __forceinline__ void probe_and(const Index &ix, uint64_t x, uint32_t seg, Seg<SEG> (&acc)[MAXR]) {
#pragma unroll
    for (int r = 0; r < MAXR; r++) {
        if (r < (int)ix.R) {
#pragma unroll
            for (int j = 0; j < MAXETA; j++) {
                if (j < (int)ix.eta) {
                    const uint64_t pos = bloom_pos(ix, (uint32_t)r * ix.eta + j, x);
                    const Seg<SEG> v = load_seg<SEG>(row_ptr(ix, r, pos) + seg * SEG);
#pragma unroll
                    for (int s = 0; s < SEG; s++) acc[r].w[s] &= v.w[s];
                }
            }
        }
    }
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
template <int G>
__device__ __forceinline__ uint32_t and_across_groups(uint32_t v) {
#pragma unroll
    for (int off = G; off < 64; off <<= 1) v &= __shfl_xor(v, off);
    // one lane per term: the result is the same in every lane; keeping it in
    // a scalar register frees vector registers for loads in flight
    if constexpr (G == 1) v = __builtin_amdgcn_readfirstlane(v);
    return v;
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

// Probe term x in repetition r only: AND over j of rows (r, h_{r,j}(x)),
// this lane's segment.
template <int SEG>
__device__ __forceinline__ void probe_rep(const Index &ix, uint64_t x, uint32_t seg, int r, Seg<SEG> &acc) {
#pragma unroll
    for (int j = 0; j < MAXETA; j++) {
        if (j < (int)ix.eta) {
            const uint64_t pos = bloom_pos(ix, (uint32_t)r * ix.eta + j, x);
            const Seg<SEG> v = load_seg<SEG>(row_ptr(ix, r, pos) + seg * SEG);
#pragma unroll
            for (int s = 0; s < SEG; s++) acc.w[s] &= v.w[s];
        }
    }
}

// Probe one term in repetition r into cm (the lanes of a term group split the
// row); for G > 1 the group's term is fetched from the lane that extracted it.
template <int SEG, int G>
__device__ __forceinline__ void probe_rep_step(const Index &ix, const Window &wv, bool valid, uint32_t lane, int r,
                                               Seg<SEG> &cm) {
#pragma unroll
    for (int s = 0; s < SEG; s++) cm.w[s] = 0xFFFFFFFFu;
    if constexpr (G == 1) {
        if (valid) probe_rep<SEG>(ix, wv.canon, 0, r, cm);
    } else {
        constexpr int KPW = 64 / G;
#pragma unroll 1
        for (int sub = 0; sub < G; sub++) {
            const int src = sub * KPW + (int)(lane / G);
            const uint64_t x = __shfl(wv.canon, src);
            const int v = __shfl((int)valid, src);
            if (v) probe_rep<SEG>(ix, x, lane % G, r, cm);
        }
    }
}

// AND a repetition's step mask across the wave into the running mask;
// returns whether the running mask is still non-empty.
template <int SEG, int G>
__device__ __forceinline__ bool fold_rep(const Seg<SEG> &cm, Seg<SEG> &acc) {
    const uint64_t group0 = (G >= 64) ? ~0ULL : ((1ULL << G) - 1);
    uint32_t o = 0;
#pragma unroll
    for (int s = 0; s < SEG; s++) {
        acc.w[s] &= and_across_groups<G>(cm.w[s]);
        o |= acc.w[s];
    }
    if constexpr (G == 1) return o != 0;  // uniform already
    else return (__ballot(o != 0) & group0) != 0;
}

// One step of 64 windows: repetition 0 first, then the other repetitions
// together (their loads all in flight at once). The step's masks are ANDed
// across the wave (G lanes share a term) into the read's running masks acc.
// With early exit the step stops once a running mask is empty -- the read's
// answer is then empty whatever the other repetitions hold (Section 3.3.1);
// random and erroneous reads mostly end at repetition 0 of their first
// step. Returns the number of repetitions probed; *dead tells whether the
// read ended.
template <int SEG, int G>
__device__ __forceinline__ uint32_t probe_step(const Index &ix, const Window &wv, bool valid, uint32_t lane,
                                               Seg<SEG> (&acc)[MAXR], bool early_exit, bool *dead) {
    *dead = false;
    Seg<SEG> cm0;
    probe_rep_step<SEG, G>(ix, wv, valid, lane, 0, cm0);
    if (!fold_rep<SEG, G>(cm0, acc[0]) && early_exit) {
        *dead = true;
        return 1;
    }
    // repetitions 1.. in groups of four (one group for R <= 5), all loads of a
    // group in flight together
    constexpr int GR = 4;
    bool alive = true;
#pragma unroll
    for (int g0 = 1; g0 < MAXR; g0 += GR) {
        if (g0 < (int)ix.R && (alive || !early_exit)) {
            Seg<SEG> cm[GR];
#pragma unroll
            for (int k = 0; k < GR; k++)
                if (g0 + k < MAXR && g0 + k < (int)ix.R) probe_rep_step<SEG, G>(ix, wv, valid, lane, g0 + k, cm[k]);
#pragma unroll
            for (int k = 0; k < GR; k++)
                if (g0 + k < MAXR && g0 + k < (int)ix.R) alive &= fold_rep<SEG, G>(cm[k], acc[g0 + k]);
        }
    }
    *dead = early_exit && !alive;
    return ix.R;
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

__device__ __forceinline__ uint32_t mask_bit(const uint32_t *M, uint32_t b) {
    return (M[b >> 5] >> (b & 31)) & 1u;
}

// Dense: every document tests its R cells; lane l handles document 64 w + l
// and a ballot forms result word w.
__device__ __forceinline__ void resolve_dense(const Index &ix, const uint32_t *M, uint64_t *out, uint32_t lane) {
    for (uint32_t w0 = 0; w0 < ix.W; w0 += 64) {
        uint64_t mine = 0;
        const uint32_t nw = min(64u, ix.W - w0);
        for (uint32_t t = 0; t < nw; t++) {
            const uint64_t d = (uint64_t)(w0 + t) * 64 + lane;
            bool keep = d < ix.K;
            for (uint32_t r = 0; r < ix.R && keep; r++)
                keep = mask_bit(M + r * ix.RW, ix.phi[(uint64_t)r * ix.K + d]);
            const uint64_t word = __ballot(keep);
            if (lane == t) mine = word;
        }
        if (lane < nw) out[w0 + lane] = mine;
    }
}

// Candidate: only documents of positive repetition-0 cells can survive the
// intersection (Algorithm 2); each is tested in repetitions 1..R-1 and set in
// an LDS bitset `res` (W words), which is then written out.
__device__ __forceinline__ void resolve_candidates(const Index &ix, const uint32_t *M, uint64_t *res,
                                                   uint64_t *out, uint32_t lane) {
    for (uint32_t w = lane; w < ix.W; w += 64) res[w] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (uint32_t wi = 0; wi < ix.RW; wi++) {
        uint32_t bits = M[wi] & cell_mask(ix, wi);
        while (bits) {
            const uint32_t b = wi * 32 + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1;
            const uint32_t beg = ix.boff[b], end = ix.boff[b + 1];
            for (uint32_t i = beg + lane; i < end; i += 64) {
                const uint32_t d = ix.bdoc[i];
                bool keep = true;
                for (uint32_t r = 1; r < ix.R && keep; r++)
                    keep = mask_bit(M + r * ix.RW, ix.phi[(uint64_t)r * ix.K + d]);
                if (keep) atomicOr((unsigned long long *)&res[d >> 6], 1ULL << (d & 63));
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t w = lane; w < ix.W; w += 64) out[w] = res[w];
}

__device__ __forceinline__ uint64_t popcount_cells(const Index &ix, const uint32_t *M0) {
    uint64_t n = 0;
    for (uint32_t wi = 0; wi < ix.RW; wi++) {
        uint32_t bits = M0[wi] & cell_mask(ix, wi);
        while (bits) {
            const uint32_t b = wi * 32 + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1;
            n += ix.boff[b + 1] - ix.boff[b];
        }
    }
    return n;
}

// resolve: 0 auto, 1 dense, 2 candidate (res == nullptr forces dense)
__device__ __forceinline__ void resolve(const Index &ix, const uint32_t *M, uint64_t *res, uint64_t *out,
                                        uint32_t lane, int mode) {
    bool cand = false;
    if (res != nullptr) {
        if (mode == 2) cand = true;
        else if (mode == 0) cand = popcount_cells(ix, M) * (ix.R - 1) * 2 < ix.K * ix.R;
    }
    if (cand) resolve_candidates(ix, M, res, out, lane);
    else resolve_dense(ix, M, out, lane);
}

__device__ __forceinline__ void write_zeros(uint64_t *out, uint32_t W, uint32_t lane) {
    for (uint32_t w = lane; w < W; w += 64) out[w] = 0;
}

}  // namespace rambo
