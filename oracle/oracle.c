/*
 * RAMBO CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the RAMBO hot
 * path computes (Gupta et al., "Fast Processing and Querying of 170TB of
 * Genomics Data via a Repeated And Merged BloOm Filter (RAMBO)", SIGMOD 2021).
 * Only the tests, the package smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code with the GPU library and must never be on
 * the product path.
 *
 * Layout: BFU-major, the paper's own picture of the structure (Section 3,
 * Figure 2): an R x B array of Bloom filters, each m bits,
 *     bits[(r * B + b) * wpb + p / 64] bit (p % 64),  wpb = ceil(m / 64).
 *
 * Definitions (each function cites the passage it follows):
 *   - k-mer terms: length-31 sliding windows, stride 1, over ACGT, two bits
 *     per base in a 64-bit integer (Section 1, Figure 1; Section 5.1
 *     "k-mer size"). Canonical form and bit order are readings (see below).
 *   - Bloom filter: insert sets bits h_1(x)..h_eta(x); a test ANDs them
 *     (Section 2.1).
 *   - RAMBO: R independent 2-universal partition hashes phi_r map documents
 *     to B cells; BFU(r, b) is the Bloom filter of the union of the k-mer sets
 *     of documents d with phi_r(d) = b (Section 3, Section 3.2, Algorithm 1).
 *   - Query: union of the documents of positive BFUs within a repetition,
 *     intersection across repetitions (Section 3.3, Algorithm 2); a sequence
 *     query ANDs the outputs of all its terms (Section 3.3.1).
 *
 * Readings where the paper is silent or garbled:
 *   - Encoding: A=0 C=1 G=2 T=3 (case-insensitive), first base in the two
 *     most significant bits; canonical = min(forward, reverse complement) as
 *     unsigned; a window holding any other byte is not a term.
 *   - Hash families (Section 2.1 cites Carter-Wegman universal hashing but
 *     fixes no family): phi_r(d) = ((a_r d + b_r) mod P) mod B, P = 2^61 - 1
 *     (Carter-Wegman); h_{r,j}(x) = floor(m * y / 2^64) with
 *     y = floor(((A_{r,j} x + C_{r,j}) mod 2^128) / 2^64), A, C uniform
 *     128-bit (Dietzfelbinger's multiply-add-shift, strongly universal for
 *     62-bit keys). Each repetition draws its own eta functions; all BFUs of
 *     one repetition share them.
 *   - Parameters come from SplitMix64 seeded with `seed`, drawn in this
 *     order: for r < R: a_r = 1 + next mod (P - 1), b_r = next mod P; then
 *     for r < R, j < eta: A_lo, A_hi, C_lo, C_hi.
 *   - Algorithm 1 writes phi_d(x); Section 3.2 makes the partition a function
 *     of the document, so the oracle uses phi_r(document). Its repetition
 *     range {0..R} is read as R repetitions.
 *   - A query with no term (every window invalid) returns every document:
 *     the vacuous "every x in Q is in the BFU" of Algorithm 2.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define KMER 31
#define P61 ((1ULL << 61) - 1)

typedef struct {
    uint64_t K, m, seed, wpb, W;
    uint32_t B, R, eta;
    uint64_t *pa, *pb;                 /* [R] */
    uint64_t *Alo, *Ahi, *Clo, *Chi;   /* [R * eta] */
    uint64_t *bits;                    /* [R][B][wpb], may be NULL */
    uint32_t *cells;                   /* [R][K] explicit partition, or NULL: phi_r */
    uint32_t *bucket_off;              /* [R][B + 1] */
    uint64_t *bucket_doc;              /* [R][K] documents grouped by cell, ascending */
} orc_t;

/* ---- SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) ---------------------- */
static uint64_t sm_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ---- partition hash phi_r (Section 3.2; Carter-Wegman) ------------------ */
uint32_t orc_phi(const orc_t *o, uint32_t r, uint64_t d) {
    u128 v = (u128)o->pa[r] * d + o->pb[r];
    return (uint32_t)((uint64_t)(v % P61) % o->B);
}

/* The cell of document d in repetition r: phi_r(d), or, for an index whose
 * partition is given as a table (the two-level partition of Section 5.3),
 * the table's entry. */
static uint32_t cell_of(const orc_t *o, uint32_t r, uint64_t d) {
    return o->cells ? o->cells[(size_t)r * o->K + d] : orc_phi(o, r, d);
}

/* Routing of Section 5.3: tau(d) = ((a d + b) mod P) mod G, a random hash of
 * the document id that picks one of G shards, with a = 1 + x0 mod (P - 1),
 * b = x1 mod P for the first two SplitMix64 outputs x0, x1 of route_seed. */
uint32_t orc_route(uint64_t route_seed, uint32_t G, uint64_t d) {
    uint64_t s = route_seed;
    const uint64_t a = 1 + sm_next(&s) % (P61 - 1), b = sm_next(&s) % P61;
    u128 v = (u128)a * d + b;
    return (uint32_t)((uint64_t)(v % P61) % G);
}

/* ---- Bloom filter hash h_{r,j} (Section 2.1) ---------------------------- */
uint64_t orc_h(const orc_t *o, uint32_t r, uint32_t j, uint64_t x) {
    uint32_t i = r * o->eta + j;
    u128 A = ((u128)o->Ahi[i] << 64) | o->Alo[i];
    u128 C = ((u128)o->Chi[i] << 64) | o->Clo[i];
    uint64_t y = (uint64_t)((A * x + C) >> 64);
    return (uint64_t)(((u128)y * o->m) >> 64);
}

/* ---- k-mer encoding (Section 5.1: k = 31, two bits per base) ------------ */
static int base_code(uint8_t c) {
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

/* reverse complement of a 31-mer code: base i moves to position 30 - i and
 * is complemented (A<->T, C<->G, i.e. code -> 3 - code) */
uint64_t orc_revcomp(uint64_t x) {
    uint64_t y = 0;
    for (int i = 0; i < KMER; i++) {
        uint64_t c = (x >> (2 * (KMER - 1 - i))) & 3;  /* base i, first base most significant */
        y |= (3 - c) << (2 * i);
    }
    return y;
}

uint64_t orc_canon(uint64_t x) {
    uint64_t y = orc_revcomp(x);
    return x < y ? x : y;
}

/* Canonical code of the window seq[p .. p+30]; returns 0 if a byte is not
 * ACGT (window skipped), 1 otherwise. */
int orc_window(const uint8_t *seq, uint64_t p, uint64_t *out) {
    uint64_t fwd = 0;
    for (int i = 0; i < KMER; i++) {
        int c = base_code(seq[p + i]);
        if (c < 0) return 0;
        fwd = (fwd << 2) | (uint64_t)c;
    }
    *out = orc_canon(fwd);
    return 1;
}

/* ---- construction ------------------------------------------------------- */
static void build_buckets(orc_t *o) {
    o->bucket_off = calloc((size_t)o->R * (o->B + 1), sizeof(uint32_t));
    o->bucket_doc = malloc((size_t)o->R * o->K * sizeof(uint64_t));
    for (uint32_t r = 0; r < o->R; r++) {
        uint32_t *off = o->bucket_off + (size_t)r * (o->B + 1);
        for (uint64_t d = 0; d < o->K; d++) off[cell_of(o, r, d) + 1]++;
        for (uint32_t b = 0; b < o->B; b++) off[b + 1] += off[b];
        uint32_t *fill = calloc(o->B, sizeof(uint32_t));
        for (uint64_t d = 0; d < o->K; d++) {
            uint32_t b = cell_of(o, r, d);
            o->bucket_doc[(size_t)r * o->K + off[b] + fill[b]++] = d;
        }
        free(fill);
    }
}

static orc_t *new_index(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                        int alloc_bits, const uint32_t *cells) {
    if (K == 0 || B == 0 || R == 0 || m == 0 || eta == 0 || K >= P61) return NULL;
    orc_t *o = calloc(1, sizeof(orc_t));
    if (cells) {
        for (uint64_t i = 0; i < (uint64_t)R * K; i++)
            if (cells[i] >= B) { free(o); return NULL; }
        o->cells = malloc((size_t)R * K * sizeof(uint32_t));
        memcpy(o->cells, cells, (size_t)R * K * sizeof(uint32_t));
    }
    o->K = K; o->B = B; o->R = R; o->m = m; o->eta = eta; o->seed = seed;
    o->wpb = (m + 63) / 64;
    o->W = (K + 63) / 64;
    o->pa = malloc(R * sizeof(uint64_t));
    o->pb = malloc(R * sizeof(uint64_t));
    o->Alo = malloc((size_t)R * eta * sizeof(uint64_t));
    o->Ahi = malloc((size_t)R * eta * sizeof(uint64_t));
    o->Clo = malloc((size_t)R * eta * sizeof(uint64_t));
    o->Chi = malloc((size_t)R * eta * sizeof(uint64_t));
    uint64_t s = seed;
    for (uint32_t r = 0; r < R; r++) {
        o->pa[r] = 1 + sm_next(&s) % (P61 - 1);
        o->pb[r] = sm_next(&s) % P61;
    }
    for (uint32_t i = 0; i < R * eta; i++) {
        o->Alo[i] = sm_next(&s);
        o->Ahi[i] = sm_next(&s);
        o->Clo[i] = sm_next(&s);
        o->Chi[i] = sm_next(&s);
    }
    if (alloc_bits) {
        o->bits = calloc((size_t)R * B * o->wpb, sizeof(uint64_t));
        if (!o->bits) { free(o); return NULL; }
    }
    build_buckets(o);
    return o;
}

orc_t *orc_new(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed, int alloc_bits) {
    return new_index(K, B, R, m, eta, seed, alloc_bits, NULL);
}

/* An index whose partition is the table cells[r * K + d] (< B) instead of
 * phi_r; the Bloom hash functions are those of orc_new with the same seed,
 * R and eta (they do not depend on B). Used for the two-level partition
 * b * tau(d) + phi_r(d) of Section 5.3 and for shards whose documents keep
 * their global ids. NULL if a cell is out of range. */
orc_t *orc_new_cells(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                     const uint32_t *cells, int alloc_bits) {
    return new_index(K, B, R, m, eta, seed, alloc_bits, cells);
}

void orc_free(orc_t *o) {
    if (!o) return;
    free(o->cells);
    free(o->pa); free(o->pb); free(o->Alo); free(o->Ahi); free(o->Clo); free(o->Chi);
    free(o->bits); free(o->bucket_off); free(o->bucket_doc);
    free(o);
}

uint64_t *orc_bits(orc_t *o) { return o->bits; }
uint64_t orc_wpb(const orc_t *o) { return o->wpb; }
uint64_t orc_result_words(const orc_t *o) { return o->W; }
void orc_params(const orc_t *o, uint64_t *pa, uint64_t *pb, uint64_t *Alo, uint64_t *Ahi,
                uint64_t *Clo, uint64_t *Chi) {
    memcpy(pa, o->pa, o->R * 8); memcpy(pb, o->pb, o->R * 8);
    memcpy(Alo, o->Alo, (size_t)o->R * o->eta * 8); memcpy(Ahi, o->Ahi, (size_t)o->R * o->eta * 8);
    memcpy(Clo, o->Clo, (size_t)o->R * o->eta * 8); memcpy(Chi, o->Chi, (size_t)o->R * o->eta * 8);
}

static inline uint64_t *bfu(const orc_t *o, uint32_t r, uint32_t b) {
    return o->bits + ((size_t)r * o->B + b) * o->wpb;
}

/* Bloom filter insertion into one BFU (Section 2.1) */
static void bf_insert(const orc_t *o, uint32_t r, uint64_t *f, uint64_t x) {
    for (uint32_t j = 0; j < o->eta; j++) {
        uint64_t p = orc_h(o, r, j, x);
        f[p >> 6] |= 1ULL << (p & 63);
    }
}

/* Bloom filter test: AND of the eta bits (Section 2.1) */
static int bf_test(const orc_t *o, uint32_t r, const uint64_t *f, uint64_t x) {
    for (uint32_t j = 0; j < o->eta; j++) {
        uint64_t p = orc_h(o, r, j, x);
        if (!((f[p >> 6] >> (p & 63)) & 1)) return 0;
    }
    return 1;
}

/* Algorithm 1 for one document given as 2-bit k-mer codes (either strand):
 * every term goes into BFU(r, phi_r(d)) of every repetition. Returns -1 if a
 * value is not a 31-mer code (>= 4^31) or d >= K; nothing is inserted then. */
int orc_insert_kmers(orc_t *o, uint64_t d, const uint64_t *kmers, uint64_t n) {
    if (d >= o->K) return -1;
    for (uint64_t i = 0; i < n; i++)
        if (kmers[i] >> 62) return -1;
    for (uint32_t r = 0; r < o->R; r++) {
        uint64_t *f = bfu(o, r, cell_of(o, r, d));
        for (uint64_t i = 0; i < n; i++) bf_insert(o, r, f, orc_canon(kmers[i]));
    }
    return 0;
}

/* Algorithm 1 for one document given as a sequence: its terms are its valid
 * 31-windows (Figure 1). */
int orc_insert_seq(orc_t *o, uint64_t d, const uint8_t *seq, uint64_t len) {
    if (d >= o->K) return -1;
    for (uint32_t r = 0; r < o->R; r++) {
        uint64_t *f = bfu(o, r, cell_of(o, r, d));
        for (uint64_t p = 0; p + KMER <= len; p++) {
            uint64_t x;
            if (orc_window(seq, p, &x)) bf_insert(o, r, f, x);
        }
    }
    return 0;
}

/* The terms of documents d0 .. d0+nd-1 (each doc_len bytes, concatenated in
 * `docs`) inserted into the BFUs of one repetition/cell at a time: every
 * thread owns whole BFUs, so no two threads write the same filter. */
int orc_build_docs(orc_t *o, const uint8_t *docs, uint64_t doc_len, uint64_t d0, uint64_t nd,
                   int nthreads) {
    if (d0 + nd > o->K) return -1;
    int64_t cells = (int64_t)o->R * o->B;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t c = 0; c < cells; c++) {
        uint32_t r = (uint32_t)(c / o->B), b = (uint32_t)(c % o->B);
        uint64_t *f = bfu(o, r, b);
        for (uint64_t i = 0; i < nd; i++) {
            if (cell_of(o, r, d0 + i) != b) continue;
            const uint8_t *s = docs + i * doc_len;
            for (uint64_t p = 0; p + KMER <= doc_len; p++) {
                uint64_t x;
                if (orc_window(s, p, &x)) bf_insert(o, r, f, x);
            }
        }
    }
    return 0;
}

/* Insert one document's terms into an external m-bit filter standing for
 * BFU(r, phi_r(d)) -- used to build single sampled BFUs of a large index. */
void orc_bfu_insert_seq(const orc_t *o, uint32_t r, uint64_t *f, const uint8_t *seq, uint64_t len) {
    for (uint64_t p = 0; p + KMER <= len; p++) {
        uint64_t x;
        if (orc_window(seq, p, &x)) bf_insert(o, r, f, x);
    }
}

/* "Q in BFU" of Algorithm 2 against an external filter of repetition r:
 * 1 iff every term of the sequence passes (vacuously 1 with no term). */
int orc_bfu_test_seq(const orc_t *o, uint32_t r, const uint64_t *f, const uint8_t *seq, uint64_t len) {
    for (uint64_t p = 0; p + KMER <= len; p++) {
        uint64_t x;
        if (orc_window(seq, p, &x) && !bf_test(o, r, f, x)) return 0;
    }
    return 1;
}

/* orc_bfu_test_seq for n reads (seqs[offsets[i] .. offsets[i+1])) into
 * out[i], parallel over reads. */
void orc_bfu_test_seqs(const orc_t *o, uint32_t r, const uint64_t *f, const uint8_t *seqs, const uint64_t *offsets,
                       uint64_t n, uint8_t *out, int nthreads) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; i++)
        out[i] = (uint8_t)orc_bfu_test_seq(o, r, f, seqs + offsets[i], offsets[i + 1] - offsets[i]);
}

static inline void setbit(uint64_t *out, uint64_t d) { out[d >> 6] |= 1ULL << (d & 63); }

/* ---- one repetition at a time ---------------------------------------------
 * The answer of Algorithm 2 is the intersection over repetitions of G_r (the
 * documents of the BFUs of repetition r that hold every term), so an index
 * too large for host memory can be evaluated one repetition at a time: the
 * B filters of repetition r alone, rep_bits[B][wpb], built by Algorithm 1
 * restricted to r, then G_r of every query intersected into its answer. */

/* Algorithm 1 for repetition r only: the terms of documents d0 .. d0+nd-1
 * (doc_len bytes each, concatenated in `docs`) into rep_bits[phi_r(d)].
 * Threads own whole filters. */
int orc_build_rep(const orc_t *o, uint32_t r, uint64_t *rep_bits, const uint8_t *docs, uint64_t doc_len,
                  uint64_t d0, uint64_t nd, int nthreads) {
    if (r >= o->R || d0 + nd > o->K) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t b = 0; b < (int64_t)o->B; b++) {
        uint64_t *f = rep_bits + (uint64_t)b * o->wpb;
        for (uint64_t i = 0; i < nd; i++) {
            if (cell_of(o, r, d0 + i) != (uint32_t)b) continue;
            const uint8_t *s = docs + i * doc_len;
            for (uint64_t p = 0; p + KMER <= doc_len; p++) {
                uint64_t x;
                if (orc_window(s, p, &x)) bf_insert(o, r, f, x);
            }
        }
    }
    return 0;
}

/* Repetition r of Algorithm 2 for n sequence queries (seqs[offsets[i] ..
 * offsets[i+1])): G_r = the union of the documents of every BFU of
 * repetition r in which every term of the query passes (vacuously every BFU
 * for a query without a term); out[i] (W words) becomes G_r if `first`, else
 * out[i] AND G_r. Parallel over queries. */
void orc_alg2_rep(const orc_t *o, uint32_t r, const uint64_t *rep_bits, const uint8_t *seqs,
                  const uint64_t *offsets, uint64_t n, uint64_t *out, int first, int nthreads) {
    const uint32_t *off = o->bucket_off + (size_t)r * (o->B + 1);
    const uint64_t *cell_docs = o->bucket_doc + (size_t)r * o->K;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        const uint8_t *s = seqs + offsets[i];
        const uint64_t len = offsets[i + 1] - offsets[i];
        uint64_t *G = calloc(o->W, 8);
        for (uint32_t b = 0; b < o->B; b++) {
            const uint64_t *f = rep_bits + (uint64_t)b * o->wpb;
            int holds_all = 1;
            for (uint64_t p = 0; p + KMER <= len && holds_all; p++) {
                uint64_t x;
                if (orc_window(s, p, &x) && !bf_test(o, r, f, x)) holds_all = 0;
            }
            if (holds_all)
                for (uint32_t k = off[b]; k < off[b + 1]; k++) setbit(G, cell_docs[k]);
        }
        uint64_t *a = out + (uint64_t)i * o->W;
        for (uint64_t w = 0; w < o->W; w++) a[w] = first ? G[w] : (a[w] & G[w]);
        free(G);
    }
}

uint64_t orc_popcount_bfu(const orc_t *o, uint32_t r, uint32_t b) {
    uint64_t c = 0;
    const uint64_t *f = bfu(o, r, b);
    for (uint64_t w = 0; w < o->wpb; w++) c += (uint64_t)__builtin_popcountll(f[w]);
    return c;
}

/* ---- queries ------------------------------------------------------------ */

/* Definition mode, one term: document d is reported iff for every repetition
 * r the BFU it belongs to, BFU(r, phi_r(d)), passes the Bloom test
 * (Section 3.3: union within a repetition, intersection across). Evaluated
 * document by document, without forming per-repetition sets first. */
void orc_query_kmer_def(const orc_t *o, uint64_t x, uint64_t *out) {
    x = orc_canon(x);
    memset(out, 0, o->W * 8);
    for (uint64_t d = 0; d < o->K; d++) {
        int keep = 1;
        for (uint32_t r = 0; r < o->R && keep; r++) keep = bf_test(o, r, bfu(o, r, cell_of(o, r, d)), x);
        if (keep) setbit(out, d);
    }
}

/* The query of Section 3.3 / Algorithm 2 through the cells, for a term set Q
 * of n terms. A cell b of repetition r is positive when its BFU holds every
 * term of Q (its Bloom test passes for each). Within a repetition the
 * documents of the positive cells are merged (a union: each document lies in
 * exactly one cell), and across repetitions only documents found in every
 * repetition remain (an intersection). Without terms every cell is
 * positive. With early_exit a cell's test stops at the first term it does
 * not hold, and no further repetition is examined once the remaining set is
 * empty: an intersection with an empty set stays empty (Section 3.3.1).
 * Returns the number of single-term Bloom tests performed. */
static uint64_t alg2(const orc_t *o, const uint64_t *Q, uint64_t n, uint64_t *out, int early_exit) {
    uint64_t tests = 0;
    uint8_t *positive = malloc(o->B);
    uint64_t *merged = malloc(o->W * 8);
    /* the remaining set starts as every document (bits >= K stay zero) */
    for (uint64_t w = 0; w < o->W; w++) out[w] = ~0ULL;
    if (o->K & 63) out[o->W - 1] = (1ULL << (o->K & 63)) - 1;
    for (uint32_t r = 0; r < o->R; r++) {
        for (uint32_t b = 0; b < o->B; b++) {
            const uint64_t *f = bfu(o, r, b);
            positive[b] = 1;
            for (uint64_t i = 0; i < n; i++) {
                tests++;
                if (!bf_test(o, r, f, Q[i])) {
                    positive[b] = 0;
                    if (early_exit) break;
                }
            }
        }
        /* union of the documents of the positive cells */
        memset(merged, 0, o->W * 8);
        const uint32_t *off = o->bucket_off + (size_t)r * (o->B + 1);
        const uint64_t *cell_docs = o->bucket_doc + (size_t)r * o->K;
        for (uint32_t b = 0; b < o->B; b++)
            if (positive[b])
                for (uint32_t k = off[b]; k < off[b + 1]; k++) setbit(merged, cell_docs[k]);
        /* intersection with what the earlier repetitions left */
        uint64_t left = 0;
        for (uint64_t w = 0; w < o->W; w++) {
            out[w] &= merged[w];
            left |= out[w];
        }
        if (early_exit && !left) break;
    }
    free(merged);
    free(positive);
    return tests;
}

void orc_query_kmer_alg2(const orc_t *o, uint64_t x, uint64_t *out) {
    uint64_t c = orc_canon(x);
    alg2(o, &c, 1, out, 0);
}

/* the canonical terms of a sequence, in order (duplicates kept) */
static uint64_t terms(const uint8_t *seq, uint64_t len, uint64_t *Q) {
    uint64_t n = 0;
    for (uint64_t p = 0; p + KMER <= len; p++)
        if (orc_window(seq, p, &Q[n])) n++;
    return n;
}

/* Definition mode for a sequence (Section 3.3.1): document d is reported iff
 * every term of the sequence is reported for d. */
void orc_query_seq_def(const orc_t *o, const uint8_t *seq, uint64_t len, uint64_t *out) {
    uint64_t *Q = malloc((len + 1) * 8);
    uint64_t n = terms(seq, len, Q);
    memset(out, 0, o->W * 8);
    for (uint64_t d = 0; d < o->K; d++) {
        int keep = 1;
        for (uint64_t i = 0; i < n && keep; i++)
            for (uint32_t r = 0; r < o->R && keep; r++)
                keep = bf_test(o, r, bfu(o, r, cell_of(o, r, d)), Q[i]);
        if (keep) setbit(out, d);
    }
    free(Q);
}

uint64_t orc_query_seq_alg2(const orc_t *o, const uint8_t *seq, uint64_t len, uint64_t *out, int early_exit) {
    uint64_t *Q = malloc((len + 1) * 8);
    uint64_t n = terms(seq, len, Q);
    uint64_t t = alg2(o, Q, n, out, early_exit);
    free(Q);
    return t;
}

/* batches, parallel over independent queries */
void orc_query_kmers(const orc_t *o, const uint64_t *xs, uint64_t n, uint64_t *out, int mode, int nthreads) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        if (mode == 0) orc_query_kmer_def(o, xs[i], out + (uint64_t)i * o->W);
        else orc_query_kmer_alg2(o, xs[i], out + (uint64_t)i * o->W);
    }
}

uint64_t orc_query_seqs(const orc_t *o, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                        uint64_t *out, int mode, int early_exit, int nthreads) {
    uint64_t tests = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : tests) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        const uint8_t *s = seqs + offsets[i];
        uint64_t len = offsets[i + 1] - offsets[i];
        if (mode == 0) orc_query_seq_def(o, s, len, out + (uint64_t)i * o->W);
        else tests += orc_query_seq_alg2(o, s, len, out + (uint64_t)i * o->W, early_exit);
    }
    return tests;
}

/* ---- opaque terms (document indexing with word terms, Section 5.4) --------- */
/* Documents as sets of opaque 64-bit terms (word ids): Algorithm 1 and the
 * queries of Section 3.3 with the terms taken as they are -- no k-mer
 * encoding, any 64-bit value is a term. */
int orc_insert_terms(orc_t *o, uint64_t d, const uint64_t *t, uint64_t n) {
    if (d >= o->K) return -1;
    for (uint32_t r = 0; r < o->R; r++) {
        uint64_t *f = bfu(o, r, cell_of(o, r, d));
        for (uint64_t i = 0; i < n; i++) bf_insert(o, r, f, t[i]);
    }
    return 0;
}

/* documents d0 .. d0+nd-1 with terms t[offs[k] .. offs[k+1]); each thread
 * owns whole BFUs (no two threads write one filter) */
int orc_build_term_docs(orc_t *o, const uint64_t *t, const uint64_t *offs, uint64_t d0, uint64_t nd, int nthreads) {
    if (d0 + nd > o->K) return -1;
    int64_t cells = (int64_t)o->R * o->B;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t c = 0; c < cells; c++) {
        uint32_t r = (uint32_t)(c / o->B), b = (uint32_t)(c % o->B);
        uint64_t *f = bfu(o, r, b);
        for (uint64_t k = 0; k < nd; k++) {
            if (cell_of(o, r, d0 + k) != b) continue;
            for (uint64_t i = offs[k]; i < offs[k + 1]; i++) bf_insert(o, r, f, t[i]);
        }
    }
    return 0;
}

/* Definition mode for a term set Q of n opaque terms (n = 1: one term):
 * document d is reported iff every term passes the Bloom test of
 * BFU(r, phi_r(d)) in every repetition r (Section 3.3, 3.3.1). */
void orc_query_termset_def(const orc_t *o, const uint64_t *Q, uint64_t n, uint64_t *out) {
    memset(out, 0, o->W * 8);
    for (uint64_t d = 0; d < o->K; d++) {
        int keep = 1;
        for (uint64_t i = 0; i < n && keep; i++)
            for (uint32_t r = 0; r < o->R && keep; r++) keep = bf_test(o, r, bfu(o, r, cell_of(o, r, d)), Q[i]);
        if (keep) setbit(out, d);
    }
}

/* Algorithm 2 for a term set of opaque terms */
uint64_t orc_query_termset_alg2(const orc_t *o, const uint64_t *Q, uint64_t n, uint64_t *out, int early_exit) {
    return alg2(o, Q, n, out, early_exit);
}

/* batches: single terms, and term sets t[offs[i] .. offs[i+1]) */
void orc_query_terms(const orc_t *o, const uint64_t *xs, uint64_t n, uint64_t *out, int mode, int nthreads) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        if (mode == 0) orc_query_termset_def(o, xs + i, 1, out + (uint64_t)i * o->W);
        else alg2(o, xs + i, 1, out + (uint64_t)i * o->W, 0);
    }
}

uint64_t orc_query_termsets(const orc_t *o, const uint64_t *t, const uint64_t *offs, uint64_t n, uint64_t *out,
                            int mode, int early_exit, int nthreads) {
    uint64_t tests = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : tests) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        const uint64_t *Q = t + offs[i];
        uint64_t len = offs[i + 1] - offs[i];
        if (mode == 0) orc_query_termset_def(o, Q, len, out + (uint64_t)i * o->W);
        else tests += alg2(o, Q, len, out + (uint64_t)i * o->W, early_exit);
    }
    return tests;
}

/* ---- folding over (Section 5.3, Figure 3) -------------------------------- */
/* BFU'(r, b) = BFU(r, b) OR BFU(r, b + B/2) for b < B/2; B must be even. The
 * folded index keeps R, m and the hash functions; a document's cell becomes
 * phi_r(d) mod (B/2). Returns a new oracle. */
orc_t *orc_fold(const orc_t *o) {
    if (o->B % 2 || !o->bits) return NULL;
    orc_t *f = orc_new(o->K, o->B, o->R, o->m, o->eta, o->seed, 0);
    f->B = o->B / 2;
    if (o->cells) {  /* an explicit partition folds the same way: cell mod B/2 */
        f->cells = malloc((size_t)f->R * f->K * sizeof(uint32_t));
        for (uint64_t i = 0; i < (uint64_t)f->R * f->K; i++) f->cells[i] = o->cells[i] % f->B;
    }
    f->bits = calloc((size_t)f->R * f->B * f->wpb, sizeof(uint64_t));
    for (uint32_t r = 0; r < o->R; r++)
        for (uint32_t b = 0; b < f->B; b++) {
            uint64_t *dst = f->bits + ((size_t)r * f->B + b) * f->wpb;
            const uint64_t *lo = bfu(o, r, b), *hi = bfu(o, r, b + f->B);
            for (uint64_t w = 0; w < f->wpb; w++) dst[w] = lo[w] | hi[w];
        }
    free(f->bucket_off); free(f->bucket_doc);
    /* cells of the folded index: phi_r(d) mod B/2 */
    f->bucket_off = calloc((size_t)f->R * (f->B + 1), sizeof(uint32_t));
    f->bucket_doc = malloc((size_t)f->R * f->K * sizeof(uint64_t));
    for (uint32_t r = 0; r < f->R; r++) {
        uint32_t *off = f->bucket_off + (size_t)r * (f->B + 1);
        for (uint64_t d = 0; d < f->K; d++) off[cell_of(o, r, d) % f->B + 1]++;
        for (uint32_t b = 0; b < f->B; b++) off[b + 1] += off[b];
        uint32_t *fill = calloc(f->B, sizeof(uint32_t));
        for (uint64_t d = 0; d < f->K; d++) {
            uint32_t b = cell_of(o, r, d) % f->B;
            f->bucket_doc[(size_t)r * f->K + off[b] + fill[b]++] = d;
        }
        free(fill);
    }
    return f;
}

/* the cell of every document in every repetition: out[r * K + d] */
void orc_cells(const orc_t *o, uint32_t *out) {
    for (uint32_t r = 0; r < o->R; r++)
        for (uint64_t d = 0; d < o->K; d++) out[(size_t)r * o->K + d] = cell_of(o, r, d);
}

/* cell of document d in repetition r as this oracle's index sees it */
uint32_t orc_cell(const orc_t *o, uint32_t r, uint64_t d) {
    const uint32_t *off = o->bucket_off + (size_t)r * (o->B + 1);
    for (uint32_t b = 0; b < o->B; b++)
        for (uint32_t k = off[b]; k < off[b + 1]; k++)
            if (o->bucket_doc[(size_t)r * o->K + k] == d) return b;
    return (uint32_t)-1;
}
