/*
 * Seeded synthetic inputs: genomes, reads and k-mer queries.
 *
 * This module is input plumbing only. It holds none of the indexing method's
 * arithmetic (no canonical form, no hashing, no Bloom filter). It is shared by
 * the tests, the benchmark and the CPU oracle so that every side sees the same
 * bytes; nothing here is linked into the GPU library.
 *
 * Every value is a pure function of (seed, tag, index): any document base, any
 * read or any query can be regenerated on its own, in any order, by any thread.
 *
 * Randomness: the SplitMix64 output function ("fmix" below; Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) used
 * as a counter-based generator, keyed by a two-input mix H(a, b).
 *
 * Workload shape (the paper's genomic setting, scaled down): documents are
 * related genomes, mutated copies of a few random ancestors, over the ACGT
 * alphabet; queries are 31-mers or reads of a few hundred bases.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

enum { TAG_ANC = 1, TAG_DOC = 2, TAG_READ = 3, TAG_KQ = 4 };

static const char BASES[4] = {'A', 'C', 'G', 'T'};

static inline uint64_t fmix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* SplitMix64 sequential generator: exposed so tests can check the published
 * reference outputs of the function this module is keyed with. */
uint64_t gen_splitmix64_next(uint64_t *state) {
    *state += GAMMA;
    return fmix(*state);
}

static inline uint64_t H(uint64_t a, uint64_t b) { return fmix(a ^ fmix(b + GAMMA)); }

static inline uint64_t key(uint64_t seed, uint64_t tag, uint64_t idx) {
    return H(H(seed, tag), idx);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double unit53(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }

/* probability threshold on the top 53 bits: event iff (v >> 11) < thr */
static inline uint64_t thr53(double p) {
    if (p <= 0.0) return 0;
    if (p >= 1.0) return 1ULL << 53;
    return (uint64_t)(p * 0x1.0p53);
}

/* ------------------------------------------------------------------------ */
/* Documents                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t seed;         /* data seed */
    uint64_t len;          /* bases per document */
    uint64_t docs_per_anc; /* documents sharing one ancestor */
    double mu_lo, mu_hi;   /* per-document substitution rate, uniform in [lo, hi] */
} docmodel_t;

static inline int anc_base(const docmodel_t *m, uint64_t anc, uint64_t i) {
    uint64_t w = H(key(m->seed, TAG_ANC, anc), i >> 5);
    return (int)((w >> ((i & 31) * 2)) & 3);
}

static inline uint64_t doc_key(const docmodel_t *m, uint64_t d) { return key(m->seed, TAG_DOC, d); }

static inline uint64_t doc_thr(const docmodel_t *m, uint64_t kd) {
    double mu = m->mu_lo + (m->mu_hi - m->mu_lo) * unit53(H(kd, ~0ULL));
    return thr53(mu);
}

/* base (0..3) of document d at position i */
static inline int doc_base_k(const docmodel_t *m, uint64_t d, uint64_t kd, uint64_t t, uint64_t i) {
    uint64_t anc = d / m->docs_per_anc;
    int b = anc_base(m, anc, i);
    if (t) {
        uint64_t v = H(kd, i);
        if ((v >> 11) < t) b = (b + 1 + (int)((v & 0xFFFFFFFFULL) % 3)) & 3;
    }
    return b;
}

static void fill_doc(const docmodel_t *m, uint64_t d, uint64_t start, uint64_t n, char *out) {
    uint64_t kd = doc_key(m, d), t = doc_thr(m, kd);
    uint64_t anc = d / m->docs_per_anc, ka = key(m->seed, TAG_ANC, anc);
    uint64_t i = start, end = start + n;
    while (i < end) {
        uint64_t w = H(ka, i >> 5);
        uint64_t stop = ((i >> 5) + 1) << 5;
        if (stop > end) stop = end;
        for (; i < stop; i++) {
            int b = (int)((w >> ((i & 31) * 2)) & 3);
            if (t) {
                uint64_t v = H(kd, i);
                if ((v >> 11) < t) b = (b + 1 + (int)((v & 0xFFFFFFFFULL) % 3)) & 3;
            }
            out[i - start] = BASES[b];
        }
    }
}

/* Bases [start, start+n) of document d, as ASCII "ACGT". */
void gen_doc(uint64_t seed, uint64_t len, uint64_t dpa, double mu_lo, double mu_hi, uint64_t d,
             uint64_t start, uint64_t n, char *out) {
    docmodel_t m = {seed, len, dpa ? dpa : 1, mu_lo, mu_hi};
    fill_doc(&m, d, start, n, out);
}

/* nd whole documents d0 .. d0+nd-1, concatenated (each len bytes). */
void gen_docs(uint64_t seed, uint64_t len, uint64_t dpa, double mu_lo, double mu_hi, uint64_t d0,
              uint64_t nd, char *out, int nthreads) {
    docmodel_t m = {seed, len, dpa ? dpa : 1, mu_lo, mu_hi};
    /* split long documents into blocks so few documents still use every thread */
    const uint64_t blk = 1ULL << 16;
    uint64_t per = (len + blk - 1) / blk, total = nd * per;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t t = 0; t < (int64_t)total; t++) {
        uint64_t di = (uint64_t)t / per, b = (uint64_t)t % per;
        uint64_t s = b * blk, n = (s + blk <= len) ? blk : len - s;
        fill_doc(&m, d0 + di, s, n, out + di * len + s);
    }
}

/* The 2-bit code of every length-k window of document d, in generator order
 * (window at position p, first base in the two most significant bits,
 * A=0 C=1 G=2 T=3). This is the generator's own k-mer format for feeding
 * k-mer level inputs; it is not canonical. */
void gen_doc_window_codes(uint64_t seed, uint64_t len, uint64_t dpa, double mu_lo, double mu_hi,
                          uint64_t d, uint32_t k, uint64_t *out) {
    docmodel_t m = {seed, len, dpa ? dpa : 1, mu_lo, mu_hi};
    if (len < k) return;
    uint64_t kd = doc_key(&m, d), t = doc_thr(&m, kd);
    uint64_t mask = (k >= 32) ? ~0ULL : ((1ULL << (2 * k)) - 1);
    uint64_t code = 0;
    for (uint64_t i = 0; i < len; i++) {
        code = ((code << 2) | (uint64_t)doc_base_k(&m, d, kd, t, i)) & mask;
        if (i + 1 >= k) out[i + 1 - k] = code;
    }
}

/* ------------------------------------------------------------------------ */
/* Single k-mer queries: a fraction present (a window of a random document),  */
/* the rest fresh random 62-bit codes.                                        */
/* ------------------------------------------------------------------------ */
void gen_kmer_queries(uint64_t seed, uint64_t len, uint64_t dpa, double mu_lo, double mu_hi,
                      uint64_t n_docs, uint64_t qseed, double frac_present, uint32_t k, uint64_t n,
                      uint64_t *out, int64_t *src_doc, int nthreads) {
    docmodel_t m = {seed, len, dpa ? dpa : 1, mu_lo, mu_hi};
    uint64_t tp = thr53(frac_present);
    uint64_t mask = (k >= 32) ? ~0ULL : ((1ULL << (2 * k)) - 1);
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t q = 0; q < (int64_t)n; q++) {
        uint64_t kq = key(qseed, TAG_KQ, (uint64_t)q);
        if ((H(kq, 0) >> 11) < tp && len >= k) {
            uint64_t d = H(kq, 1) % n_docs, p = H(kq, 2) % (len - k + 1);
            uint64_t kd = doc_key(&m, d), t = doc_thr(&m, kd), c = 0;
            for (uint32_t i = 0; i < k; i++) c = (c << 2) | (uint64_t)doc_base_k(&m, d, kd, t, p + i);
            out[q] = c;
            if (src_doc) src_doc[q] = (int64_t)d;
        } else {
            out[q] = H(kq, 3) & mask;
            if (src_doc) src_doc[q] = -1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Reads                                                                      */
/* ------------------------------------------------------------------------ */
/* Length model: kind 0 = log-normal, round(median * exp(sigma * Z)), clipped
 * to [lo, hi]; kind 1 = uniform integer in [lo, hi]. */
typedef struct {
    uint64_t qseed;
    uint64_t src_lo, src_hi; /* documents reads are drawn from: [src_lo, src_hi) */
    double frac_doc;         /* fraction of reads copied from a document */
    int len_kind;
    double median, sigma;
    uint64_t lo, hi;
    double err_lo, err_hi; /* per-read substitution error rate, uniform in [lo, hi] */
} readmodel_t;

static uint64_t read_len(const readmodel_t *r, uint64_t kr, uint64_t doc_len) {
    uint64_t L;
    if (r->len_kind == 0) {
        double u1 = ((double)(H(kr, 2) >> 11) + 1.0) * 0x1.0p-53; /* (0, 1] */
        double u2 = unit53(H(kr, 3));
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
        double x = r->median * exp(r->sigma * z);
        if (x < (double)r->lo) x = (double)r->lo;
        if (x > (double)r->hi) x = (double)r->hi;
        L = (uint64_t)llround(x);
    } else {
        L = r->lo + H(kr, 2) % (r->hi - r->lo + 1);
    }
    if (doc_len && L > doc_len) L = doc_len;
    return L;
}

static void rm_init(readmodel_t *r, uint64_t qseed, uint64_t src_lo, uint64_t src_hi, double frac_doc,
                    int len_kind, double median, double sigma, uint64_t lo, uint64_t hi, double err_lo,
                    double err_hi) {
    r->qseed = qseed; r->src_lo = src_lo; r->src_hi = src_hi; r->frac_doc = frac_doc;
    r->len_kind = len_kind; r->median = median; r->sigma = sigma; r->lo = lo; r->hi = hi;
    r->err_lo = err_lo; r->err_hi = err_hi;
}

/* Pass 1: offsets[0..n] of reads i0 .. i0+n-1 (offsets[0] = 0). */
void gen_read_offsets(uint64_t seed, uint64_t len, uint64_t qseed, uint64_t src_lo, uint64_t src_hi,
                      double frac_doc, int len_kind, double median, double sigma, uint64_t lo,
                      uint64_t hi, double err_lo, double err_hi, uint64_t i0, uint64_t n,
                      uint64_t *offsets) {
    readmodel_t r;
    rm_init(&r, qseed, src_lo, src_hi, frac_doc, len_kind, median, sigma, lo, hi, err_lo, err_hi);
    (void)seed;
    offsets[0] = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t kr = key(qseed, TAG_READ, i0 + i);
        offsets[i + 1] = offsets[i] + read_len(&r, kr, len);
    }
}

/* Pass 2: the read bytes, and per read its source document (-1 if random),
 * start position, number of substitution errors and strand (1 = reverse
 * complement). Any of the metadata pointers may be NULL. */
void gen_read_fill(uint64_t seed, uint64_t len, uint64_t dpa, double mu_lo, double mu_hi, uint64_t qseed,
                   uint64_t src_lo, uint64_t src_hi, double frac_doc, int len_kind, double median,
                   double sigma, uint64_t lo, uint64_t hi, double err_lo, double err_hi, uint64_t i0,
                   uint64_t n, const uint64_t *offsets, char *out, int64_t *src, int64_t *start,
                   int64_t *nerr, int8_t *rc, int nthreads) {
    docmodel_t m = {seed, len, dpa ? dpa : 1, mu_lo, mu_hi};
    readmodel_t r;
    rm_init(&r, qseed, src_lo, src_hi, frac_doc, len_kind, median, sigma, lo, hi, err_lo, err_hi);
    uint64_t tdoc = thr53(frac_doc);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t ii = 0; ii < (int64_t)n; ii++) {
        uint64_t i = (uint64_t)ii;
        uint64_t kr = key(qseed, TAG_READ, i0 + i);
        uint64_t L = offsets[i + 1] - offsets[i];
        char *o = out + offsets[i];
        int64_t s_src = -1, s_start = -1, s_err = 0;
        int8_t s_rc = 0;
        if ((H(kr, 0) >> 11) < tdoc && src_hi > src_lo && len >= L) {
            uint64_t d = src_lo + H(kr, 1) % (src_hi - src_lo);
            uint64_t st = H(kr, 4) % (len - L + 1);
            fill_doc(&m, d, st, L, o);
            double e = r.err_lo + (r.err_hi - r.err_lo) * unit53(H(kr, 5));
            uint64_t te = thr53(e);
            if (te) {
                for (uint64_t p = 0; p < L; p++) {
                    uint64_t v = H(kr, 16 + p);
                    if ((v >> 11) < te) {
                        int b = 0;
                        switch (o[p]) { case 'A': b = 0; break; case 'C': b = 1; break;
                                        case 'G': b = 2; break; default: b = 3; }
                        o[p] = BASES[(b + 1 + (int)((v & 0xFFFFFFFFULL) % 3)) & 3];
                        s_err++;
                    }
                }
            }
            s_rc = (int8_t)(H(kr, 6) & 1);
            if (s_rc) {
                for (uint64_t a = 0, b = L ? L - 1 : 0; a < b; a++, b--) {
                    char t = o[a]; o[a] = o[b]; o[b] = t;
                }
                for (uint64_t p = 0; p < L; p++) {
                    switch (o[p]) { case 'A': o[p] = 'T'; break; case 'C': o[p] = 'G'; break;
                                    case 'G': o[p] = 'C'; break; default: o[p] = 'A'; }
                }
            }
            s_src = (int64_t)d; s_start = (int64_t)st;
        } else {
            for (uint64_t p = 0; p < L; p++) {
                uint64_t w = H(kr, (1ULL << 40) | (p >> 5));
                o[p] = BASES[(w >> ((p & 31) * 2)) & 3];
            }
        }
        if (src) src[i] = s_src;
        if (start) start[i] = s_start;
        if (nerr) nerr[i] = s_err;
        if (rc) rc[i] = s_rc;
    }
}

/* Poisson arrival times (seconds) for an open-loop request stream of rate
 * lam: exponential gaps drawn by inversion. */
void gen_poisson_arrivals(uint64_t aseed, double lam, uint64_t n, double *t_out) {
    double t = 0.0;
    for (uint64_t i = 0; i < n; i++) {
        double u = ((double)(H(key(aseed, 5, 0), i) >> 11) + 1.0) * 0x1.0p-53;
        t += -log(u) / lam;
        t_out[i] = t;
    }
}

/* ------------------------------------------------------------------------ */
/* Word-term documents (the web-document setting: a document is a set of     */
/* word unigrams). A vocabulary of V words with Zipf(s) frequencies, word w  */
/* ranked w (0 most frequent); word w's term id is a 64-bit key of (seed, w), */
/* standing for the hash of the token. Document d draws n_d words, n_d       */
/* uniform in [mean/2, 3 mean/2], by inverse-CDF sampling of the Zipf law;  */
/* term i of document d depends on (seed, d, i) only. Repeated words are     */
/* kept (documents are sets downstream).                                     */
/* ------------------------------------------------------------------------ */
enum { TAG_TERM = 6, TAG_TDOC = 7, TAG_TQ = 8, TAG_TP = 9 };

uint64_t gen_term_id(uint64_t seed, uint64_t w) { return key(seed, TAG_TERM, w); }

uint64_t gen_term_doc_len(uint64_t seed, uint64_t mean, uint64_t d) {
    uint64_t lo = mean / 2, span = mean + 1; /* [mean/2, mean/2 + mean] */
    return lo + H(key(seed, TAG_TDOC, d), ~0ULL) % span;
}

/* cdf[w] = sum_{v <= w} (v+1)^-s / Z, w < V */
void gen_zipf_cdf(uint64_t V, double s, double *cdf) {
    double z = 0.0;
    for (uint64_t w = 0; w < V; w++) z += pow((double)(w + 1), -s);
    double acc = 0.0;
    for (uint64_t w = 0; w < V; w++) {
        acc += pow((double)(w + 1), -s) / z;
        cdf[w] = acc;
    }
    cdf[V - 1] = 1.0;
}

static inline uint64_t zipf_draw(const double *cdf, uint64_t V, uint64_t v) {
    double u = unit53(v);
    uint64_t lo = 0, hi = V - 1; /* smallest w with cdf[w] > u */
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > u) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

static inline uint64_t term_of(uint64_t seed, const double *cdf, uint64_t V, uint64_t d, uint64_t i) {
    return gen_term_id(seed, zipf_draw(cdf, V, H(key(seed, TAG_TDOC, d), i)));
}

/* documents d0 .. d0+nd-1: document d0+k's terms at out[offs[k] .. offs[k+1]) */
void gen_term_docs(uint64_t seed, uint64_t V, const double *cdf, uint64_t d0, uint64_t nd, const uint64_t *offs,
                   uint64_t *out, int nthreads) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t k = 0; k < (int64_t)nd; k++)
        for (uint64_t i = 0; i < offs[k + 1] - offs[k]; i++) out[offs[k] + i] = term_of(seed, cdf, V, d0 + k, i);
}

/* single-term queries: a fraction present (a random term of a random
 * document, source returned), the rest fresh random 64-bit values (-1) */
void gen_term_queries(uint64_t seed, uint64_t V, const double *cdf, uint64_t mean, uint64_t n_docs,
                      uint64_t qseed, double frac_present, uint64_t n, uint64_t *out, int64_t *src, int nthreads) {
    uint64_t tp = thr53(frac_present);
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t q = 0; q < (int64_t)n; q++) {
        uint64_t kq = key(qseed, TAG_TQ, (uint64_t)q);
        if ((H(kq, 0) >> 11) < tp) {
            uint64_t d = H(kq, 1) % n_docs, len = gen_term_doc_len(seed, mean, d);
            out[q] = term_of(seed, cdf, V, d, H(kq, 2) % len);
            if (src) src[q] = (int64_t)d;
        } else {
            out[q] = H(kq, 3);
            if (src) src[q] = -1;
        }
    }
}

/* phrase queries (term sets): query q has len_q terms, len_q uniform in
 * [lo, hi]; a fraction are consecutive terms of a random document (source
 * returned), the rest terms of random documents mixed (source -1). Lengths
 * first (gen_term_phrase_lens), then the terms at out[offs[q] ..]. */
void gen_term_phrase_lens(uint64_t qseed, uint64_t lo, uint64_t hi, uint64_t n, uint64_t *lens) {
    for (uint64_t q = 0; q < n; q++) lens[q] = lo + H(key(qseed, TAG_TP, q), 0) % (hi - lo + 1);
}

void gen_term_phrases(uint64_t seed, uint64_t V, const double *cdf, uint64_t mean, uint64_t n_docs, uint64_t qseed,
                      double frac_doc, uint64_t n, const uint64_t *offs, uint64_t *out, int64_t *src, int nthreads) {
    uint64_t tp = thr53(frac_doc);
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t q = 0; q < (int64_t)n; q++) {
        uint64_t kq = key(qseed, TAG_TP, (uint64_t)q), len = offs[q + 1] - offs[q];
        if ((H(kq, 1) >> 11) < tp) {
            uint64_t d = H(kq, 2) % n_docs, dl = gen_term_doc_len(seed, mean, d);
            uint64_t start = dl > len ? H(kq, 3) % (dl - len + 1) : 0;
            for (uint64_t i = 0; i < len; i++) out[offs[q] + i] = term_of(seed, cdf, V, d, (start + i) % dl);
            if (src) src[q] = (int64_t)d;
        } else {
            for (uint64_t i = 0; i < len; i++) {
                uint64_t d = H(kq, 10 + 2 * i) % n_docs, dl = gen_term_doc_len(seed, mean, d);
                out[offs[q] + i] = term_of(seed, cdf, V, d, H(kq, 11 + 2 * i) % dl);
            }
            if (src) src[q] = -1;
        }
    }
}
