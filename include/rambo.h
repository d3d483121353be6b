/*
 * rambo.h -- C ABI of librambo.so, a RAMBO index (Repeated And Merged BloOm
 * filter; Gupta et al., SIGMOD 2021) resident in the HBM of one AMD Instinct
 * MI355X (gfx950).
 *
 * The index is an R x B array of Bloom filters of m bits ("BFUs", Section 3):
 * document d belongs to BFU(r, phi_r(d)) in each repetition r; BFU(r, b) is
 * the Bloom filter (Section 2.1) of the union of the k-mer sets of its
 * documents. Terms are canonical 31-mers (Section 5.1). A query term is
 * reported for d iff BFU(r, phi_r(d)) passes its Bloom test in every
 * repetition (Section 3.3, Algorithm 2); a sequence query ANDs the answers of
 * all its terms (Section 3.3.1).
 *
 * Conventions shared by every entry point:
 *  - k = 31. A k-mer value is a 2-bit code, A=0 C=1 G=2 T=3, first base in
 *    the two most significant of the 62 low bits; values >= 4^31 are not
 *    k-mers. The library canonicalises every value it is given
 *    (min(code, reverse complement)), so either strand may be passed.
 *  - Sequences are bytes; A/C/G/T in either case are bases; a window of 31
 *    bytes holding any other byte is not a term and is skipped.
 *  - Results are K-bit bitsets of W = ceil(K / 64) uint64 words per query:
 *    document d is bit (d & 63) of word (d >> 6); bits >= K are zero.
 *  - Hash functions (fixed by definition, shared with no other code): with P
 *    = 2^61 - 1 and SplitMix64 seeded by `seed`, drawn in the order below,
 *      phi_r(d)    = ((a_r d + b_r) mod P) mod B           (Carter-Wegman)
 *      h_{r,j}(x)  = floor(m * hi64((A_{r,j} x + C_{r,j}) mod 2^128) / 2^64)
 *    where for r < R: a_r = 1 + next mod (P - 1), b_r = next mod P; then for
 *    r < R, j < eta: A = next | next << 64 (low word first), C likewise.
 *  - Pointers named "device" are HIP device pointers (e.g. torch tensors on
 *    the GPU); `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream). Entry points that take a stream only enqueue work and return;
 *    the caller orders them (same stream, or events). Device buffers stay
 *    owned by the caller and must stay valid until the enqueued work ends.
 *  - Every entry point returns a status (RAMBO_OK = 0, negative on error)
 *    and records a message readable with rambo_last_error() on the calling
 *    thread. Errors detected on the GPU (invalid k-mer values in a device
 *    batch) are counted and reported by the next rambo_sync(), and so are
 *    queries that hold no term (RAMBO_OK_EMPTYQ, not an error).
 *  - Queries may run concurrently on one handle. Insertions and queries must
 *    be ordered by the caller; a query that overlaps an insertion is
 *    unsupported. Batched-form queries with the same (seqs, offsets, n, out)
 *    share one captured graph and its work-queue state, so calls that
 *    overlap in time need distinct output buffers (they would write the same
 *    output anyway).
 */
#ifndef RAMBO_H
#define RAMBO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rambo_s rambo_t;

enum {
    RAMBO_OK = 0,
    RAMBO_OK_EMPTYQ = 1, /* success; some query held no term (a read with no
                            valid 31-window, an empty term set) and was
                            answered with every document, the vacuous
                            "every term of Q is in the BFU" of Algorithm 2 */
    RAMBO_EINVAL = -1,  /* bad argument or invalid k-mer value */
    RAMBO_ENOMEM = -2,  /* device or host allocation failed */
    RAMBO_EDEVICE = -3, /* HIP runtime error */
    RAMBO_ETRUNC = -4,  /* id output too small (see rambo_query_seqs_ids) */
    RAMBO_EBUSY = -5,   /* server queue full / admission refused */
    RAMBO_EIO = -6,     /* index file: open, read or write failed, or not a
                           valid index file (see rambo_save) */
};

/* Query execution forms for rambo_query_seqs. */
enum {
    RAMBO_MODE_PLAIN = 0,   /* one launch, one wavefront per read */
    RAMBO_MODE_BATCHED = 1, /* persistent launch over (read, k-mer tile) work
                               items, replayed from a captured HIP graph */
};

/* Resolve strategies (Section 3.3, Algorithm 2: union of the documents of
 * positive BFUs per repetition, intersection across repetitions). */
enum {
    RAMBO_RESOLVE_AUTO = 0,      /* pick per query from the cell sizes */
    RAMBO_RESOLVE_DENSE = 1,     /* every document d tests its R cells */
    RAMBO_RESOLVE_CANDIDATE = 2, /* documents of positive repetition-0 cells
                                    are tested in the other repetitions */
};

/* Limits: 1 <= R <= 8, 1 <= eta <= 16, 1 <= B <= 8192, 1 <= K < 2^32,
 * 1 <= m <= 2^40. R and B are bounded by the layout: a document's cells are
 * one 16-byte record (R 16-bit slots), and a query keeps R masks of B bits
 * per wave in LDS while a row of B bits is read by at most 64 lanes x 16
 * bytes in one load instruction. */
#define RAMBO_MAX_R 8
#define RAMBO_MAX_ETA 16
#define RAMBO_MAX_B 8192

/* ---------------------------------------------------------------------- */
/* Lifetime and errors                                                     */
/* ---------------------------------------------------------------------- */

/* Allocate an empty index of K documents (ids 0..K-1; K is the capacity, so
 * documents can be added later: insertion into a built index, Section 3.2), R
 * repetitions of B BFUs of m bits each, eta Bloom hash functions, on the
 * current HIP device. The index is a bit-sliced array rows[R][m] of B-bit
 * rows, each padded to a power of two >= 32 bits, zeroed. Returns NULL on
 * error (RAMBO_EINVAL for out-of-range parameters, RAMBO_ENOMEM if the
 * device cannot hold the index); see rambo_last_error(). The handle owns all
 * its device memory. */
rambo_t *rambo_create(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed);

enum {
    RAMBO_TERMS_OPAQUE = 1, /* creation flag: documents are sets of opaque terms */
    RAMBO_SHARD = 2,        /* reported by rambo_layout (and kept in index
                               files) for an index made by rambo_create_shard */
};

/* As rambo_create, with flags. RAMBO_TERMS_OPAQUE: an index of documents
 * given as sets of opaque 64-bit terms (word ids; the document indexing of
 * Section 5.4) instead of 31-mers: rambo_insert, rambo_insert_batch,
 * rambo_query_kmers and rambo_query_term_sets take the values as they are
 * (no k-mer encoding, no range check: every 64-bit value is a term), and the
 * sequence entry points (rambo_insert_seqs, rambo_query_seqs,
 * rambo_query_seqs_ids, rambo_server_start) return RAMBO_EINVAL. Unknown
 * flags: RAMBO_EINVAL. */
rambo_t *rambo_create_ex(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                         uint32_t flags);

/* Free the index and everything the handle owns. NULL-safe. Waits for the
 * handle's own outstanding work. */
void rambo_destroy(rambo_t *h);

/* Message and status of the last failing call on this thread. */
const char *rambo_last_error(void);
int rambo_last_status(void);

/* Wait for all work the handle enqueued on `stream` (NULL: the null stream)
 * and report what the GPU counted since the previous call: RAMBO_EINVAL if
 * any k-mer value >= 4^31 (or document id >= K) was skipped by an insertion
 * or answered with an empty result by a query; otherwise RAMBO_OK_EMPTYQ if
 * a sequence or term-set query (rambo_query_seqs, rambo_query_term_sets, the
 * server's batches) held no term; otherwise RAMBO_OK. The counters belong to
 * the handle: work on other streams that ran meanwhile is counted too. */
int rambo_sync(rambo_t *h, void *stream);

/* ---------------------------------------------------------------------- */
/* Introspection                                                           */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint64_t K, m, seed;
    uint32_t B, R, eta;
    uint32_t row_words;  /* 32-bit words per row: power of two >= ceil(B/32) */
    uint64_t W;          /* result words per query */
    uint64_t index_bytes;/* R * m * row_words * 4 */
    void *rows;          /* device pointer to rows[R][m][row_words] (uint32) */
    uint32_t flags;      /* creation flags (RAMBO_TERMS_OPAQUE) */
} rambo_layout_t;

int rambo_layout(const rambo_t *h, rambo_layout_t *out);
uint64_t rambo_result_words(const rambo_t *h);
uint64_t rambo_index_bytes(const rambo_t *h);

/* The derived hash parameters (host arrays: pa, pb of R entries; Alo, Ahi,
 * Clo, Chi of R*eta entries, index r*eta + j). */
int rambo_hash_params(const rambo_t *h, uint64_t *pa, uint64_t *pb, uint64_t *Alo, uint64_t *Ahi,
                      uint64_t *Clo, uint64_t *Chi);

/* phi_r(d) for every r < R, d < K into a host array phi[r * K + d]. */
int rambo_phi_table(const rambo_t *h, uint32_t *phi);

/* BFU(r, b) as a plain m-bit Bloom filter: bit p of host word out[p / 64]
 * (ceil(m/64) words) is the bit of cell b in row p of repetition r.
 * Synchronous. */
int rambo_dump_bfu(rambo_t *h, uint32_t r, uint32_t b, uint64_t *out);

/* Copy `bytes` bytes of the raw row array, starting at byte `offset`, to the
 * host buffer `dst`. Synchronous. */
int rambo_copy_rows(rambo_t *h, uint64_t offset, uint64_t bytes, void *dst);

/* Index files: the index is built once and queried many times (Section 5.3
 * builds shards on many nodes and queries the stored indexes). rambo_save
 * writes a 96-byte little-endian header -- magic "RAMBOIX1", format version
 * 1, header size, K, m, seed, row array bytes, checksum, B, R, eta, flags,
 * row_words -- and then the raw row array (rows[R][m][row_words], uint32), so
 * the file is rambo_index_bytes + 96 bytes. The hash functions are not
 * stored: they are derived from (seed, B, R, eta, m) as at creation (a folded
 * index is stored with its folded B, which derives the folded partition).
 * The checksum covers the row array (computed on the device) and the
 * header's parameters; rambo_load recomputes it after the upload. Rows stream through two pinned host
 * buffers of 64 MiB, copies overlapping file I/O. Both are synchronous and
 * must not overlap an insert on the same handle.
 * rambo_save: RAMBO_EINVAL on a null argument, RAMBO_EIO if the file cannot
 * be written (a partial file may remain), RAMBO_EDEVICE/ENOMEM on runtime
 * errors.
 * rambo_load: a new handle on the current device, or NULL with
 * rambo_last_status() = RAMBO_EIO for a missing, short, foreign or corrupted
 * file (bad magic, version, sizes or checksum), RAMBO_EINVAL for parameters
 * out of range, RAMBO_ENOMEM if the device cannot hold the index. */
int rambo_save(rambo_t *h, const char *path);
rambo_t *rambo_load(const char *path);

/* ---------------------------------------------------------------------- */
/* Sharding by document (Section 5.3, Figure 3)                            */
/* ---------------------------------------------------------------------- */

/* Routing: shard[i] = tau(doc_ids[i]) = ((a d + b) mod P) mod G, with P =
 * 2^61 - 1, a = 1 + x0 mod (P - 1), b = x1 mod P for the first two outputs
 * x0, x1 of SplitMix64 seeded with route_seed -- a random (2-universal for
 * ids below P) hash of the document id picking one of G shards. Device
 * arrays (n ids, n outputs); enqueued on `stream`. RAMBO_EINVAL if G = 0. */
int rambo_route(const uint64_t *doc_ids, uint64_t n, uint32_t G, uint64_t route_seed, uint32_t *shard,
                void *stream);

/* A shard: an index of K local documents (local ids 0..K-1) where local
 * document l stands for global document global_ids[l] (host array of K
 * ids, copied). Everything is as rambo_create with (K, B, R, m, eta, seed)
 * except the cells: local document l lies in cell phi_r(global_ids[l]) of
 * repetition r, the node-local partition of the global id. G shards made
 * with the same (B, R, m, eta, seed) over the documents routed to them
 * (rambo_route) are, stacked, the index built directly with the two-level
 * partition B * tau(d) + phi_r(d) over G * B cells: a document's answer is
 * its answer in its own shard, which answers with a K-bit row over its
 * local ids (rambo_stack_slice puts it back at the global ids). Inserts and
 * queries take local ids. rambo_save keeps the ids (RAMBO_SHARD in the file
 * header, the K ids after it) and rambo_load restores them. Errors as
 * rambo_create; RAMBO_EINVAL for a null global_ids. */
rambo_t *rambo_create_shard(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                            const uint64_t *global_ids);

/* The global ids of a shard's local documents (host array of K words). */
int rambo_shard_ids(const rambo_t *h, uint64_t *out);

/* Stacking: for every query i < n and every local document l set in
 * slice[i * W + (l >> 6)] (the shard's answer rows, device, W =
 * rambo_result_words of the shard), set bit global_ids[l] of row i of out
 * (device, n rows of out_words words). ORs into out, which the caller zeroes
 * before stacking the first shard; the shards of one partition own disjoint
 * documents, so any order of shards gives the same rows. Enqueued on
 * `stream`. RAMBO_EINVAL if h is not a shard or a global id does not fit
 * out_words. */
int rambo_stack_slice(rambo_t *h, const uint64_t *slice, uint64_t n, uint64_t *out, uint64_t out_words,
                      void *stream);

/* ---------------------------------------------------------------------- */
/* Construction (Algorithm 1)                                              */
/* ---------------------------------------------------------------------- */

/* Insert document doc_id given n k-mer values (host array, either strand,
 * duplicates allowed). Every term goes into BFU(r, phi_r(doc_id)) for every
 * r. Synchronous. RAMBO_EINVAL (and nothing inserted) if doc_id >= K or any
 * value >= 4^31. Inserting twice is harmless (bits are ORed). */
int rambo_insert(rambo_t *h, uint64_t doc_id, const uint64_t *kmers, uint64_t n);

/* Insert n_docs documents from device arrays: document i has id doc_ids[i]
 * and k-mers kmers[kmer_offsets[i] .. kmer_offsets[i+1]) (offsets
 * non-decreasing, n_docs+1 entries). Enqueued on `stream`. Values >= 4^31 are
 * skipped and reported by rambo_sync(); ids >= K are skipped likewise. */
int rambo_insert_batch(rambo_t *h, const uint64_t *doc_ids, const uint64_t *kmer_offsets,
                       const uint64_t *kmers, uint64_t n_docs, void *stream);

/* Insert n_docs documents given as sequences (device arrays): document i has
 * id doc_ids[i] and bytes seqs[offsets[i] .. offsets[i+1]); its terms are its
 * valid 31-windows (Figure 1). Extraction runs on the GPU. Enqueued on
 * `stream`. */
int rambo_insert_seqs(rambo_t *h, const uint64_t *doc_ids, const uint8_t *seqs,
                      const uint64_t *offsets, uint64_t n_docs, void *stream);

/* Folding over (Section 5.3, Figure 3): OR the BFUs of cells B/2 .. B-1 onto
 * cells 0 .. B/2-1 in every repetition, leaving an index of B/2 cells with the
 * same R, m and hash functions (a document's cell becomes phi_r(d) mod B/2),
 * the same as building with B/2 cells directly. B must be even. Smaller and
 * faster, with a higher false-positive rate. Allocates the folded rows before
 * freeing the old ones (needs the folded size free), synchronous; resets the
 * batched form's launch shape. */
int rambo_fold(rambo_t *h);

/* ---------------------------------------------------------------------- */
/* Queries (Algorithm 2, Section 3.3.1)                                    */
/* ---------------------------------------------------------------------- */

/* n single k-mer queries (device array). out (device, n * W words) receives
 * one K-bit result per query. A value >= 4^31 gets an empty result and is
 * reported by rambo_sync(). Plain one-batch kernel. Enqueued on `stream`.
 * With a NULL stream, kmers and out may instead both be host arrays: they
 * are then copied in and out through device buffers the call allocates and
 * frees, and the call returns when out holds the results (RAMBO_EINVAL if one
 * array is on the host and the other on the device). */
int rambo_query_kmers(rambo_t *h, const uint64_t *kmers, uint64_t n, uint64_t *out, void *stream);

/* n sequence queries: read i is seqs[offsets[i] .. offsets[i+1]) (device
 * arrays; offsets non-decreasing; a read holds fewer than 2^32 bytes, the
 * kernels' window arithmetic within a read being 32-bit). out (device,
 * n * W words) receives, per
 * read, the documents that hold every term of the read. A read with no valid
 * window gets every document (the vacuous "every term is in the BFU" of
 * Algorithm 2) and is counted for rambo_sync (RAMBO_OK_EMPTYQ). Once the
 * running AND of some repetition is empty the read is finished: no later
 * term can bring a document back (Section 3.3.1). Uses the handle's mode
 * (rambo_set_mode). Enqueued on `stream`. */
int rambo_query_seqs(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                     uint64_t *out, void *stream);

/* Term-set queries (Section 3.3.1 for a query given as its terms, e.g. a
 * phrase of words): query i is terms[offsets[i] .. offsets[i+1]) and its
 * answer is the documents that hold every term: per repetition the AND of
 * the terms' positive-BFU masks, then the per-document AND over repetitions
 * (Algorithm 2). On a k-mer index the values are 2-bit 31-mer codes of either
 * strand; a query holding a value >= 4^31 answers no document and is counted
 * as invalid (reported by rambo_sync). On an opaque-term index any value is a
 * term. An empty set answers every document (counted for rambo_sync as
 * RAMBO_OK_EMPTYQ). Device arrays (offsets n + 1
 * words, non-decreasing; out n * W words as rambo_query_kmers), asynchronous
 * on `stream`; one wave per set, repetition 0 over all terms before the
 * others; the resolve and early exit settings apply. */
int rambo_query_term_sets(rambo_t *h, const uint64_t *terms, const uint64_t *offsets, uint64_t n, uint64_t *out,
                          void *stream);

/* As rambo_query_seqs, but results are ascending document-id lists: read i's
 * ids are ids[id_offsets[i] .. id_offsets[i+1]) (device arrays, id_offsets
 * has n+1 entries, ids has room for ids_cap entries). Uses `scratch` (device,
 * n * W words) for the bitsets of non-empty answers, of which only the
 * non-zero words are written (the rest of `scratch` is unspecified
 * afterwards), which spares the bitset traffic of the many empty answers and
 * empty words. Synchronous on `stream` (it must learn the total). If the
 * total exceeds ids_cap, returns RAMBO_ETRUNC with id_offsets filled
 * (id_offsets[n] = required capacity) and ids untouched. Returns
 * RAMBO_OK_EMPTYQ instead of RAMBO_OK if some read had no valid window (its
 * list holds every document). Calls on one handle are serialised (per-handle
 * buffers hold the answer sizes and, per read, (W + 63) / 64 words marking
 * its non-zero bitset words; allocated or grown by the call when n exceeds
 * every earlier n). */
int rambo_query_seqs_ids(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                         uint64_t *scratch, uint32_t *ids, uint64_t *id_offsets, uint64_t ids_cap,
                         void *stream);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc between calls): rambo_query_seqs_ids with
 * the same arguments, results and statuses, making no allocation of any kind.
 * The answer sizes and scan scratch that rambo_query_seqs_ids allocates per
 * handle come instead from one fixed array of the library, of
 * RAMBO_NOALLOC_MAX_READS + 1 + RAMBO_NOALLOC_MAX_READS / 1024 + 64 uint64
 * words (about 8 MiB), held on each device the library runs on until the
 * process ends. n may be at most RAMBO_NOALLOC_MAX_READS (RAMBO_EINVAL
 * beyond). Always the plain form (one wavefront per read), whatever
 * rambo_set_mode chose. Synchronous on `stream`. Every call on one device
 * shares that device's array, which keeps the last call's contents: calls
 * from threads of this process are serialised by the library; calls that
 * overlapped on one GPU would race. */
#define RAMBO_NOALLOC_MAX_READS (1u << 20)
int rambo_query_seqs_ids_noalloc(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                                 uint64_t *bits, uint32_t *ids, uint64_t *id_offsets, uint64_t ids_cap,
                                 void *stream);

/* Select the execution form of rambo_query_seqs (RAMBO_MODE_*). */
int rambo_set_mode(rambo_t *h, int mode);

/* Select the resolve strategy (RAMBO_RESOLVE_*); all give identical bits. */
int rambo_set_resolve(rambo_t *h, int resolve);

/* Disable (0) or enable (1, default) early exit in sequence queries; the
 * results are identical either way (only the work differs). */
int rambo_set_early_exit(rambo_t *h, int on);

/* Device counter that sequence queries add the number of issued row probes
 * to (NULL disables counting). Owned by the caller; one uint64. */
int rambo_set_probe_counter(rambo_t *h, uint64_t *device_counter);

/* RAMBO+ measurement (Section 5.1, query time speedup: in repetition r only
 * the BFUs that hold documents returned by the earlier repetitions need a
 * test). With device_counters set (6 uint64 device words, owned by the
 * caller; NULL disables), plain-form sequence queries under schedules 1 and
 * 2 (rambo_tune_t.sched) also tally, before each step of repetitions
 * 1..R-1, what probes restricted to such BFUs could skip: [0] += probes of
 * repetitions >= 1, [1] += those whose row holds no candidate cell, [2] +=
 * 16-byte row segments (128 cells) holding no candidate cell, [3] += row
 * segments probed, [4] += 128-byte lines holding none, [5] += lines probed;
 * the candidates of repetition r being the documents whose cells are set in
 * the read's running masks of repetitions 0..r-1. The answers are
 * unchanged; the tallies make the queries much slower (measurement only). */
int rambo_set_sparse_counter(rambo_t *h, uint64_t *device_counters);

/* Launch shape of the batched form (RAMBO_MODE_BATCHED). */
typedef struct {
    int seg;          /* 32-bit row words one lane reads: 1, 2 or 4 (row split
                         over row_words / seg lanes) */
    int tile;         /* windows per work item, a multiple of 64 */
    int waves_per_cu; /* resident waves per compute unit of the persistent grid */
    int wpb;          /* waves per workgroup: 1, 2 or 4 */
    int grab;         /* work items taken per queue access */
    int sched;        /* probe schedule of a read's windows, same results
                         under both (Section 3.3.1), also used by the plain
                         form: 0 = per step of 64 windows, repetition 0 then
                         the others; 1 = repetition 0 over the whole work
                         item first, then the others; 2 = as 1, after
                         repetition 0 on every 31st window (and the last)
                         first: the plain form does it in its kernel, read
                         by read; the batched form in a pass of its own over
                         every read of the batch before the work queue, which
                         then holds only the reads that pass did not end */
    int tuned;        /* output of rambo_get_tune: 1 once chosen or set */
} rambo_tune_t;

/* Search the batched form's launch shape on a representative batch (device
 * arrays as in rambo_query_seqs; `out` receives the batch's results). The
 * first batched query of a handle runs this search itself unless the
 * environment sets RAMBO_TUNE=off; RAMBO_TUNE_CACHE names a file that keeps
 * chosen shapes across processes. Synchronous on `stream`. */
int rambo_autotune(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n, uint64_t *out,
                   void *stream);
int rambo_get_tune(const rambo_t *h, rambo_tune_t *out);

/* Device time of the most recent batched launch on this handle, from HIP
 * events recorded inside its graph: the whole graph (graph_ms) and its
 * persistent query kernel alone (kernel_ms). Waits for that launch.
 * RAMBO_EINVAL if no batched launch has run or the runtime could not record
 * events inside the graph. */
int rambo_last_batch_ms(rambo_t *h, float *graph_ms, float *kernel_ms);
int rambo_set_tune(rambo_t *h, const rambo_tune_t *t);

/* ---------------------------------------------------------------------- */
/* Serving loop (continuous batching)                                      */
/* ---------------------------------------------------------------------- */

typedef struct rambo_server_s rambo_server_t;

enum {
    RAMBO_SERVE_CONTINUOUS = 0, /* batches form from whatever is pending while
                                   up to `slots` earlier batches run; batched
                                   form replayed from per-slot graphs */
    RAMBO_SERVE_SERIAL = 1,     /* baseline: take everything that has arrived,
                                   run the plain kernel, wait, repeat */
};

typedef struct {
    uint64_t budget_bytes;    /* admission budget: device bytes of in-flight
                                 reads and their result state (read bytes +
                                 8 + W*8 + R*row_words*4 + 16 per read) */
    uint32_t slots;           /* batches in flight at once (1..64) */
    uint32_t max_batch_reads; /* reads per batch (slot capacity) */
    uint64_t max_batch_bytes; /* read bytes per batch (slot capacity) */
    uint32_t policy;          /* RAMBO_SERVE_* */
    uint32_t queue_cap;       /* pending reads before submit returns RAMBO_EBUSY */
    uint32_t direct_below;    /* continuous policy: batches of fewer reads launch
                                 the plain kernel directly instead of replaying
                                 a graph of the slot (0: always replay). Batches
                                 of up to 64 reads are read in place from pinned
                                 memory, larger ones through device copies; 65,
                                 the Python binding's default, launches the
                                 former directly (lowest latency at 1k-50k
                                 reads/s on MI355X) and replays graphs for the
                                 latter (higher throughput near saturation) */
    uint32_t batch_wait_us;   /* batching window: a batch smaller than
                                 max_batch_reads is held until its oldest read
                                 has been pending this long (0: never held,
                                 the lowest latency) */
} rambo_server_config_t;

typedef struct {
    uint64_t tag;         /* as submitted */
    double t_arrival;     /* as submitted (rambo_clock() seconds) */
    double t_admit;       /* its batch was formed */
    double t_done;        /* its result reached host memory */
    int32_t status;       /* RAMBO_OK */
    uint32_t batch_reads; /* reads in the batch it ran in */
} rambo_completion_t;

typedef struct {
    uint64_t submitted, completed, rejected, batches;
    uint64_t max_batch_reads, max_inflight_bytes, backpressure_waits;
    uint64_t pending, inflight_bytes;
} rambo_server_stats_t;

/* Monotonic clock (seconds) the server stamps times with. */
double rambo_clock(void);

/* Start a server on index h (which must stay alive and receive no other work
 * until rambo_server_stop). Allocates the slots' pinned staging buffers,
 * device buffers and graphs, and starts a dispatcher and a completion
 * thread. NULL on error. */
rambo_server_t *rambo_server_start(rambo_t *h, const rambo_server_config_t *cfg);

/* Queue one read (host bytes, copied). t_arrival is the caller's arrival
 * time on rambo_clock(). RAMBO_EBUSY if queue_cap reads are pending,
 * RAMBO_EINVAL if the read can never fit a batch or the budget. */
int rambo_server_submit(rambo_server_t *s, const uint8_t *read, uint64_t len, uint64_t tag, double t_arrival);

/* Open-loop replay: copy n reads (host arrays as in rambo_query_seqs) and
 * submit read i, with tag tag0 + i, at time t_arrival[i] on rambo_clock()
 * from a feeder thread. Returns at once. */
int rambo_server_submit_schedule(rambo_server_t *s, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                                 const double *t_arrival, uint64_t tag0);

/* Take up to max completions (and, if results is not NULL, their W-word
 * bitsets into results[k*W ..]), waiting up to timeout_s for the first.
 * Returns the number taken, or a negative status if the server failed. */
int rambo_server_poll(rambo_server_t *s, rambo_completion_t *out, uint64_t *results, uint32_t max,
                      double timeout_s);

int rambo_server_stats(rambo_server_t *s, rambo_server_stats_t *out);

/* Stop the feeder, finish every queued and in-flight read, join the threads
 * and free the server. Completions not yet polled are discarded. */
int rambo_server_stop(rambo_server_t *s);

#ifdef __cplusplus
}
#endif

#endif /* RAMBO_H */
