// C ABI of librambo: handle lifetime, hash parameters, introspection, and
// the entry points that validate arguments and dispatch to the kernels.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "rambo_int.h"

namespace rambo {

static thread_local std::string g_err;
static thread_local int g_status = RAMBO_OK;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    g_status = status;
    return status;
}

int ok() { return RAMBO_OK; }

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), sequential form.
static uint64_t splitmix_next(uint64_t &s) {
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static constexpr uint64_t P61 = (1ULL << 61) - 1;

// Draw the partition and Bloom hash parameters, then phi_r(d) for all d.
static void derive_hashes(rambo_s *h) {
    uint64_t s = h->seed;
    h->pa.resize(h->R);
    h->pb.resize(h->R);
    for (uint32_t r = 0; r < h->R; r++) {
        h->pa[r] = 1 + splitmix_next(s) % (P61 - 1);
        h->pb[r] = splitmix_next(s) % P61;
    }
    const uint32_t E = h->R * h->eta;
    h->Alo.resize(E); h->Ahi.resize(E); h->Clo.resize(E); h->Chi.resize(E);
    for (uint32_t i = 0; i < E; i++) {
        h->Alo[i] = splitmix_next(s);
        h->Ahi[i] = splitmix_next(s);
        h->Clo[i] = splitmix_next(s);
        h->Chi[i] = splitmix_next(s);
    }
    // phi_r(d) = ((a_r d + b_r) mod P) mod B, Carter-Wegman over the Mersenne
    // prime P; a_r d + b_r < 2^125 fits 128 bits. A shard's local document d
    // takes the cells of its global id (Section 5.3: the node-local partition
    // of the global document).
    h->phi.resize((size_t)h->R * h->K);
    for (uint32_t r = 0; r < h->R; r++) {
        for (uint64_t d = 0; d < h->K; d++) {
            const uint64_t id = h->gids.empty() ? d : h->gids[d];
            unsigned __int128 v = (unsigned __int128)h->pa[r] * id + h->pb[r];
            h->phi[(size_t)r * h->K + d] = (uint32_t)((uint64_t)(v % P61) % h->B);
        }
    }
}

static void free_device(rambo_s *h) {
    if (h->rows) (void)hipFree(h->rows);
    if (h->d_hp) (void)hipFree(h->d_hp);
    if (h->d_cells) (void)hipFree(h->d_cells);
    if (h->d_cells0) (void)hipFree(h->d_cells0);
    if (h->d_ids_counts) (void)hipFree(h->d_ids_counts);
    if (h->d_ids_wm) (void)hipFree(h->d_ids_wm);
    if (h->d_ids_aux) (void)hipFree(h->d_ids_aux);
    if (h->d_boff) (void)hipFree(h->d_boff);
    if (h->d_bdoc) (void)hipFree(h->d_bdoc);
    if (h->d_invalid) (void)hipFree(h->d_invalid);
    if (h->d_gids) (void)hipFree(h->d_gids);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    h->rows = nullptr;
}

static int upload_tables(rambo_s *h) {
    HashParams hp;
    memset(&hp, 0, sizeof hp);
    for (uint32_t i = 0; i < h->R * h->eta; i++) {
        hp.h[i].alo = h->Alo[i]; hp.h[i].ahi = h->Ahi[i];
        hp.h[i].clo = h->Clo[i]; hp.h[i].chi = h->Chi[i];
    }
    HIP_CHECK(hipMalloc(&h->d_hp, sizeof hp));
    HIP_CHECK(hipMemcpy(h->d_hp, &hp, sizeof hp, hipMemcpyHostToDevice));

    // document-major cells: record d holds phi_r(d) at 16-bit slot r (B <= 8192)
    std::vector<uint16_t> cells((size_t)h->K * 8, 0);
    for (uint32_t r = 0; r < h->R; r++)
        for (uint64_t d = 0; d < h->K; d++) cells[d * 8 + r] = (uint16_t)h->phi[(size_t)r * h->K + d];
    HIP_CHECK(hipMalloc(&h->d_cells, cells.size() * 2));
    HIP_CHECK(hipMemcpy(h->d_cells, cells.data(), cells.size() * 2, hipMemcpyHostToDevice));

    // documents grouped by cell, per repetition (Algorithm 2's DocIDs(M[b, r])),
    // with cell offsets relative to the repetition's slice of bdoc
    std::vector<uint32_t> boff((size_t)h->R * (h->B + 1), 0), bdoc((size_t)h->R * h->K);
    for (uint32_t r = 0; r < h->R; r++) {
        uint32_t *off = &boff[(size_t)r * (h->B + 1)];
        const uint32_t *ph = &h->phi[(size_t)r * h->K];
        for (uint64_t d = 0; d < h->K; d++) off[ph[d] + 1]++;
        for (uint32_t b = 0; b < h->B; b++) off[b + 1] += off[b];
        std::vector<uint32_t> fill(h->B, 0);
        for (uint64_t d = 0; d < h->K; d++) {
            const uint32_t b = ph[d];
            bdoc[(size_t)r * h->K + off[b] + fill[b]++] = (uint32_t)d;
        }
        // absolute offsets into bdoc
        for (uint32_t b = 0; b <= h->B; b++) off[b] += (uint32_t)((size_t)r * h->K);
    }
    HIP_CHECK(hipMalloc(&h->d_boff, boff.size() * 4));
    HIP_CHECK(hipMemcpy(h->d_boff, boff.data(), boff.size() * 4, hipMemcpyHostToDevice));
    HIP_CHECK(hipMalloc(&h->d_bdoc, bdoc.size() * 4));
    HIP_CHECK(hipMemcpy(h->d_bdoc, bdoc.data(), bdoc.size() * 4, hipMemcpyHostToDevice));
    // the cell records again, in repetition 0's grouping: the candidate
    // resolve loads a candidate's id and record together
    std::vector<uint16_t> cells0((size_t)h->K * 8, 0);
    for (uint64_t k = 0; k < h->K; k++)
        memcpy(&cells0[k * 8], &cells[(size_t)bdoc[k] * 8], 16);
    HIP_CHECK(hipMalloc(&h->d_cells0, cells0.size() * 2));
    HIP_CHECK(hipMemcpy(h->d_cells0, cells0.data(), cells0.size() * 2, hipMemcpyHostToDevice));
    if (!h->gids.empty() && !h->d_gids) {
        HIP_CHECK(hipMalloc(&h->d_gids, h->gids.size() * 8));
        HIP_CHECK(hipMemcpy(h->d_gids, h->gids.data(), h->gids.size() * 8, hipMemcpyHostToDevice));
    }
    return RAMBO_OK;
}

}  // namespace rambo

using namespace rambo;

RAMBO_API const char *rambo_last_error(void) { return g_err.c_str(); }
RAMBO_API int rambo_last_status(void) { return g_status; }

RAMBO_API rambo_t *rambo_create(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed) {
    return rambo_create_ex(K, B, R, m, eta, seed, 0);
}

RAMBO_API rambo_t *rambo_create_ex(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                                   uint32_t flags) {
    if (flags & ~(uint32_t)RAMBO_TERMS_OPAQUE) {
        fail(RAMBO_EINVAL, "rambo_create_ex: unknown flags 0x%x", flags);
        return nullptr;
    }
    return create_index(K, B, R, m, eta, seed, flags, nullptr);
}

rambo_s *rambo::create_index(uint64_t K, uint32_t B, uint32_t R, uint64_t m, uint32_t eta, uint64_t seed,
                             uint32_t flags, const uint64_t *gids) {
    if (K == 0 || K >= (1ULL << 32) || B == 0 || B > RAMBO_MAX_B || R == 0 || R > RAMBO_MAX_R || eta == 0 ||
        eta > RAMBO_MAX_ETA || m == 0 || m > (1ULL << 40)) {
        fail(RAMBO_EINVAL, "rambo_create: parameters out of range (K=%llu B=%u R=%u m=%llu eta=%u)",
             (unsigned long long)K, B, R, (unsigned long long)m, eta);
        return nullptr;
    }
    auto *h = new rambo_s();
    h->K = K; h->B = B; h->R = R; h->m = m; h->eta = eta; h->seed = seed;
    h->opaque = (flags & RAMBO_TERMS_OPAQUE) != 0;
    if (gids) {
        h->gids.assign(gids, gids + K);
        h->gid_max = *std::max_element(h->gids.begin(), h->gids.end());
    }
    uint32_t need = (B + 31) / 32, rw = 1, lg = 0;
    while (rw < need) { rw <<= 1; lg++; }
    h->RW = rw;
    h->log2RW = lg;
    h->tune.seg = default_seg(rw);
    h->W = (K + 63) / 64;
    h->rows_bytes = (uint64_t)R * m * rw * 4;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
        fail(RAMBO_EDEVICE, "rambo_create: no usable HIP device");
        delete h;
        return nullptr;
    }
    derive_hashes(h);
    if (hipMalloc(&h->rows, h->rows_bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(RAMBO_ENOMEM, "rambo_create: cannot allocate %llu bytes of index on the device",
             (unsigned long long)h->rows_bytes);
        h->rows = nullptr;
        free_device(h);
        delete h;
        return nullptr;
    }
    int st = RAMBO_OK;
    if (hipMemset(h->rows, 0, h->rows_bytes) != hipSuccess) st = fail(RAMBO_EDEVICE, "rambo_create: memset failed");
    if (st == RAMBO_OK) st = upload_tables(h);
    if (st == RAMBO_OK && hipMalloc(&h->d_invalid, 2 * sizeof(unsigned long long)) != hipSuccess)
        st = fail(RAMBO_ENOMEM, "rambo_create: counter allocation failed");
    if (st == RAMBO_OK && hipMemset(h->d_invalid, 0, 2 * sizeof(unsigned long long)) != hipSuccess)
        st = fail(RAMBO_EDEVICE, "rambo_create: memset failed");
    if (st == RAMBO_OK) h->d_emptyq = h->d_invalid + 1;
    if (st == RAMBO_OK && hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess)
        st = fail(RAMBO_EDEVICE, "rambo_create: stream creation failed");
    if (st != RAMBO_OK) {
        free_device(h);
        delete h;
        return nullptr;
    }
    return h;
}

RAMBO_API void rambo_destroy(rambo_t *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    drop_graphs(h);
    free_device(h);
    delete h;
}

RAMBO_API int rambo_sync(rambo_t *h, void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_sync: null handle");
    hipStream_t s = (hipStream_t)stream;
    HIP_CHECK(hipStreamSynchronize(s));
    unsigned long long c[2] = {0, 0};  // invalid inputs, queries without a term
    HIP_CHECK(hipMemcpy(c, h->d_invalid, sizeof c, hipMemcpyDeviceToHost));
    if (c[0] || c[1]) HIP_CHECK(hipMemset(h->d_invalid, 0, sizeof c));
    if (c[0]) return fail(RAMBO_EINVAL, "%llu invalid k-mer values or document ids were skipped", c[0]);
    return c[1] ? RAMBO_OK_EMPTYQ : RAMBO_OK;
}

RAMBO_API int rambo_layout(const rambo_t *h, rambo_layout_t *out) {
    if (!h || !out) return fail(RAMBO_EINVAL, "rambo_layout: null argument");
    out->K = h->K; out->m = h->m; out->seed = h->seed;
    out->B = h->B; out->R = h->R; out->eta = h->eta;
    out->row_words = h->RW;
    out->W = h->W;
    out->index_bytes = h->rows_bytes;
    out->rows = h->rows;
    out->flags = (h->opaque ? RAMBO_TERMS_OPAQUE : 0u) | (h->gids.empty() ? 0u : RAMBO_SHARD);
    return RAMBO_OK;
}

RAMBO_API uint64_t rambo_result_words(const rambo_t *h) { return h ? h->W : 0; }
RAMBO_API uint64_t rambo_index_bytes(const rambo_t *h) { return h ? h->rows_bytes : 0; }

RAMBO_API int rambo_hash_params(const rambo_t *h, uint64_t *pa, uint64_t *pb, uint64_t *Alo, uint64_t *Ahi,
                                uint64_t *Clo, uint64_t *Chi) {
    if (!h || !pa || !pb || !Alo || !Ahi || !Clo || !Chi) return fail(RAMBO_EINVAL, "rambo_hash_params: null argument");
    memcpy(pa, h->pa.data(), h->R * 8);
    memcpy(pb, h->pb.data(), h->R * 8);
    const size_t E = (size_t)h->R * h->eta * 8;
    memcpy(Alo, h->Alo.data(), E); memcpy(Ahi, h->Ahi.data(), E);
    memcpy(Clo, h->Clo.data(), E); memcpy(Chi, h->Chi.data(), E);
    return RAMBO_OK;
}

RAMBO_API int rambo_phi_table(const rambo_t *h, uint32_t *phi) {
    if (!h || !phi) return fail(RAMBO_EINVAL, "rambo_phi_table: null argument");
    memcpy(phi, h->phi.data(), h->phi.size() * 4);
    return RAMBO_OK;
}

RAMBO_API int rambo_dump_bfu(rambo_t *h, uint32_t r, uint32_t b, uint64_t *out) {
    if (!h || !out || r >= h->R || b >= h->B) return fail(RAMBO_EINVAL, "rambo_dump_bfu: bad argument");
    const uint64_t words = (h->m + 63) / 64;
    uint64_t *d = nullptr;
    HIP_CHECK(hipMalloc(&d, words * 8));
    int st = launch_dump_bfu(h, r, b, d, h->aux);
    if (st == RAMBO_OK && hipStreamSynchronize(h->aux) != hipSuccess) st = fail(RAMBO_EDEVICE, "rambo_dump_bfu: kernel failed");
    if (st == RAMBO_OK && hipMemcpy(out, d, words * 8, hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(RAMBO_EDEVICE, "rambo_dump_bfu: copy failed");
    (void)hipFree(d);
    return st;
}

RAMBO_API int rambo_fold(rambo_t *h) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_fold: null handle");
    if (h->B < 2 || h->B % 2) return fail(RAMBO_EINVAL, "rambo_fold: B=%u is not even", h->B);
    HIP_CHECK(hipDeviceSynchronize());
    const uint32_t half = h->B / 2;
    uint32_t need = (half + 31) / 32, rw = 1, lg = 0;
    while (rw < need) { rw <<= 1; lg++; }
    const uint64_t bytes = (uint64_t)h->R * h->m * rw * 4;
    uint32_t *nrows = nullptr;
    if (hipMalloc(&nrows, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RAMBO_ENOMEM, "rambo_fold: cannot allocate %llu bytes for the folded index",
                    (unsigned long long)bytes);
    }
    int st = launch_fold(h, h->rows, nrows, h->RW, lg, half, h->aux);
    if (st == RAMBO_OK && hipStreamSynchronize(h->aux) != hipSuccess) st = fail(RAMBO_EDEVICE, "rambo_fold: kernel failed");
    if (st != RAMBO_OK) {
        (void)hipFree(nrows);
        return st;
    }
    (void)hipFree(h->rows);
    h->rows = nrows;
    h->RW = rw;
    h->log2RW = lg;
    h->rows_bytes = bytes;
    h->B = half;
    // the same hash functions with B/2 cells: phi'_r(d) = phi_r(d) mod B/2
    derive_hashes(h);
    (void)hipFree(h->d_hp);
    (void)hipFree(h->d_cells);
    (void)hipFree(h->d_cells0);
    (void)hipFree(h->d_boff);
    (void)hipFree(h->d_bdoc);
    h->d_hp = nullptr;
    h->d_cells = h->d_cells0 = nullptr;
    h->d_boff = h->d_bdoc = nullptr;
    st = upload_tables(h);
    std::lock_guard<std::mutex> g(h->mu);
    drop_graphs(h);
    h->tuned = false;
    h->tune = Tune();
    h->tune.seg = default_seg(h->RW);
    return st;
}

RAMBO_API int rambo_copy_rows(rambo_t *h, uint64_t offset, uint64_t bytes, void *dst) {
    if (!h || !dst || offset > h->rows_bytes || bytes > h->rows_bytes - offset)
        return fail(RAMBO_EINVAL, "rambo_copy_rows: range outside the index");
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(dst, (const char *)h->rows + offset, bytes, hipMemcpyDeviceToHost));
    return RAMBO_OK;
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------
RAMBO_API int rambo_insert(rambo_t *h, uint64_t doc_id, const uint64_t *kmers, uint64_t n) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_insert: null handle");
    if (doc_id >= h->K) return fail(RAMBO_EINVAL, "rambo_insert: doc_id %llu >= K", (unsigned long long)doc_id);
    if (n == 0) return RAMBO_OK;
    if (!kmers) return fail(RAMBO_EINVAL, "rambo_insert: null k-mer array");
    for (uint64_t i = 0; i < n && !h->opaque; i++)
        if (kmers[i] >> 62)
            return fail(RAMBO_EINVAL, "rambo_insert: value %llu at %llu is not a 31-mer code",
                        (unsigned long long)kmers[i], (unsigned long long)i);
    uint64_t *d = nullptr;
    HIP_CHECK(hipMalloc(&d, n * 8 + 3 * 8));
    const uint64_t meta[3] = {doc_id, 0, n};  // doc_ids[1], offsets[2]
    int st = RAMBO_OK;
    if (hipMemcpyAsync(d, kmers, n * 8, hipMemcpyHostToDevice, h->aux) != hipSuccess ||
        hipMemcpyAsync(d + n, meta, sizeof meta, hipMemcpyHostToDevice, h->aux) != hipSuccess)
        st = fail(RAMBO_EDEVICE, "rambo_insert: copy failed");
    if (st == RAMBO_OK) st = launch_build_kmers(h, d, d + n + 1, d + n, 1, h->aux);
    if (hipStreamSynchronize(h->aux) != hipSuccess && st == RAMBO_OK) st = fail(RAMBO_EDEVICE, "rambo_insert: kernel failed");
    (void)hipFree(d);
    return st;
}

RAMBO_API int rambo_insert_batch(rambo_t *h, const uint64_t *doc_ids, const uint64_t *kmer_offsets,
                                 const uint64_t *kmers, uint64_t n_docs, void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_insert_batch: null handle");
    if (n_docs == 0) return RAMBO_OK;
    if (!doc_ids || !kmer_offsets || !kmers) return fail(RAMBO_EINVAL, "rambo_insert_batch: null array");
    return launch_build_kmers(h, kmers, kmer_offsets, doc_ids, n_docs, (hipStream_t)stream);
}

RAMBO_API int rambo_insert_seqs(rambo_t *h, const uint64_t *doc_ids, const uint8_t *seqs, const uint64_t *offsets,
                                uint64_t n_docs, void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_insert_seqs: null handle");
    if (n_docs == 0) return RAMBO_OK;
    if (!doc_ids || !seqs || !offsets) return fail(RAMBO_EINVAL, "rambo_insert_seqs: null array");
    if (h->opaque) return fail(RAMBO_EINVAL, "rambo_insert_seqs: the index holds opaque terms, not 31-mers");
    return launch_build_seqs(h, seqs, offsets, doc_ids, n_docs, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// queries
// ---------------------------------------------------------------------------
// Memory the runtime does not know (pageable host memory) or host memory.
static bool host_memory(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return a.type == hipMemoryTypeUnregistered || a.type == hipMemoryTypeHost;
}

RAMBO_API int rambo_query_kmers(rambo_t *h, const uint64_t *kmers, uint64_t n, uint64_t *out, void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_query_kmers: null handle");
    if (n == 0) return RAMBO_OK;
    if (!kmers || !out) return fail(RAMBO_EINVAL, "rambo_query_kmers: null array");
    if (stream != nullptr) return launch_query_kmers(h, kmers, n, out, (hipStream_t)stream);
    const bool hk = host_memory(kmers), ho = host_memory(out);
    if (!hk && !ho) return launch_query_kmers(h, kmers, n, out, nullptr);
    if (!hk || !ho) return fail(RAMBO_EINVAL, "rambo_query_kmers: kmers and out must both be host or both device arrays");
    // host arrays: synchronous copy in, query, copy out
    const hipStream_t s = h->aux;
    uint64_t *dk = nullptr, *dout = nullptr;
    HIP_CHECK(hipMallocAsync((void **)&dk, n * 8, s));
    int st = RAMBO_OK;
    if (hipMallocAsync((void **)&dout, n * h->W * 8, s) != hipSuccess) {
        (void)hipGetLastError();
        dout = nullptr;
        st = fail(RAMBO_ENOMEM, "rambo_query_kmers: cannot allocate %llu result bytes on the device",
                  (unsigned long long)(n * h->W * 8));
    }
    if (st == RAMBO_OK && hipMemcpyAsync(dk, kmers, n * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        st = fail(RAMBO_EDEVICE, "rambo_query_kmers: copy in failed");
    if (st == RAMBO_OK) st = launch_query_kmers(h, dk, n, dout, s);
    if (st == RAMBO_OK && hipMemcpyAsync(out, dout, n * h->W * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = fail(RAMBO_EDEVICE, "rambo_query_kmers: copy out failed");
    if (dout) (void)hipFreeAsync(dout, s);
    (void)hipFreeAsync(dk, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == RAMBO_OK) st = fail(RAMBO_EDEVICE, "rambo_query_kmers: failed");
    return st;
}

RAMBO_API int rambo_query_seqs(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n, uint64_t *out,
                               void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_query_seqs: null handle");
    if (n == 0) return RAMBO_OK;
    if (!seqs || !offsets || !out) return fail(RAMBO_EINVAL, "rambo_query_seqs: null array");
    if (h->opaque) return fail(RAMBO_EINVAL, "rambo_query_seqs: the index holds opaque terms, not 31-mers");
    if (h->mode == RAMBO_MODE_BATCHED) return query_seqs_batched(h, seqs, offsets, n, out, (hipStream_t)stream);
    return launch_query_seqs_plain(h, seqs, offsets, n, out, (hipStream_t)stream, default_seg(h->RW));
}

RAMBO_API int rambo_query_term_sets(rambo_t *h, const uint64_t *terms, const uint64_t *offsets, uint64_t n,
                                    uint64_t *out, void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_query_term_sets: null handle");
    if (n == 0) return RAMBO_OK;
    if (!terms || !offsets || !out) return fail(RAMBO_EINVAL, "rambo_query_term_sets: null array");
    return launch_query_termsets(h, terms, offsets, n, out, (hipStream_t)stream);
}

RAMBO_API int rambo_query_seqs_ids(rambo_t *h, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                                   uint64_t *scratch, uint32_t *ids, uint64_t *id_offsets, uint64_t ids_cap,
                                   void *stream) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids: null handle");
    if (!id_offsets) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids: null id_offsets");
    if (h->opaque) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids: the index holds opaque terms, not 31-mers");
    if (n > 0 && (!scratch || !seqs || !offsets)) return fail(RAMBO_EINVAL, "rambo_query_seqs_ids: null array");
    if (n == 0) return launch_ids(h, scratch, 0, ids, id_offsets, ids_cap, (hipStream_t)stream, nullptr, nullptr);
    // id-list mode: the query writes each read's answer size and the bitsets
    // of non-empty answers only
    std::lock_guard<std::mutex> g(h->ids_mu);
    if (h->ids_counts_cap < n) {
        if (h->d_ids_counts) (void)hipFree(h->d_ids_counts);
        if (h->d_ids_wm) (void)hipFree(h->d_ids_wm);
        if (h->d_ids_aux) (void)hipFree(h->d_ids_aux);
        h->d_ids_counts = nullptr;
        h->d_ids_wm = nullptr;
        h->d_ids_aux = nullptr;
        h->ids_counts_cap = 0;
        HIP_CHECK(hipMalloc(&h->d_ids_counts, (n + 1) * 8));
        HIP_CHECK(hipMalloc(&h->d_ids_wm, n * ((h->W + 63) / 64) * 8));
        HIP_CHECK(hipMalloc(&h->d_ids_aux, ids_aux_words(n) * 8));
        h->ids_counts_cap = n;
    }
    const hipStream_t s = (hipStream_t)stream;
    int st = launch_store_u64(reinterpret_cast<uint64_t *>(h->d_ids_counts) + n, 0, s);  // reads without a term
    if (st != RAMBO_OK) return st;
    st = h->mode == RAMBO_MODE_BATCHED
                 ? query_seqs_batched(h, seqs, offsets, n, scratch, s, h->d_ids_counts, h->d_ids_wm)
                 : launch_query_seqs_plain(h, seqs, offsets, n, scratch, s, default_seg(h->RW), nullptr,
                                           h->d_ids_counts, h->d_ids_wm);
    if (st != RAMBO_OK) return st;
    return launch_ids(h, scratch, n, ids, id_offsets, ids_cap, s, h->d_ids_counts, h->d_ids_aux, h->d_ids_wm);
}

RAMBO_API int rambo_set_mode(rambo_t *h, int mode) {
    if (!h || (mode != RAMBO_MODE_PLAIN && mode != RAMBO_MODE_BATCHED)) return fail(RAMBO_EINVAL, "rambo_set_mode: bad mode");
    h->mode = mode;
    return RAMBO_OK;
}

RAMBO_API int rambo_set_resolve(rambo_t *h, int resolve) {
    if (!h || resolve < RAMBO_RESOLVE_AUTO || resolve > RAMBO_RESOLVE_CANDIDATE)
        return fail(RAMBO_EINVAL, "rambo_set_resolve: bad strategy");
    std::lock_guard<std::mutex> g(h->mu);
    h->resolve = resolve;
    drop_graphs(h);
    return RAMBO_OK;
}

RAMBO_API int rambo_set_early_exit(rambo_t *h, int on) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_set_early_exit: null handle");
    std::lock_guard<std::mutex> g(h->mu);
    h->early_exit = on ? 1 : 0;
    drop_graphs(h);
    return RAMBO_OK;
}

RAMBO_API int rambo_set_sparse_counter(rambo_t *h, uint64_t *device_counters) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_set_sparse_counter: null handle");
    std::lock_guard<std::mutex> g(h->mu);
    h->sparse_counter = (unsigned long long *)device_counters;
    drop_graphs(h);
    return RAMBO_OK;
}

RAMBO_API int rambo_set_probe_counter(rambo_t *h, uint64_t *device_counter) {
    if (!h) return fail(RAMBO_EINVAL, "rambo_set_probe_counter: null handle");
    std::lock_guard<std::mutex> g(h->mu);
    h->probe_counter = (unsigned long long *)device_counter;
    drop_graphs(h);
    return RAMBO_OK;
}

// ---------------------------------------------------------------------------
// index files
// ---------------------------------------------------------------------------
namespace {

struct FileHeader {
    char magic[8];  // "RAMBOIX1"
    uint32_t version, header_bytes;
    uint64_t K, m, seed, rows_bytes, checksum;
    uint32_t B, R, eta, flags, row_words, reserved[5];
};
static_assert(sizeof(FileHeader) == 96, "index file header is 96 bytes");

constexpr uint64_t kFileChunk = 64ull << 20;

// The header's fields enter the checksum too (each through the same output
// function as the row words, tagged by its place), so that a header altered
// to other parameters -- which would derive other hash functions for the same
// rows -- is refused as well.
uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
uint64_t header_sum(const FileHeader &h) {
    const uint64_t f[] = {h.K, h.m, h.seed, h.rows_bytes, h.B, h.R, h.eta, h.flags, h.row_words};
    uint64_t s = 0;
    for (uint64_t i = 0; i < sizeof f / sizeof f[0]; i++) s += mix64(f[i] ^ ((i + 1) << 56));
    return s;
}
// a shard's global document ids enter the checksum likewise, each with its place
uint64_t gids_sum(const std::vector<uint64_t> &g) {
    uint64_t s = 0;
    for (uint64_t i = 0; i < g.size(); i++) s += mix64(g[i] + mix64(i ^ (0xABull << 56)));
    return s;
}

// Two pinned staging buffers and their events, freed on scope exit.
struct Staging {
    void *buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Staging() {
        for (int k = 0; k < 2; k++) {
            if (ev[k]) (void)hipEventSynchronize(ev[k]);  // no copy still uses the buffer
            if (ev[k]) (void)hipEventDestroy(ev[k]);
            if (buf[k]) (void)hipHostFree(buf[k]);
        }
    }
    int init() {
        for (int k = 0; k < 2; k++) {
            if (hipHostMalloc(&buf[k], kFileChunk) != hipSuccess) {
                buf[k] = nullptr;
                return fail(RAMBO_ENOMEM, "index file: cannot allocate pinned staging memory");
            }
            HIP_CHECK(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        }
        return RAMBO_OK;
    }
};

struct File {
    FILE *f = nullptr;
    ~File() {
        if (f) fclose(f);
    }
};

}  // namespace

RAMBO_API int rambo_save(rambo_t *h, const char *path) {
    if (!h || !path) return fail(RAMBO_EINVAL, "rambo_save: null argument");
    const hipStream_t s = h->aux;
    HIP_CHECK(hipDeviceSynchronize());  // earlier inserts on any stream are complete
    FileHeader hd{};
    memcpy(hd.magic, "RAMBOIX1", 8);
    hd.version = 1;
    hd.header_bytes = sizeof(FileHeader);
    hd.K = h->K; hd.m = h->m; hd.seed = h->seed; hd.rows_bytes = h->rows_bytes;
    hd.B = h->B; hd.R = h->R; hd.eta = h->eta;
    hd.flags = (h->opaque ? RAMBO_TERMS_OPAQUE : 0u) | (h->gids.empty() ? 0u : RAMBO_SHARD);
    hd.row_words = h->RW;
    int st = rows_checksum(h, &hd.checksum, s);
    if (st != RAMBO_OK) return st;
    hd.checksum += header_sum(hd) + gids_sum(h->gids);
    Staging sg;
    if ((st = sg.init()) != RAMBO_OK) return st;
    File fl;
    fl.f = fopen(path, "wb");
    if (!fl.f) return fail(RAMBO_EIO, "rambo_save: cannot open %s for writing", path);
    if (fwrite(&hd, sizeof hd, 1, fl.f) != 1) return fail(RAMBO_EIO, "rambo_save: write failed (%s)", path);
    if (!h->gids.empty() && fwrite(h->gids.data(), 8, h->gids.size(), fl.f) != h->gids.size())
        return fail(RAMBO_EIO, "rambo_save: write failed (%s)", path);
    // chunk k is copied into buffer k & 1 while chunk k - 1 is written out
    const uint64_t n = (h->rows_bytes + kFileChunk - 1) / kFileChunk;
    const char *src = reinterpret_cast<const char *>(h->rows);
    for (uint64_t k = 0; k <= n; k++) {
        if (k < n) {
            const uint64_t len = std::min(kFileChunk, h->rows_bytes - k * kFileChunk);
            HIP_CHECK(hipMemcpyAsync(sg.buf[k & 1], src + k * kFileChunk, len, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipEventRecord(sg.ev[k & 1], s));
        }
        if (k > 0) {
            const uint64_t j = k - 1, len = std::min(kFileChunk, h->rows_bytes - j * kFileChunk);
            HIP_CHECK(hipEventSynchronize(sg.ev[j & 1]));
            if (fwrite(sg.buf[j & 1], 1, len, fl.f) != len)
                return fail(RAMBO_EIO, "rambo_save: write failed (%s)", path);
        }
    }
    HIP_CHECK(hipStreamSynchronize(s));
    FILE *f = fl.f;
    fl.f = nullptr;
    if (fclose(f) != 0) return fail(RAMBO_EIO, "rambo_save: write failed (%s)", path);
    return ok();
}

RAMBO_API rambo_t *rambo_load(const char *path) {
    if (!path) {
        fail(RAMBO_EINVAL, "rambo_load: null path");
        return nullptr;
    }
    File fl;
    fl.f = fopen(path, "rb");
    if (!fl.f) {
        fail(RAMBO_EIO, "rambo_load: cannot open %s", path);
        return nullptr;
    }
    FileHeader hd{};
    if (fread(&hd, sizeof hd, 1, fl.f) != 1 || memcmp(hd.magic, "RAMBOIX1", 8) != 0 || hd.version != 1 ||
        hd.header_bytes != sizeof(FileHeader)) {
        fail(RAMBO_EIO, "rambo_load: %s is not a RAMBO index file (version 1)", path);
        return nullptr;
    }
    if (hd.flags & ~(uint32_t)(RAMBO_TERMS_OPAQUE | RAMBO_SHARD)) {
        fail(RAMBO_EIO, "rambo_load: %s has unknown flags 0x%x", path, hd.flags);
        return nullptr;
    }
    std::vector<uint64_t> gids;
    if (hd.flags & RAMBO_SHARD) {
        if (hd.K == 0 || hd.K >= (1ULL << 32)) {
            fail(RAMBO_EIO, "rambo_load: %s is not a valid index file", path);
            return nullptr;
        }
        gids.resize(hd.K);
        if (fread(gids.data(), 8, hd.K, fl.f) != hd.K) {
            fail(RAMBO_EIO, "rambo_load: %s is shorter than its header says", path);
            return nullptr;
        }
    }
    rambo_t *h = create_index(hd.K, hd.B, hd.R, hd.m, hd.eta, hd.seed, hd.flags & RAMBO_TERMS_OPAQUE,
                              gids.empty() ? nullptr : gids.data());
    if (!h) return nullptr;  // status and message from the creation
    auto drop = [&](int status, const char *msg) -> rambo_t * {
        rambo_destroy(h);
        fail(status, "rambo_load: %s (%s)", msg, path);
        return nullptr;
    };
    if (h->rows_bytes != hd.rows_bytes || h->RW != hd.row_words) return drop(RAMBO_EIO, "row array size mismatch");
    Staging sg;
    if (sg.init() != RAMBO_OK) return drop(RAMBO_ENOMEM, "cannot allocate pinned staging memory");
    // chunk k is read into buffer k & 1 while chunk k - 1 is copied up;
    // before buffer k & 1 is refilled, the copy of chunk k - 2 from it ends
    const hipStream_t s = h->aux;
    if (hipDeviceSynchronize() != hipSuccess) return drop(RAMBO_EDEVICE, "device error");  // creation's zeroing
    const uint64_t n = (h->rows_bytes + kFileChunk - 1) / kFileChunk;
    char *dst = reinterpret_cast<char *>(h->rows);
    for (uint64_t k = 0; k < n; k++) {
        const uint64_t len = std::min(kFileChunk, h->rows_bytes - k * kFileChunk);
        if (k >= 2 && hipEventSynchronize(sg.ev[k & 1]) != hipSuccess) return drop(RAMBO_EDEVICE, "copy failed");
        if (fread(sg.buf[k & 1], 1, len, fl.f) != len) return drop(RAMBO_EIO, "file is shorter than its header says");
        if (hipMemcpyAsync(dst + k * kFileChunk, sg.buf[k & 1], len, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(sg.ev[k & 1], s) != hipSuccess)
            return drop(RAMBO_EDEVICE, "copy failed");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return drop(RAMBO_EDEVICE, "copy failed");
    char extra;
    if (fread(&extra, 1, 1, fl.f) != 0) return drop(RAMBO_EIO, "file is longer than its header says");
    uint64_t sum = 0;
    if (rows_checksum(h, &sum, s) != RAMBO_OK) return drop(RAMBO_EDEVICE, "checksum failed");
    if (sum + header_sum(hd) + gids_sum(gids) != hd.checksum)
        return drop(RAMBO_EIO, "checksum mismatch: the file is corrupted");
    ok();
    return h;
}
