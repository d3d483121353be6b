// Serving loop: continuous batching of arriving reads against a resident
// index.
//
// Requests wait in a host queue. A dispatcher thread forms a batch from
// everything pending that fits a free staging slot and the admission budget
// (device bytes of the in-flight reads and their result state), copies it
// on the slot's own stream; up to `slots` batches are in flight at once, so
// the work of one batch overlaps that of another and reads that arrive while
// others run join the next batch. Batches of up to 64 reads are read by the
// kernel straight from the slot's pinned staging area and answered straight
// into its pinned result area (no copy operations: one launch or one graph
// replay per batch); larger ones are copied to the device, run there (the
// plain kernel launched directly below direct_below reads, else the slot's
// captured graphs: the plain kernel's up to 2,048 reads, the persistent
// form's beyond) and their results copied back. A completion
// thread takes each batch as soon as it is done (in any order), hands its
// results over and stamps the completion time. Each result is the same
// bitset rambo_query_seqs gives for that read alone: reads are independent
// within a batch.
//
// The serial policy is the one-batch-at-a-time baseline: take everything
// that has arrived, run the plain kernel, wait, repeat.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "batch.h"

namespace rambo {

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    const uint8_t *bytes;  // into owned storage
    uint64_t len;
    uint64_t tag;
    double t_arrival;
    std::shared_ptr<std::vector<uint8_t>> own;  // single submissions own their bytes
    double t_pending = 0;                       // entered the pending queue (rambo_clock)
};

// A slot's staging area (pinned on the host, mirrored on the device) holds
// one batch packed as [InputHdr | offsets (n + 1) | read bytes], so a batch
// goes to the device in a single copy and the captured graphs find it
// through the header at the start.
static constexpr uint64_t kHdrBytes = 256;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t *h_stage = nullptr, *d_stage = nullptr;
    uint64_t *h_out = nullptr, *d_out = nullptr;
    // the pinned staging and result areas as the device addresses them
    uint8_t *hd_stage = nullptr;
    uint64_t *hd_out = nullptr;
    // plain-kernel graphs for small batches (on the pinned areas, and on the
    // device copy), the persistent form's for large ones
    std::shared_ptr<BatchGraph> small, mid, large;
    std::vector<Request> reqs;
    uint64_t budget = 0;
    double t_admit = 0;
};

}  // namespace rambo

struct rambo_server_s {
    rambo_s *h = nullptr;
    rambo_server_config_t cfg{};
    std::vector<rambo::Slot> slots;
    std::mutex mu;  // pending queue, free slots, budget, stats
    std::condition_variable cv_dispatch, cv_done, cv_poll;
    std::deque<rambo::Request> pending;
    std::atomic<uint64_t> n_pending{0};  // pending.size(), readable without the lock
    std::deque<int> free_slots, inflight;
    uint64_t budget_used = 0;
    bool stopping = false;
    std::atomic<int> error{RAMBO_OK};  // written under mu, read under either lock
    std::string error_msg;
    std::thread dispatcher, completer, feeder;
    // completions
    std::mutex cmu;
    std::deque<rambo_completion_t> comp;
    std::deque<std::vector<uint64_t>> comp_bits;
    // scheduled submissions
    std::vector<uint8_t> sched_bytes;
    std::vector<uint64_t> sched_offs;
    std::vector<double> sched_t;
    uint64_t sched_tag0 = 0;
    std::atomic<bool> feeder_stop{false};
    rambo_server_stats_t stats{};
};

namespace rambo {

static uint64_t request_cost(const rambo_s *h, uint64_t len) {
    // read bytes, its offset, its result bitset, its running masks
    return len + 8 + h->W * 8 + (uint64_t)h->R * h->RW * 4 + 16;
}

static void server_fail(rambo_server_s *s, int st) {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error == RAMBO_OK) {
        // the message is written before the code: readers under the other
        // lock look at the message only once they see the code set
        s->error_msg = rambo_last_error();
        s->error = st;
    }
    s->stopping = true;
    s->cv_dispatch.notify_all();
    s->cv_done.notify_all();
    s->cv_poll.notify_all();
}

// Pack the slot's requests into its staging area; returns the bytes to copy.
// The header points at the batch where the kernels will read it: in the
// device copy (base = d_stage), or in the pinned area itself (hd_stage).
static uint64_t pack_slot(Slot &sl, const uint8_t *base) {
    const uint64_t n = sl.reqs.size();
    uint64_t *offs = (uint64_t *)(sl.h_stage + kHdrBytes);
    uint8_t *bytes = (uint8_t *)(offs + n + 1);
    uint64_t off = 0;
    offs[0] = 0;
    for (uint64_t i = 0; i < n; i++) {
        memcpy(bytes + off, sl.reqs[i].bytes, sl.reqs[i].len);
        off += sl.reqs[i].len;
        offs[i + 1] = off;
    }
    InputHdr *hdr = (InputHdr *)sl.h_stage;
    hdr->n = n;
    hdr->offs = (const uint64_t *)(base + kHdrBytes);
    hdr->seqs = base + kHdrBytes + (n + 1) * 8;
    hdr->pad = 0;
    return kHdrBytes + (n + 1) * 8 + off;
}

// Batches of at most this many reads are served from the pinned areas in
// place: the kernel's byte loads and result stores then cross the host bus,
// which for a few reads costs less than the two copies, and for hundreds of
// reads (the batches of high arrival rates) far more.
static constexpr uint64_t kZeroCopyMaxReads = 64;

// Whether the continuous policy serves an n-read batch from the pinned areas
// directly (the plain kernel launched directly, or the slot's plain-kernel
// graph, both reading the pinned staging area and writing the pinned result
// area) rather than through device copies.
static bool zero_copy(const rambo_server_s *s, const Slot &sl, uint64_t n) {
    return s->cfg.policy == RAMBO_SERVE_CONTINUOUS && n <= kZeroCopyMaxReads &&
           (n < s->cfg.direct_below || n <= sl.small->cap);
}

static int launch_slot(rambo_server_s *s, Slot &sl, uint64_t n) {
    rambo_s *h = s->h;
    const bool zc = zero_copy(s, sl, n);
    const uint64_t copy_bytes = pack_slot(sl, zc ? sl.hd_stage : sl.d_stage);
    int st;
    if (zc && n < s->cfg.direct_below) {
        // one launch: reads from the staging area, answers into the result area
        const uint8_t *base = sl.hd_stage + kHdrBytes;
        st = launch_query_seqs_plain(h, base + (n + 1) * 8, (const uint64_t *)base, n, sl.hd_out, sl.stream,
                                     default_seg(h->RW));
    } else if (zc) {
        st = launch_batch_graph(h, *sl.small, sl.stream);
    } else {
        HIP_CHECK(hipMemcpyAsync(sl.d_stage, sl.h_stage, copy_bytes, hipMemcpyHostToDevice, sl.stream));
        if (s->cfg.policy == RAMBO_SERVE_SERIAL || n < s->cfg.direct_below) {
            const uint64_t *offs = (const uint64_t *)(sl.d_stage + kHdrBytes);
            st = launch_query_seqs_plain(h, sl.d_stage + kHdrBytes + (n + 1) * 8, offs, n, sl.d_out, sl.stream,
                                         default_seg(h->RW));
        } else if (n <= sl.mid->cap) {
            st = launch_batch_graph(h, *sl.mid, sl.stream);
        } else {
            st = launch_batch_graph(h, *sl.large, sl.stream);
        }
        if (st == RAMBO_OK)
            HIP_CHECK(hipMemcpyAsync(sl.h_out, sl.d_out, n * h->W * 8, hipMemcpyDeviceToHost, sl.stream));
    }
    if (st != RAMBO_OK) return st;
    HIP_CHECK(hipEventRecord(sl.done, sl.stream));
    return RAMBO_OK;
}

static void dispatcher_main(rambo_server_s *s) {
    (void)hipSetDevice(s->h->device);
    const uint64_t W = s->h->W;
    (void)W;
    for (;;) {
        int slot = -1;
        uint64_t n = 0, bytes = 0, cost = 0;
        // an arrival is seen sooner by polling than by a wake-up: poll for up
        // to 2 ms before sleeping on the condition variable (at rates above
        // 500 reads/s the dispatcher never sleeps)
        for (const double until = now_s() + 2e-3; s->n_pending.load(std::memory_order_acquire) == 0 && now_s() < until;)
            std::this_thread::yield();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_dispatch.wait(lk, [&] {
                return s->stopping || (!s->pending.empty() && !s->free_slots.empty() &&
                                       s->budget_used + request_cost(s->h, s->pending.front().len) <= s->cfg.budget_bytes);
            });
            if (s->stopping && (s->pending.empty() || s->error != RAMBO_OK)) return;
            if (s->pending.empty() || s->free_slots.empty()) continue;
            // batching window: a partial batch waits until it fills or its
            // oldest read has been pending batch_wait_us
            if (s->cfg.batch_wait_us && !s->stopping && s->pending.size() < s->cfg.max_batch_reads) {
                const double due = s->pending.front().t_pending + s->cfg.batch_wait_us * 1e-6;
                const double d = due - now_s();
                if (d > 0) {
                    s->cv_dispatch.wait_for(lk, std::chrono::duration<double>(std::min(d, 1e-3)));
                    continue;
                }
            }
            slot = s->free_slots.front();
            s->free_slots.pop_front();
            Slot &sl = s->slots[slot];
            sl.reqs.clear();
            // everything that has arrived and fits the slot and the budget
            while (!s->pending.empty() && n < s->cfg.max_batch_reads) {
                const Request &r = s->pending.front();
                const uint64_t c = request_cost(s->h, r.len);
                if (bytes + r.len > s->cfg.max_batch_bytes) break;
                if (s->budget_used + cost + c > s->cfg.budget_bytes) {
                    s->stats.backpressure_waits++;
                    break;
                }
                sl.reqs.push_back(r);
                s->pending.pop_front();
                s->n_pending.fetch_sub(1, std::memory_order_relaxed);
                bytes += r.len;
                cost += c;
                n++;
            }
            s->budget_used += cost;
            if (s->budget_used > s->stats.max_inflight_bytes) s->stats.max_inflight_bytes = s->budget_used;
            s->stats.batches++;
            if (n > s->stats.max_batch_reads) s->stats.max_batch_reads = n;
        }
        Slot &sl = s->slots[slot];
        sl.budget = cost;
        sl.t_admit = now_s();
        int st = launch_slot(s, sl, n);
        if (st != RAMBO_OK) {
            server_fail(s, st);
            return;
        }
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->inflight.push_back(slot);
        }
        s->cv_done.notify_one();
        if (s->cfg.policy == RAMBO_SERVE_SERIAL) {
            // one batch at a time: wait until the completion thread has freed it
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_dispatch.wait(lk, [&] { return s->stopping || s->inflight.empty(); });
        }
    }
}

static void completer_main(rambo_server_s *s) {
    (void)hipSetDevice(s->h->device);
    const uint64_t W = s->h->W;
    std::vector<int> look;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.wait(lk, [&] { return !s->inflight.empty() || (s->stopping && s->pending.empty()) || s->error; });
            if (s->inflight.empty()) {
                if (s->stopping) return;
                continue;
            }
            look.assign(s->inflight.begin(), s->inflight.end());
        }
        // the first in-flight batch found done, in any order (spinning on the
        // events: completion latency matters more than one host core)
        int slot = -1;
        for (size_t k = 0; slot < 0; k = (k + 1) % look.size()) {
            const hipError_t e = hipEventQuery(s->slots[look[k]].done);
            if (e == hipSuccess) {
                slot = look[k];
            } else if (e != hipErrorNotReady) {
                fail(RAMBO_EDEVICE, "server: batch failed: %s", hipGetErrorString(e));
                server_fail(s, RAMBO_EDEVICE);
                return;
            } else if (k + 1 == look.size()) {
                std::this_thread::yield();
                // batches dispatched meanwhile join the polling
                std::lock_guard<std::mutex> g(s->mu);
                look.assign(s->inflight.begin(), s->inflight.end());
            }
        }
        Slot &sl = s->slots[slot];
        const double t_done = now_s();
        // the batch's completions and result copies are made before the
        // lock is taken, and only moved in under it (a poller holding the
        // lock must not stall this thread for long)
        const size_t nr = sl.reqs.size();
        std::vector<rambo_completion_t> cs(nr);
        std::vector<std::vector<uint64_t>> bs(nr);
        for (size_t i = 0; i < nr; i++) {
            rambo_completion_t &c = cs[i];
            c.tag = sl.reqs[i].tag;
            c.t_arrival = sl.reqs[i].t_arrival;
            c.t_admit = sl.t_admit;
            c.t_done = t_done;
            c.status = RAMBO_OK;
            c.batch_reads = (uint32_t)nr;
            bs[i].assign(sl.h_out + i * W, sl.h_out + (i + 1) * W);
        }
        {
            std::lock_guard<std::mutex> g(s->cmu);
            for (size_t i = 0; i < nr; i++) {
                s->comp.push_back(cs[i]);
                s->comp_bits.push_back(std::move(bs[i]));
            }
        }
        s->cv_poll.notify_all();
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->inflight.erase(std::find(s->inflight.begin(), s->inflight.end(), slot));
            s->budget_used -= sl.budget;
            s->stats.completed += sl.reqs.size();
            sl.reqs.clear();
            s->free_slots.push_back(slot);
        }
        s->cv_dispatch.notify_all();
    }
}

static int enqueue_request(rambo_server_s *s, Request r) {
    if (r.len > s->cfg.max_batch_bytes || request_cost(s->h, r.len) > s->cfg.budget_bytes)
        return fail(RAMBO_EINVAL, "server: read of %llu bytes exceeds the batch or budget capacity",
                    (unsigned long long)r.len);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->error != RAMBO_OK) return fail(s->error, "server stopped: %s", s->error_msg.c_str());
        if (s->stopping) return fail(RAMBO_EINVAL, "server is stopping");
        if (s->pending.size() >= s->cfg.queue_cap) {
            s->stats.rejected++;
            return fail(RAMBO_EBUSY, "server queue full (%u pending)", s->cfg.queue_cap);
        }
        r.t_pending = now_s();
        s->pending.push_back(std::move(r));
        s->n_pending.fetch_add(1, std::memory_order_release);
        s->stats.submitted++;
    }
    s->cv_dispatch.notify_one();
    return RAMBO_OK;
}

static void feeder_main(rambo_server_s *s) {
    const uint64_t n = s->sched_t.size();
    for (uint64_t i = 0; i < n && !s->feeder_stop.load(); i++) {
        const double t = s->sched_t[i];
        for (;;) {
            const double d = t - now_s();
            if (d <= 0) break;
            if (d > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(d - 1e-4));
            else std::this_thread::yield();
        }
        Request r{s->sched_bytes.data() + s->sched_offs[i], s->sched_offs[i + 1] - s->sched_offs[i], s->sched_tag0 + i, t,
                  nullptr};
        // open loop: a full queue drops nothing here, the feeder waits for room
        while (!s->feeder_stop.load()) {
            int st = enqueue_request(s, r);
            if (st == RAMBO_OK) break;
            if (st != RAMBO_EBUSY) return;
            std::this_thread::yield();
        }
    }
}

static void free_slot(Slot &sl) {
    sl.small.reset();
    sl.mid.reset();
    sl.large.reset();
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_stage) (void)hipHostFree(sl.h_stage);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.d_stage) (void)hipFree(sl.d_stage);
    if (sl.d_out) (void)hipFree(sl.d_out);
}

// The runtime sets up its copy engines on their first use, for several
// milliseconds each during which the issuing call blocks, once per process;
// which engine a copy takes depends on the copies already in flight. Copies
// of every size class in both directions, in flight on all slots' streams at
// once, meet those set-up costs here rather than in the middle of a burst.
static int warm_copies(rambo_server_s *s) {
    const uint64_t R = s->cfg.max_batch_reads, BY = s->cfg.max_batch_bytes;
    const uint64_t stage = kHdrBytes + (R + 1) * 8 + BY, out_bytes = R * s->h->W * 8;
    for (int rep = 0; rep < 2; rep++) {
        for (uint64_t sz : {uint64_t(4) << 10, uint64_t(64) << 10, uint64_t(1) << 20, ~uint64_t(0)}) {
            for (Slot &sl : s->slots) {
                HIP_CHECK(hipMemcpyAsync(sl.d_stage, sl.h_stage, std::min(sz, stage), hipMemcpyHostToDevice,
                                         sl.stream));
                HIP_CHECK(hipMemcpyAsync(sl.h_out, sl.d_out, std::min(sz, out_bytes), hipMemcpyDeviceToHost,
                                         sl.stream));
            }
        }
        for (Slot &sl : s->slots) HIP_CHECK(hipStreamSynchronize(sl.stream));
    }
    return RAMBO_OK;
}

static int setup_slot(rambo_server_s *s, Slot &sl) {
    rambo_s *h = s->h;
    const uint64_t R = s->cfg.max_batch_reads, BY = s->cfg.max_batch_bytes;
    const uint64_t stage = kHdrBytes + (R + 1) * 8 + BY;
    HIP_CHECK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    HIP_CHECK(hipHostMalloc((void **)&sl.h_stage, stage, hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void **)&sl.h_out, R * h->W * 8, hipHostMallocDefault));
    HIP_CHECK(hipMalloc(&sl.d_stage, stage));
    HIP_CHECK(hipMalloc(&sl.d_out, R * h->W * 8));
    HIP_CHECK(hipHostGetDevicePointer((void **)&sl.hd_stage, sl.h_stage, 0));
    HIP_CHECK(hipHostGetDevicePointer((void **)&sl.hd_out, sl.h_out, 0));
    if (s->cfg.policy == RAMBO_SERVE_CONTINUOUS) {
        Tune large = h->tune;
        if (!h->tuned) large.seg = default_seg(h->RW);
        // small batches: the plain kernel, one wave per read, on the pinned
        // areas; large ones: the persistent form with the handle's tuned
        // shape on the device copy
        const uint64_t small_cap = std::min<uint64_t>(R, kZeroCopyMaxReads), mid_cap = std::min<uint64_t>(R, 2048);
        int st = make_plain_graph(h, (const InputHdr *)sl.hd_stage, small_cap, sl.hd_out, sl.small);
        if (st == RAMBO_OK) st = make_plain_graph(h, (const InputHdr *)sl.d_stage, mid_cap, sl.d_out, sl.mid);
        if (st == RAMBO_OK)
            st = make_batch_graph(h, large, (const InputHdr *)sl.d_stage, nullptr, R, sl.d_out, sl.large);
        if (st != RAMBO_OK) return st;
        // replay both graphs once on an empty batch, so that the first real
        // batch does not pay for loading their kernels
        InputHdr *hdr = (InputHdr *)sl.h_stage;
        hdr->n = 0;
        hdr->offs = (const uint64_t *)(sl.hd_stage + kHdrBytes);
        hdr->seqs = sl.hd_stage + kHdrBytes;
        HIP_CHECK(hipMemcpy(sl.d_stage, sl.h_stage, sizeof(InputHdr), hipMemcpyHostToDevice));
        if ((st = launch_batch_graph(h, *sl.small, sl.stream)) != RAMBO_OK) return st;
        if ((st = launch_batch_graph(h, *sl.mid, sl.stream)) != RAMBO_OK) return st;
        if ((st = launch_batch_graph(h, *sl.large, sl.stream)) != RAMBO_OK) return st;
        HIP_CHECK(hipStreamSynchronize(sl.stream));
    }
    return RAMBO_OK;
}

}  // namespace rambo

using namespace rambo;

RAMBO_API double rambo_clock(void) { return now_s(); }

RAMBO_API rambo_server_t *rambo_server_start(rambo_t *h, const rambo_server_config_t *cfg) {
    if (h && h->opaque) {
        fail(RAMBO_EINVAL, "rambo_server_start: the index holds opaque terms, not 31-mers");
        return nullptr;
    }
    if (!h || !cfg || cfg->slots == 0 || cfg->slots > 64 || cfg->max_batch_reads == 0 || cfg->max_batch_bytes == 0 ||
        cfg->budget_bytes == 0 || cfg->queue_cap == 0 ||
        (cfg->policy != RAMBO_SERVE_CONTINUOUS && cfg->policy != RAMBO_SERVE_SERIAL)) {
        fail(RAMBO_EINVAL, "rambo_server_start: bad configuration");
        return nullptr;
    }
    auto *s = new rambo_server_s();
    s->h = h;
    s->cfg = *cfg;
    const uint32_t nslots = cfg->policy == RAMBO_SERVE_SERIAL ? 1 : cfg->slots;
    s->slots.resize(nslots);
    int st = RAMBO_OK;
    for (uint32_t i = 0; i < nslots && st == RAMBO_OK; i++) {
        st = setup_slot(s, s->slots[i]);
        s->free_slots.push_back((int)i);
    }
    if (st == RAMBO_OK) st = warm_copies(s);
    if (st != RAMBO_OK) {
        for (auto &sl : s->slots) free_slot(sl);
        delete s;
        return nullptr;
    }
    s->dispatcher = std::thread(dispatcher_main, s);
    s->completer = std::thread(completer_main, s);
    return s;
}

RAMBO_API int rambo_server_submit(rambo_server_t *s, const uint8_t *read, uint64_t len, uint64_t tag, double t_arrival) {
    if (!s || (!read && len)) return fail(RAMBO_EINVAL, "rambo_server_submit: bad argument");
    auto own = std::make_shared<std::vector<uint8_t>>(read, read + len);
    Request r{own->data(), len, tag, t_arrival, own};
    return enqueue_request(s, r);
}

RAMBO_API int rambo_server_submit_schedule(rambo_server_t *s, const uint8_t *seqs, const uint64_t *offsets, uint64_t n,
                                           const double *t_arrival, uint64_t tag0) {
    if (!s || !offsets || !t_arrival || (n && !seqs)) return fail(RAMBO_EINVAL, "rambo_server_submit_schedule: bad argument");
    if (s->feeder.joinable()) return fail(RAMBO_EBUSY, "rambo_server_submit_schedule: a schedule is already running");
    for (uint64_t i = 0; i < n; i++)
        if (offsets[i + 1] < offsets[i]) return fail(RAMBO_EINVAL, "rambo_server_submit_schedule: offsets decrease");
    s->sched_bytes.assign(seqs, seqs + (n ? offsets[n] - offsets[0] : 0));
    s->sched_offs.resize(n + 1);
    for (uint64_t i = 0; i <= n; i++) s->sched_offs[i] = offsets[i] - offsets[0];
    s->sched_t.assign(t_arrival, t_arrival + n);
    s->sched_tag0 = tag0;
    s->feeder_stop = false;
    s->feeder = std::thread(feeder_main, s);
    return RAMBO_OK;
}

RAMBO_API int rambo_server_poll(rambo_server_t *s, rambo_completion_t *out, uint64_t *results, uint32_t max,
                                double timeout_s) {
    if (!s || (!out && max)) return fail(RAMBO_EINVAL, "rambo_server_poll: bad argument");
    const uint64_t W = s->h->W;
    // take the completions out under the lock (moves only) and copy them to
    // the caller's arrays after it is released, so the completion thread,
    // which needs the lock for every batch, is not held up by the copies
    std::vector<std::vector<uint64_t>> bits;
    uint32_t k = 0;
    int err = RAMBO_OK;
    {
        std::unique_lock<std::mutex> lk(s->cmu);
        if (s->comp.empty() && timeout_s > 0) {
            s->cv_poll.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !s->comp.empty() || s->error; });
        }
        const uint32_t take = (uint32_t)std::min<uint64_t>(max, s->comp.size());
        bits.reserve(take);
        while (k < take) {
            out[k] = s->comp.front();
            bits.push_back(std::move(s->comp_bits.front()));
            s->comp.pop_front();
            s->comp_bits.pop_front();
            k++;
        }
        err = s->error;
    }
    if (results)
        for (uint32_t i = 0; i < k; i++) memcpy(results + (uint64_t)i * W, bits[i].data(), W * 8);
    if (k == 0 && err != RAMBO_OK) return fail(err, "server failed: %s", s->error_msg.c_str());
    return (int)k;
}

RAMBO_API int rambo_server_stats(rambo_server_t *s, rambo_server_stats_t *out) {
    if (!s || !out) return fail(RAMBO_EINVAL, "rambo_server_stats: bad argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->pending = s->pending.size();
    out->inflight_bytes = s->budget_used;
    return RAMBO_OK;
}

RAMBO_API int rambo_server_stop(rambo_server_t *s) {
    if (!s) return RAMBO_OK;
    s->feeder_stop = true;
    if (s->feeder.joinable()) s->feeder.join();
    {
        // drain: let pending and in-flight batches finish
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_dispatch.notify_all();
        s->cv_dispatch.wait_for(lk, std::chrono::seconds(60),
                                [&] { return s->error || (s->pending.empty() && s->inflight.empty()); });
        s->stopping = true;
    }
    s->cv_dispatch.notify_all();
    s->cv_done.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    if (s->completer.joinable()) s->completer.join();
    int st = s->error;
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        free_slot(sl);
    }
    if (st != RAMBO_OK) fail(st, "server failed: %s", s->error_msg.c_str());
    delete s;
    return st;
}
