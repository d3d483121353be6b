#!/usr/bin/env python3
"""Benchmark of the RAMBO hot path on one MI355X.

Workload (the K = 10,000 configuration the headline metric is quoted on):
K = 10,000 documents (100 random ancestors x 100 mutants of 500 kbp, per
document substitution rate uniform in 0.5-2 %), R = 5, B = 100, m = 2^29
bits per BFU, eta = 2 (a 40 GiB bit-sliced index); 100,000 reads with
log-normal lengths (median 300 bp, sigma 1, clipped to 31-10,000 bp), 70 %
copied from a random document with 0-1 % errors, 30 % random. Seeded,
synthetic (the paper's ENA archive is not available).

A step is one query batch of all 100,000 reads (every k-mer of every read
counted, including those early exit skips), with the index and the reads
resident in HBM. The batched form (persistent launch replayed from a HIP
graph, autotuned shape) gives `value`; the plain one-launch kernel and the
build are reported beside it, with the served form's latency when run.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
# Bytes one isolated random row read moves from HBM on this GPU: every read
# request from L2 to memory is a 128-byte request, for random 16-byte rows as
# for streaming copies (request-size counters TCC_EA0_RDREQ_32B/64B/128B, one
# 128-byte request per probe; profiles/probe_granule_MI355X.md).
GRANULE = 128
GRANULE_SOURCE = "profiles/probe_granule_MI355X.md"
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "batched_query_K10000_traffic.json")


def measured_traffic():
    """HBM bytes per batched query pass (all its kernels) from the committed
    counter profile, or None if the kernels' sources changed since it was
    taken."""
    import hashlib
    try:
        prof = json.load(open(TRAFFIC_PROFILE))
        h = hashlib.sha256()
        for s in prof["sources"]:
            h.update(open(os.path.join(ROOT, s), "rb").read())
        return prof["traffic_bytes_per_launch"] if h.hexdigest() == prof["sources_sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print("[bench %7.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def up(a, dev):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a).to(dev)


def build_index(w, dev, docs_per_chunk=1000):
    """Create the index, stage all documents in HBM, build in one launch."""
    import torch
    import gen
    from paper_1910_04358_amd import Rambo

    idx = Rambo(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    L, nd = w.docs.length, w.docs.n_docs
    seqs = torch.empty(nd * L, dtype=torch.uint8, device=dev)
    host = torch.empty(docs_per_chunk * L, dtype=torch.uint8, pin_memory=True)
    hnp = host.numpy()
    for c0 in range(0, nd, docs_per_chunk):
        c1 = min(nd, c0 + docs_per_chunk)
        w.docs.docs(c0, c1 - c0, out=hnp[: (c1 - c0) * L])
        seqs[c0 * L: c1 * L].copy_(host[: (c1 - c0) * L], non_blocking=False)
    log("documents staged in HBM: %.2f GB" % (nd * L / 1e9))
    offs = up(np.arange(nd + 1, dtype=np.uint64) * np.uint64(L), dev)
    ids = up(np.arange(nd, dtype=np.uint64), dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    idx.insert_seqs(ids, seqs, offs)
    e1.record()
    idx.sync()
    build_ms = e0.elapsed_time(e1)
    kmers = nd * (L - 30)
    del seqs
    torch.cuda.empty_cache()
    return idx, build_ms, kmers


def kmer_queries_run(dev, steps, warmup):
    """Single k-mer queries (plain kernel) on the K = 1,000 workload: 20
    ancestors x 50 mutants of 200 kbp (1 % substitutions), R=4, B=32,
    m=2^26, eta=3; 10^7 queries, half windows of documents, half random."""
    import torch
    import gen

    w = gen.workload(2)
    idx, build_ms, build_kmers = build_index(w, dev)
    q, _ = gen.kmer_queries(w.docs, w.kmer_qseed, w.n_kmer_queries, 0.5)
    qd = up(q, dev)
    out = torch.empty((q.size, idx.W), dtype=torch.int64, device=dev)
    ms = time_steps(lambda: idx.query_kmers(qd, out=out), steps, warmup)
    probes = q.size * w.R * w.eta
    rec = {"workload": w.name, "queries": int(q.size), "ms_per_batch": ms, "kmer_per_s": q.size / ms * 1e3,
           "probes_per_s": probes / ms * 1e3, "out_bytes": int(q.size * idx.W * 8),
           "build_ms": build_ms, "build_input_GBps_u64_kmers": build_kmers * 8 / build_ms / 1e6}
    log("k-mer queries (%s): %.3f ms per 10^7, %.3g k-mer/s; build %.0f ms" % (w.name, ms, rec["kmer_per_s"],
                                                                               build_ms))
    idx.close()
    del out, qd
    torch.cuda.empty_cache()
    return rec


def rambo_plus(idx, step, dev):
    """What RAMBO+ (Section 5.1, query time speedup: in repetition r test only
    the BFUs holding documents the earlier repetitions returned) could save on
    this batch: one plain-form pass with the library's tallies on (scout
    schedule, early exit; not timed). A probe of repetition r >= 1 could skip
    the 16-byte row segments (128 cells) and 128-byte lines whose cells hold
    none of the candidates left by repetitions 0..r-1."""
    import torch
    from paper_1910_04358_amd import MODE_PLAIN
    c = torch.zeros(6, dtype=torch.int64, device=dev)
    idx.set_mode(MODE_PLAIN)
    idx.set_sparse_counter(c)
    step()
    torch.cuda.synchronize()
    idx.set_sparse_counter(None)
    v = [int(x) for x in c.cpu().tolist()]
    return {"probes_rep_ge1": v[0], "probes_without_candidate_cell": v[1],
            "frac_probes_skippable": v[1] / max(1, v[0]),
            "untouched_16B_segment_frac": v[2] / max(1, v[3]),
            "untouched_128B_line_frac": v[4] / max(1, v[5]),
            "segments_per_row": v[3] / max(1, v[0]), "lines_per_row": v[5] / max(1, v[0])}


def stream_insert(idx, w, dev):
    """Streaming insertion (Section 3.2): the workload's new documents
    (ids w.stream_docs) inserted into the built, resident index in one call;
    returns (ms, k-mers) timed with events around the insertion kernel."""
    import torch
    s0, ns = w.stream_docs
    L = w.docs.length
    host = torch.empty(ns * L, dtype=torch.uint8, pin_memory=True)
    w.docs.docs(s0, ns, out=host.numpy())
    seqs = host.to(dev)
    offs = up(np.arange(ns + 1, dtype=np.uint64) * np.uint64(L), dev)
    ids = up(np.arange(s0, s0 + ns, dtype=np.uint64), dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    idx.insert_seqs(ids, seqs, offs)
    e1.record()
    idx.sync()
    ms = e0.elapsed_time(e1)
    del seqs, host
    return ms, ns * (L - 30)


def k101000_run(dev, steps, warmup, tune=None):
    """One GPU's share of a cluster-scale index: K = 101,000 capacity, 1,000
    ancestors x 100 mutants of 100 kbp (1 %), R=6, B=1,000, m=2^27, eta=2
    (96 GiB); build of 100,000 documents (10^10 k-mers), streaming insertion
    of 1,000 new documents (10 new ancestors x 100 mutants, ids 100,000 ..
    100,999) into the built index, then 10^6 reads of U(100, 1000) bp (70 %
    from any of the 101,000 documents with 1 % errors), batched form,
    answered as bitsets and as document-id lists."""
    import torch
    import gen
    from paper_1910_04358_amd import MODE_BATCHED, MODE_PLAIN

    w = gen.workload(5)
    idx, build_ms, build_kmers = build_index(w, dev, docs_per_chunk=2000)
    ins_ms, ins_kmers = stream_insert(idx, w, dev)
    log("K101000: streamed %d new documents (%d k-mers) in %.2f ms" % (w.stream_docs[1], ins_kmers, ins_ms))
    reads = gen.reads(w.docs, w.reads, w.n_reads)
    n_kmers = reads.n_windows()
    seqs, offs = up(reads.seqs, dev), up(reads.offsets, dev)
    out = torch.empty((reads.n, idx.W), dtype=torch.int64, device=dev)

    def step():
        idx.query_seqs(seqs, offs, out=out, check=False)

    idx.set_mode(MODE_PLAIN)
    plain_ms = time_steps(step, steps, warmup)
    idx.set_mode(MODE_BATCHED)
    if tune:
        from paper_1910_04358_amd import Tune
        idx.set_tune(Tune(*[int(v) for v in tune.split(",")]))
    step()  # autotunes the launch shape on this batch (unless set above)
    ms = time_steps(step, steps, warmup)
    probes = torch.zeros(1, dtype=torch.int64, device=dev)
    idx.set_probe_counter(probes)
    step()
    torch.cuda.synchronize()
    issued = int(probes.item())
    idx.set_probe_counter(None)
    ids_ms = time_steps(lambda: idx.query_seqs_ids(seqs, offs, ids_cap=50_000_000, scratch=out, check=False), 3, 1)
    rplus = rambo_plus(idx, step, dev)
    log("K101000: RAMBO+ could skip %.4f of the probes of repetitions >= 1, %.4f of their 16-byte segments"
        % (rplus["frac_probes_skippable"], rplus["untouched_16B_segment_frac"]))
    rec = {"workload": w.name, "index_bytes": idx.index_bytes, "build_ms": build_ms,
           "build_input_GBps_u64_kmers": build_kmers * 8 / build_ms / 1e6,
           "stream_insert": {"docs": w.stream_docs[1], "kmers": ins_kmers, "ms": ins_ms,
                             "kmer_per_s": ins_kmers / ins_ms * 1e3,
                             "input_GBps_u64_kmers": ins_kmers * 8 / ins_ms / 1e6,
                             "bases_per_s": w.stream_docs[1] * w.docs.length / ins_ms * 1e3},
           "reads": reads.n, "kmers": n_kmers,
           "plain_ms": plain_ms, "batched_ms": ms, "kmer_per_s": n_kmers / ms * 1e3, "reads_per_s": reads.n / ms * 1e3,
           "probes": issued, "row_bytes": idx.row_words * 4, "rows_per_s": issued / ms * 1e3,
           "ids_ms": ids_ms, "rambo_plus": rplus, "tune": idx.get_tune().__dict__}
    log("K101000: build %.0f ms (%.3g k-mer/s); plain %.2f ms, batched %.2f ms per 10^6 reads (%.3g k-mer/s, %.3g rows "
        "of %d B/s); as id lists %.2f ms" % (build_ms, build_kmers / build_ms * 1e3, plain_ms, ms, rec["kmer_per_s"],
                                            rec["rows_per_s"], rec["row_bytes"], ids_ms))
    idx.close()
    del out, seqs, offs
    torch.cuda.empty_cache()
    return rec


def web_terms_run(dev, steps, warmup, n_sets=100_000):
    """Document indexing with word terms (the paper's web-document setting)
    on synthetic term sets shaped like its two samples: Wiki-dump-like
    (17,618 documents of ~650 terms, B=1,000, R=2, m=200,000) and
    ClueWeb09-like (50,000 documents of ~450 terms, B=5,000, R=3,
    m=20,000); eta = 2. Build, 10^6 single-term queries (half present), and
    term-set queries of 2-8 terms (half phrases of a document)."""
    import torch
    import gen
    from paper_1910_04358_amd import Rambo

    recs = {}
    for name in ("wiki", "clueweb"):
        w = gen.term_workload(name)
        terms, offs = w.docs.docs()
        idx = Rambo(w.K, w.B, w.R, w.m, w.eta, w.index_seed, opaque_terms=True)
        ids, td, od = up(np.arange(w.K, dtype=np.uint64), dev), up(terms, dev), up(offs, dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        idx.insert_batch(ids, od, td)
        e1.record()
        torch.cuda.synchronize()
        idx.sync()
        build_ms = e0.elapsed_time(e1)
        q, _ = w.docs.term_queries(w.qseed, w.n_queries, 0.5)
        qd = up(q, dev)
        out = torch.empty((q.size, idx.W), dtype=torch.int64, device=dev)
        ms = time_steps(lambda: idx.query_kmers(qd, out=out), steps, warmup)
        pt, po, _ = w.docs.phrases(w.qseed + 1, n_sets, 2, 8, 0.5)
        ptd, pod = up(pt, dev), up(po, dev)
        out2 = torch.empty((n_sets, idx.W), dtype=torch.int64, device=dev)
        ms2 = time_steps(lambda: idx.query_term_sets(ptd, pod, out=out2, check=False), steps, warmup)
        recs[name] = {"workload": w.name, "terms_indexed": int(terms.size), "build_ms": build_ms,
                      "build_terms_per_s": terms.size / build_ms * 1e3, "index_bytes": idx.index_bytes,
                      "queries": int(q.size), "ms_per_batch": ms, "term_queries_per_s": q.size / ms * 1e3,
                      "out_GBps": q.size * idx.W * 8 / ms / 1e6, "term_sets": n_sets,
                      "ms_per_set_batch": ms2, "term_sets_per_s": n_sets / ms2 * 1e3}
        log("terms %s: build %.1f ms (%.3g terms/s); %.3g term queries/s (%.0f GB/s of results); %.3g term sets/s"
            % (w.name, build_ms, recs[name]["build_terms_per_s"], recs[name]["term_queries_per_s"],
               recs[name]["out_GBps"], recs[name]["term_sets_per_s"]))
        idx.close()
        del out, out2, qd, td, od, ptd, pod
        torch.cuda.empty_cache()
    return recs


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def pipelined_run(idx, seqs, offs, ref, steps, warmup):
    """The same batch passes, consecutive ones alternating between two streams
    (each with its own output buffer, so its own captured graphs and queue
    state): a batch's scout pass and queue building can run while the
    previous batch's persistent kernel drains. Each step is still one whole
    pass over one batch; the answers are checked against the single-stream
    ones. Timed with events: the two streams wait for a start event on the
    current stream, which waits for both at the end."""
    import torch
    outs = [torch.empty_like(ref), torch.empty_like(ref)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    cur = torch.cuda.current_stream()

    def run(k):
        for i in range(k):
            idx.query_seqs(seqs, offs, out=outs[i % 2], stream=streams[i % 2], check=False)

    for s in streams:
        s.wait_stream(cur)
    run(max(2, warmup))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for s in streams:
        s.wait_event(e0)
    run(steps)
    for s in streams:
        cur.wait_stream(s)
    e1.record(cur)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if not (torch.equal(outs[0], ref) and torch.equal(outs[1], ref)):
        raise SystemExit("two-stream batched results differ")
    return {"ms_per_step": ms, "streams": 2,
            "note": "consecutive batches alternate between two streams (own output buffers and graphs); "
                    "each step is one whole pass over one batch"}


def host_cores():
    """(threads the oracle may use, description of the host): every core this
    process may run on (its affinity set), capped by OMP_NUM_THREADS when the
    environment sets one (the share of the host granted to this job)."""
    import platform
    import subprocess
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        n = min(n, int(omp))
    model = platform.processor()
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        nproc = None
    return max(1, n), {"nproc": nproc, "os_cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
                       "omp_num_threads": omp, "model": model}


def cpu_baseline(w, sample_reads, sample_docs, nthreads):
    """The oracle (Algorithm 2, early exit) on a bounded sample of the same
    workload: an index of the same shape (R, B, m, eta) holding documents
    0..sample_docs-1, queried with reads drawn from those documents with the
    workload's length, error and random-read mix. The sample's BFUs hold a
    tenth of the workload's documents, so they are sparser and a Bloom test
    fails sooner than on the full index: the rate is an upper bound of the
    oracle's rate on the full workload."""
    import gen
    import oracle
    from dataclasses import replace

    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    t = time.time()
    step = 250
    for c0 in range(0, sample_docs, step):
        c1 = min(sample_docs, c0 + step)
        o.build_docs(w.docs.docs(c0, c1 - c0), w.docs.length, c0, c1 - c0, nthreads=nthreads)
    build_s = time.time() - t
    log("cpu oracle: built %d documents in %.1fs" % (sample_docs, build_s))
    rm = replace(w.reads, src_lo=0, src_hi=sample_docs, qseed=w.reads.qseed + 100)
    reads = gen.reads(w.docs, rm, sample_reads)
    t = time.time()
    res, tests = o.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2, early_exit=True, nthreads=nthreads)
    q_s = time.time() - t
    kmers = reads.n_windows()
    # one thread, the paper's query convention, on the first tenth
    n1 = max(1, sample_reads // 10)
    o1 = reads.offsets[: n1 + 1]
    t = time.time()
    o.query_seqs(reads.seqs[: int(o1[-1])], o1, oracle.MODE_ALG2, early_exit=True, nthreads=1)
    one_s = time.time() - t
    k1 = int(np.maximum(np.diff(o1.astype(np.int64)) - 30, 0).sum())
    del o
    return {"value": kmers / q_s, "unit": "k-mer queries/s", "cores": nthreads, "kind": "oracle",
            "sample": "Algorithm 2 with early exit on %d reads (%d k-mers) drawn from documents 0..%d of the "
                      "workload (same length, error and random mix), against an oracle index of the "
                      "workload's shape (R=%d, B=%d, m=2^%d, eta=%d) holding those %d documents (a tenth of "
                      "the workload's: sparser BFUs, so an upper bound of the oracle's rate on the full index); "
                      "query time %.2fs on %d threads (index build %.1fs not counted)"
                      % (sample_reads, kmers, sample_docs - 1, w.R, w.B, int(np.log2(w.m)), w.eta,
                         sample_docs, q_s, nthreads, build_s),
            "reads_per_s": sample_reads / q_s,
            "one_thread_kmer_per_s": k1 / one_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the served (continuous batching) runs")
    ap.add_argument("--cpu-reads", type=int, default=60000)
    ap.add_argument("--no-fold", action="store_true", help="skip folding the index at the end")
    ap.add_argument("--cpu-docs", type=int, default=1000)
    ap.add_argument("--tune", default=None,
                    help="batched launch shape seg,tile,waves_per_cu,wpb,grab (skips the autotuner)")
    ap.add_argument("--no-kmers", action="store_true", help="skip the single k-mer query workload")
    ap.add_argument("--no-terms", action="store_true", help="skip the word-term (web document) workloads")
    ap.add_argument("--no-k101000", action="store_true", help="skip the K=101,000 (96 GiB) workload")
    ap.add_argument("--tune-k101000", default=None,
                    help="batched launch shape of the K=101,000 workload (skips its autotuner)")
    ap.add_argument("--k101000-only", action="store_true",
                    help="run only the K=101,000 workload and print its record (for profiler runs)")
    ap.add_argument("--no-full", action="store_true", help="skip the runs without early exit")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="also run a 1 GiB device copy (scale for hardware byte counters)")
    ap.add_argument("--only", choices=["plain", "batched"], default=None,
                    help="time only one form (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (documents would be "
              "sharded across GPUs, one independent index per GPU: no exchange at build time, one broadcast "
              "of each read batch and one gather of the per-GPU result slices per query)", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    from paper_1910_04358_amd import MODE_BATCHED, MODE_PLAIN

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.k101000_only:
        print(json.dumps({"k101000": k101000_run(dev, args.steps, args.warmup, args.tune_k101000)}), flush=True)
        return
    w = gen.workload(3)
    log("workload", w.name)
    idx, build_ms, build_kmers = build_index(w, dev)
    log("build: %.1f ms for %d k-mers" % (build_ms, build_kmers))

    reads = gen.reads(w.docs, w.reads, w.n_reads)
    n_kmers = reads.n_windows()
    seqs, offs = up(reads.seqs, dev), up(reads.offsets, dev)
    out = torch.empty((reads.n, idx.W), dtype=torch.int64, device=dev)
    log("reads: %d, %d k-mers, %.1f MB" % (reads.n, n_kmers, reads.seqs.size / 1e6))

    def step():
        idx.query_seqs(seqs, offs, out=out, check=False)

    result = {}
    probes = torch.zeros(1, dtype=torch.int64, device=dev)
    if args.only != "batched":
        idx.set_mode(MODE_PLAIN)
        plain_ms = time_steps(step, args.steps, args.warmup)
        ref = out.clone()
        idx.set_probe_counter(probes)
        step()
        torch.cuda.synchronize()
        plain_probes = int(probes.item())
        idx.set_probe_counter(None)
        log("plain: %.3f ms/step, %.3g k-mer/s, %d probes" % (plain_ms, n_kmers / plain_ms * 1e3, plain_probes))
        result["plain"] = {"ms_per_step": plain_ms, "kmer_per_s": n_kmers / plain_ms * 1e3,
                           "reads_per_s": reads.n / plain_ms * 1e3, "probes": plain_probes}
    idx.set_mode(MODE_BATCHED)
    if args.tune:
        from paper_1910_04358_amd import Tune
        idx.set_tune(Tune(*[int(v) for v in args.tune.split(",")]))
    t = time.time()
    step()  # autotunes the launch shape on this batch (unless set above)
    torch.cuda.synchronize()
    tune = idx.get_tune()
    log("autotune: %.1fs -> %s" % (time.time() - t, tune))
    if args.only != "plain":
        batched_ms = time_steps(step, args.steps, args.warmup)
        if args.only is None and not torch.equal(out, ref):
            raise SystemExit("batched results differ from the plain kernel")
        # the main kernel's own device time from events inside the graph, and
        # the probes of the pass (scout and main kernels), per launch
        idx.set_probe_counter(probes)
        probes.zero_()
        kern, graph = [], []
        for _ in range(args.steps):
            step()
            g_ms, k_ms = idx.last_batch_ms()
            graph.append(g_ms)
            kern.append(k_ms)
        torch.cuda.synchronize()
        issued = int(probes.item()) / args.steps
        idx.set_probe_counter(None)
        kern_ms = float(np.mean(kern))
        log("batched: %.3f ms/step (graph %.3f, kernel %.3f), %.3g k-mer/s, %.0f probes/launch"
            % (batched_ms, np.mean(graph), kern_ms, n_kmers / batched_ms * 1e3, issued))
        pipelined = pipelined_run(idx, seqs, offs, out, args.steps, args.warmup)
        log("batched, consecutive batches alternating two streams: %.3f ms/step, %.3g k-mer/s"
            % (pipelined["ms_per_step"], n_kmers / pipelined["ms_per_step"] * 1e3))
        pipelined["kmer_per_s"] = n_kmers / pipelined["ms_per_step"] * 1e3
    else:
        batched_ms = kern_ms = issued = float("nan")
        pipelined = None

    row_bytes = idx.row_words * 4
    io_bytes = reads.seqs.size + 8 * (reads.n + 1) + reads.n * idx.W * 8
    alg_bytes = issued * max(GRANULE, row_bytes) + io_bytes
    # The probes are split between two kernels of one pass (the scout kernel,
    # then the persistent main kernel over the reads it left), so the roofline
    # is taken over the whole pass: its algorithmic bytes over the step time
    # measured with HIP events on the stream the pass runs on.
    achieved = alg_bytes / (batched_ms * 1e-3) / 1e9
    value = n_kmers / batched_ms * 1e3

    # Without early exit every valid window is probed in every repetition
    # (k-mers x R x eta probes): the same batch, both forms, so that the
    # roofline fraction is also shown on work that nothing skips.
    full = None
    if args.only is None and not args.no_full:
        full = {}
        idx.set_early_exit(False)
        for name, mode in (("plain", MODE_PLAIN), ("batched", MODE_BATCHED)):
            idx.set_mode(mode)
            ms = time_steps(step, min(args.steps, 5), 1)
            if not torch.equal(out, ref):
                raise SystemExit("results without early exit differ")
            idx.set_probe_counter(probes)
            probes.zero_()
            step()
            torch.cuda.synchronize()
            n_pr = int(probes.item())
            idx.set_probe_counter(None)
            by = n_pr * max(GRANULE, row_bytes) + io_bytes
            full[name] = {"ms_per_step": ms, "kmer_per_s": n_kmers / ms * 1e3, "probes": n_pr,
                          "achieved_GBps": by / ms / 1e6, "frac": by / ms / 1e6 / HBM_PEAK_GBS}
            log("no early exit, %s: %.3f ms/step, %d probes, %.0f GB/s (%.2f of peak)"
                % (name, ms, n_pr, by / ms / 1e6, by / ms / 1e6 / HBM_PEAK_GBS))
        idx.set_early_exit(True)
        idx.set_mode(MODE_BATCHED)

    # the empirical ceiling of the probe pattern: uniformly random row reads
    # over the index's own buffer (random-access microbenchmark)
    ceiling = None
    try:
        from paper_1910_04358_amd import micro
        import ctypes
        L = micro.lib()
        sink = torch.zeros(4096, dtype=torch.int32, device=dev)
        lay = idx.layout()
        blocks = torch.cuda.get_device_properties(0).multi_processor_count * 16
        best = min(L.micro_run(0, ctypes.c_void_p(lay.rows), idx.index_bytes, row_bytes, blocks, 16, 77 + k,
                               ctypes.c_void_p(sink.data_ptr())) for k in range(3))
        nload = blocks * 256 * 16 * L.micro_per_lane(0, row_bytes)
        ceiling = {"probes_per_s": nload / best * 1e3, "GBps": nload / best * 1e3 * max(GRANULE, row_bytes) / 1e9,
                   "what": "random %d-byte row reads over the %.0f GiB index buffer" % (row_bytes,
                                                                                      idx.index_bytes / 2**30)}
        log("random-read ceiling: %.3g probes/s (%.0f GB/s at %d B)" % (ceiling["probes_per_s"], ceiling["GBps"],
                                                                      max(GRANULE, row_bytes)))
    except (RuntimeError, OSError) as e:
        log("random-read ceiling not measured:", e)

    rplus = None
    if args.only is None:
        rplus = rambo_plus(idx, step, dev)
        idx.set_mode(MODE_BATCHED)
        log("RAMBO+ could skip %.4f of the probes of repetitions >= 1, %.4f of their 16-byte segments"
            % (rplus["frac_probes_skippable"], rplus["untouched_16B_segment_frac"]))

    if args.pmc_copy:
        from paper_1910_04358_amd import micro
        ms = micro.copy(1 << 30)
        log("copy kernel: 1 GiB in %.3f ms" % ms)

    web = None
    if not args.no_terms:
        web = web_terms_run(dev, min(args.steps, 10), min(args.warmup, 2))

    kq = None
    if not args.no_kmers:
        kq = kmer_queries_run(dev, args.steps, args.warmup)

    cpu = None
    if not args.no_cpu:
        nthr, host = host_cores()
        cpu = cpu_baseline(w, args.cpu_reads, args.cpu_docs, nthr)
        cpu["host"] = host
        log("cpu oracle: %.3g k-mer/s on %d threads (%s)" % (cpu["value"], nthr, host))

    served = None
    if not args.no_serve:
        try:
            import serve_bench
            served = serve_bench.run(idx, w, dev, log)
        except ImportError:
            served = None

    line = {
        "metric": "k-mer queries/s (batched form, K=10,000 documents) with read p50/p99 latency served vs plain",
        "value": value,
        "unit": "k-mer queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": batched_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 bitwise (u64 k-mer codes)",
        "data": "synthetic (seeded genomes: 100 ancestors x 100 mutants of 500 kbp; 100,000 reads)",
        "config": {"workload": w.name, "K": w.K, "B": w.B, "R": w.R, "m": w.m, "eta": w.eta,
                   "reads": reads.n, "kmers_per_step": n_kmers, "index_bytes": idx.index_bytes,
                   "tune": tune.__dict__},
        "reads_per_s": reads.n / batched_ms * 1e3,
        "build": {"ms": build_ms, "kmers": build_kmers,
                  "input_GBps_u64_kmers": build_kmers * 8 / build_ms / 1e6,
                  "bases_per_s": w.docs.n_docs * w.docs.length / build_ms * 1e3},
        "plain": result.get("plain"),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "useful_bytes_frac": (issued * row_bytes + io_bytes) / (batched_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "kernel": "batched query pass (k_batch_scout, k_batch_prep, scan, k_batch_main)",
                     "kernel_ms": batched_ms, "main_kernel_ms": kern_ms, "probes_per_launch": issued,
                     "bytes_per_probe": max(GRANULE, row_bytes), "bytes_per_probe_source": GRANULE_SOURCE,
                     "io_bytes": io_bytes,
                     "random_read_ceiling": ceiling,
                     "frac_of_ceiling": (issued / (batched_ms * 1e-3) / ceiling["probes_per_s"]) if ceiling else None},
        "cpu_baseline": cpu,
        "served": served,
        "no_early_exit": full,
        "pipelined": pipelined,
        "rambo_plus": rplus,
        "kmer_queries": kq,
        "web_terms": web,
    }
    if not args.no_fold and args.only is None:
        # folding over (B -> B/2, streaming), then the same batch on the folded index
        idx.set_mode(MODE_PLAIN)
        before = idx.index_bytes
        torch.cuda.synchronize()
        t = time.time()
        idx.fold()
        fold_s = time.time() - t
        moved = before + idx.index_bytes
        folded_ms = time_steps(step, args.steps, args.warmup)
        line["fold"] = {"B_after": idx.B, "ms": fold_s * 1e3, "bytes_moved": moved,
                        "GBps": moved / fold_s / 1e9, "frac_of_hbm_peak": moved / fold_s / 1e9 / HBM_PEAK_GBS,
                        "plain_ms_per_step_after": folded_ms,
                        "note": "wall time of the synchronous call (allocation + kernel + table rebuild)"}
        log("fold: B %d -> %d in %.1f ms (%.0f GB/s incl. allocation); plain step after: %.3f ms"
            % (w.B, idx.B, fold_s * 1e3, moved / fold_s / 1e9, folded_ms))
    idx.close()
    del seqs, offs, out
    torch.cuda.empty_cache()
    line["k101000"] = None
    if not args.no_k101000 and args.only is None:
        line["k101000"] = k101000_run(dev, min(args.steps, 5), min(args.warmup, 1), args.tune_k101000)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
