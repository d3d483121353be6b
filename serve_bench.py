"""Served (continuous batching) measurement on a resident index: open-loop
Poisson arrivals at several rates, p50/p99 latency from the *scheduled*
arrival time to the result in host memory, throughput, and the one-batch-at-
a-time plain baseline on the same arrivals. Every served result is checked
bit for bit against the plain kernel run on the whole set of reads.

Used by bench.py (run(idx, workload, device, log)), with a few seconds of
arrivals per rate; run alone (python serve_bench.py --reads 100000 ...) it
builds the K=10,000 index itself and serves a fixed number of reads per rate.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

RATES = (1000, 5000, 10000, 25000, 50000)


def _serve(idx, reads, arrivals, policy, budget, slots=4, max_batch_reads=8192, max_batch_bytes=8 << 20,
           direct_below=65):
    from paper_1910_04358_amd import Server, clock

    n = reads.n
    srv = Server(idx, budget_bytes=budget, slots=slots, max_batch_reads=max_batch_reads,
                 max_batch_bytes=max_batch_bytes, policy=policy, direct_below=direct_below)
    t0 = clock() + 0.05
    sched = t0 + arrivals
    srv.submit_schedule(reads.seqs, reads.offsets, sched)
    done = np.zeros(n, dtype=bool)
    t_done = np.zeros(n)
    t_admit = np.zeros(n)
    bits = np.zeros((n, idx.W), dtype=np.uint64)
    got = 0
    while got < n:
        comp, res = srv.poll(max_n=8192, timeout_s=0.05)
        for k, c in enumerate(comp):
            i = c.tag
            done[i] = True
            t_done[i] = c.t_done
            t_admit[i] = c.t_admit
            bits[i] = res[k]
        got += len(comp)
        if len(comp) == 0 and clock() > sched[-1] + 60:
            raise RuntimeError("server stalled")
    stats = srv.stats()
    srv.stop()
    lat = t_done - sched
    wait = t_admit - sched      # arrival to the batch being formed (queue and feeder)
    serve = t_done - t_admit    # batch formed to result in host memory (copies, kernel, completion)
    keep = np.argsort(sched)[int(0.05 * n):]  # the first 5 % of arrivals warm up
    pct = lambda a, q: float(np.percentile(a[keep], q) * 1e3)
    return {
        "p50_ms": pct(lat, 50),
        "p99_ms": pct(lat, 99),
        "mean_ms": float(lat[keep].mean() * 1e3),
        "wait_p50_ms": pct(wait, 50), "wait_p99_ms": pct(wait, 99),
        "service_p50_ms": pct(serve, 50), "service_p99_ms": pct(serve, 99),
        "throughput_reads_per_s": n / (t_done.max() - sched[0]),
        "batches": int(stats["batches"]),
        "max_batch_reads": int(stats["max_batch_reads"]),
        "max_inflight_bytes": int(stats["max_inflight_bytes"]),
    }, bits


def run(idx, w, dev, log, rates=RATES, seconds=2.0, min_reads=2000, max_reads=100_000, budget=4 << 30,
        verbose=False):
    import gen
    from paper_1910_04358_amd import MODE_PLAIN, SERVE_CONTINUOUS, SERVE_SERIAL
    import torch

    out = {"rates": [], "budget_bytes": budget, "seconds_per_rate": seconds,
           "note": "latency = result in host memory minus scheduled arrival; first 5% discarded"}
    mode = MODE_PLAIN
    idx.set_mode(mode)
    for k, lam in enumerate(rates):
        n = int(min(max_reads, max(min_reads, lam * seconds)))
        rm = replace(w.reads, qseed=w.reads.qseed + 10 + k)
        reads = gen.reads(w.docs, rm, n)
        arrivals = gen.poisson_arrivals(4000 + k, float(lam), n)
        seqs = torch.from_numpy(reads.seqs).to(dev)
        offs = torch.from_numpy(reads.offsets.view(np.int64)).to(dev)
        ref = idx.query_seqs(seqs, offs).cpu().numpy().view(np.uint64)
        rec = {"rate": lam, "reads": n}
        # served: continuous batching, batches of up to 64 reads launched
        # directly on the pinned areas, larger ones copied and replayed from
        # the slot's graphs; served_graph: every batch replayed from a graph;
        # serial_plain: the one-batch-at-a-time baseline
        for name, policy, direct in (("served", SERVE_CONTINUOUS, 65), ("served_graph", SERVE_CONTINUOUS, 0),
                                     ("serial_plain", SERVE_SERIAL, 0)):
            m, bits = _serve(idx, reads, arrivals, policy, budget, direct_below=direct)
            if not np.array_equal(bits, ref):
                raise SystemExit("served results differ from the plain kernel at rate %d (%s)" % (lam, name))
            rec[name] = m
            if verbose:
                log("serve %7d reads/s: %s done (p50 %.3f p99 %.3f ms)" % (lam, name, m["p50_ms"], m["p99_ms"]))
        log("serve %7d reads/s (%d reads): " % (lam, n) + " | ".join(
            "%s p50 %.3f p99 %.3f ms (wait %.3f/%.3f, service %.3f/%.3f; %.3g reads/s)"
            % (name, m["p50_ms"], m["p99_ms"], m["wait_p50_ms"], m["wait_p99_ms"], m["service_p50_ms"],
               m["service_p99_ms"], m["throughput_reads_per_s"]) for name, m in rec.items()
            if isinstance(m, dict)))
        out["rates"].append(rec)
    return out


def main():
    import argparse
    import json
    import sys
    import time

    import torch

    sys.path.insert(0, __import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    import bench
    import gen

    ap = argparse.ArgumentParser()
    ap.add_argument("--reads", type=int, default=100_000, help="reads per rate")
    ap.add_argument("--rates", default="1000,5000,10000,25000,50000")
    a = ap.parse_args()
    t0 = time.time()

    def log(*x):
        print("[serve %7.1fs]" % (time.time() - t0), *x, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    w = gen.workload(4)
    idx, _, _ = bench.build_index(w, dev)
    rates = [int(r) for r in a.rates.split(",")]
    out = run(idx, w, dev, log, rates=rates, seconds=1e9, min_reads=a.reads, max_reads=a.reads, verbose=True)
    out["reads_per_rate"] = a.reads
    print(json.dumps({"workload": w.name, "served": out}), flush=True)
    idx.close()


if __name__ == "__main__":
    main()
