"""The serving loop: every read's result is the same alone and in the mix
(bit-exact against the oracle), under continuous batching, the serial
baseline, a burst larger than the slots, admission back-pressure from a tiny
budget, and a full queue."""
import numpy as np
import pytest

import gen
from paper_1910_04358_amd import rambo as rb
from tests.gpu_util import make_reads
from tests.test_gpu_parity import setup_case

pytestmark = pytest.mark.gpu


def collect(srv, n, timeout=30.0):
    bits, seen = {}, 0
    t_end = rb.clock() + timeout
    while seen < n and rb.clock() < t_end:
        comp, res = srv.poll(max_n=4096, timeout_s=0.05)
        for k, c in enumerate(comp):
            assert c.status == 0
            assert c.t_done >= c.t_admit >= c.t_arrival - 1e-6
            bits[c.tag] = res[k].copy()
        seen += len(comp)
    assert seen == n, (seen, n)
    return bits


@pytest.mark.parametrize("policy,direct_below", [(rb.SERVE_CONTINUOUS, 2049), (rb.SERVE_CONTINUOUS, 65), (rb.SERVE_CONTINUOUS, 0),
                                                 (rb.SERVE_SERIAL, 0)])
def test_served_results_equal_oracle(policy, direct_below):
    """Batches launched directly (small), replayed from the slot's plain-kernel
    graph, and the serial baseline."""
    idx, o, dm, reads, want = setup_case("rw4")
    n = 1500
    arrivals = gen.poisson_arrivals(4100, 20_000.0, n)
    srv = rb.Server(idx, budget_bytes=1 << 30, slots=3, max_batch_reads=256, max_batch_bytes=1 << 20, policy=policy,
                    direct_below=direct_below)
    t0 = rb.clock() + 0.02
    offs = reads.offsets[: n + 1]
    srv.submit_schedule(reads.seqs[: int(offs[-1])], offs, t0 + arrivals)
    bits = collect(srv, n)
    st = srv.stats()
    srv.stop()
    for i in range(n):
        assert np.array_equal(bits[i], want[i]), i
    assert st["completed"] == n and st["batches"] >= 1
    assert st["max_batch_reads"] <= 256


@pytest.mark.parametrize("direct_below", [0, 2049])
def test_large_served_batches_use_the_persistent_form(direct_below):
    """All reads arrive at once and a 200 ms batching window holds the batch
    until it is complete: one batch of all 3,000 reads replays the slot's
    persistent (batched-form) graph; results equal the oracle's."""
    idx, o, dm, reads, want = setup_case("rw4")
    n = reads.n
    srv = rb.Server(idx, budget_bytes=1 << 30, slots=2, max_batch_reads=n, max_batch_bytes=64 << 20,
                    direct_below=direct_below, batch_wait_us=200_000)
    t0 = rb.clock() + 0.05
    srv.submit_schedule(reads.seqs, reads.offsets, np.full(n, t0))
    bits = collect(srv, n)
    st = srv.stats()
    srv.stop()
    for i in range(n):
        assert np.array_equal(bits[i], want[i]), i
    assert st["max_batch_reads"] > 2048, st
    assert st["batches"] <= 2, st


@pytest.mark.parametrize("direct_below", [0, 2049])
def test_medium_served_batches_through_device_copies(direct_below):
    """Batches of more than 64 reads are copied to the device rather than
    read in place from pinned memory: one batch of 500 reads (held by the
    batching window until complete) runs the plain kernel on the device copy,
    launched directly or replayed from the slot's plain-kernel graph; results
    equal the oracle's."""
    idx, o, dm, reads, want = setup_case("rw4")
    n = 500
    srv = rb.Server(idx, budget_bytes=1 << 30, slots=2, max_batch_reads=n, max_batch_bytes=64 << 20,
                    direct_below=direct_below, batch_wait_us=200_000)
    t0 = rb.clock() + 0.05
    srv.submit_schedule(reads.seqs[: int(reads.offsets[n])], reads.offsets[: n + 1], np.full(n, t0))
    bits = collect(srv, n)
    st = srv.stats()
    srv.stop()
    for i in range(n):
        assert np.array_equal(bits[i], want[i]), i
    assert st["max_batch_reads"] == n and st["batches"] == 1, st


def test_burst_alone_vs_mix_and_backpressure():
    """A burst of reads submitted at once (far more than the slots hold)
    under a budget of only a few reads: all finish, the in-flight bytes never
    exceed the budget, and each result equals the same read served alone."""
    idx, o, dm, reads, want = setup_case("rw4")
    W = idx.W
    per_read = 400 + 8 + W * 8 + idx.R * idx.row_words * 4 + 16
    budget = 4 * per_read
    srv = rb.Server(idx, budget_bytes=budget, slots=2, max_batch_reads=64, max_batch_bytes=1 << 16,
                    policy=rb.SERVE_CONTINUOUS)
    picks = [i for i in range(reads.n) if len(reads.read(i)) <= 400][:300]
    t = rb.clock()
    for k, i in enumerate(picks):
        assert srv.submit(reads.read(i), k, t) == 0
    bits = collect(srv, len(picks))
    st = srv.stats()
    srv.stop()
    assert st["max_inflight_bytes"] <= budget
    assert st["backpressure_waits"] > 0
    for k, i in enumerate(picks):
        assert np.array_equal(bits[k], want[i])
    # the same reads one at a time
    srv = rb.Server(idx, budget_bytes=1 << 20, slots=1, max_batch_reads=1, max_batch_bytes=1 << 16)
    for k, i in enumerate(picks[:40]):
        assert srv.submit(reads.read(i), k) == 0
        one = collect(srv, 1)
        assert np.array_equal(one[k], bits[k])
    srv.stop()


def test_queue_full_and_oversized_reads():
    idx, o, dm, reads, want = setup_case("rw4")
    srv = rb.Server(idx, budget_bytes=1 << 20, slots=1, max_batch_reads=16, max_batch_bytes=4096, queue_cap=4)
    codes = [srv.submit(reads.read(i), i) for i in range(200)]
    assert rb.EBUSY in codes
    assert srv.submit(b"A" * 5000, 9999) == rb.EINVAL  # never fits a batch
    accepted = sum(c == 0 for c in codes)
    bits = collect(srv, accepted)
    srv.stop()
    for i, c in enumerate(codes):
        if c == 0:
            assert np.array_equal(bits[i], want[i])


def test_edge_reads_served():
    idx, o, dm, reads, want = setup_case("rw4")
    d = dm.doc(9)
    cases = [b"", b"ACG", b"N" * 50, d[10:41], d[500:900]]
    wantc = [o.query_seq(s) for s in cases]
    srv = rb.Server(idx, budget_bytes=1 << 24, slots=2, max_batch_reads=8, max_batch_bytes=1 << 14)
    for k, s in enumerate(cases):
        assert srv.submit(s, k) == 0
    bits = collect(srv, len(cases))
    srv.stop()
    for k in range(len(cases)):
        assert np.array_equal(bits[k], wantc[k]), k
