"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times.

The oracle cannot build a 40-96 GiB index in test time, so at full size it
computes outputs one by one: whole BFUs of sampled cells (built from just the
documents of the cell, `orc_bfu_insert_seq`), compared bit for bit with the
GPU index, and the answer for sampled documents on every read (document d is
reported iff every term of the read passes in BFU(r, phi_r(d)) for all r).
Expected answers computed beforehand by the oracle one repetition at a time
(tests/golden/<workload>_answers.txt, written by
tests/golden/make_fullsize_golden.py, which calls only the oracle) give the
whole answer of 10,000 sampled reads, and the answers of sampled documents
(their cells covering every row word or row segment in every repetition)
on every read of the workload. Properties that hold at any size cover the
rest: zero false negatives, strand invariance, plain = batched, streaming
insertion.
"""
import concurrent.futures as cf
import hashlib
import os

import numpy as np
import pytest

import gen
import oracle
from paper_1910_04358_amd import rambo as rb
from tests import _ref
from tests.gpu_util import make_reads, to_dev, to_host_u64

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def build_gpu(idx, dm, d0, nd, chunk):
    import torch
    host = torch.empty(chunk * dm.length, dtype=torch.uint8, pin_memory=True)
    dev = torch.empty(chunk * dm.length, dtype=torch.uint8, device="cuda")
    hnp = host.numpy()
    for c0 in range(d0, d0 + nd, chunk):
        c1 = min(d0 + nd, c0 + chunk)
        k = c1 - c0
        dm.docs(c0, k, out=hnp[: k * dm.length])
        dev[: k * dm.length].copy_(host[: k * dm.length])
        offs = np.arange(k + 1, dtype=np.uint64) * np.uint64(dm.length)
        idx.insert_seqs(to_dev(np.arange(c0, c1, dtype=np.uint64)), dev, to_dev(offs))
        torch.cuda.synchronize()
    idx.sync()
    del dev, host


def oracle_cells(o, dm, cells, n_docs, phis):
    """Whole BFUs (r, b) built by the oracle from the documents of each cell
    among documents 0..n_docs-1, in parallel threads."""
    def one(rb_):
        r, b = rb_
        f = o.new_bfu()
        for d in np.nonzero(phis[r, :n_docs] == b)[0]:
            o.bfu_insert_seq(r, f, np.frombuffer(dm.doc(int(d)), dtype=np.uint8))
        return rb_, f
    with cf.ThreadPoolExecutor(16) as ex:
        return dict(ex.map(one, sorted(set(cells))))


def doc_answers(o, F, phis, docs, reads):
    """Oracle answer of each sampled document for every read."""
    out = {}
    for d in docs:
        keep = np.ones(reads.n, dtype=bool)
        for r in range(o.R):
            keep &= o.bfu_test_seqs(r, F[(r, int(phis[r, d]))], reads.seqs, reads.offsets)
        out[d] = keep
    return out


def bit_of(bits, d):
    return ((bits[:, d >> 6] >> np.uint64(d & 63)) & np.uint64(1)).astype(bool)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name, reads):
    """(sampled read indices, {read: ascending ids} for non-empty sampled
    answers, {doc: set of reads reporting it}) from the stored oracle
    answers; checks that the workload's reads are the ones they were
    computed for."""
    hdr, sample, ans, cols = {}, None, {}, {}
    for line in open(os.path.join(GOLDEN, "%s_answers.txt" % name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "sample":
            sample = np.array([int(x) for x in f[1:]], dtype=np.int64)
        elif f[0] == "A":
            ans[int(f[1])] = [int(x) for x in f[2:]]
        elif f[0] == "D":
            cols[int(f[1])] = {int(x) for x in f[2:]}
        else:
            hdr[f[0]] = f[1]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(reads.offsets, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(reads.seqs, dtype=np.uint8).tobytes())
    assert h.hexdigest() == hdr["reads_sha256"], "the workload's reads differ from the stored answers' reads"
    assert int(hdr["reads"]) == reads.n
    return sample, ans, cols


def test_k1000_kmer_queries_full():
    """K = 1,000 workload in full: the whole index against the oracle's
    (sampled BFUs), 10^7 k-mer queries, 20,000 checked one by one."""
    import torch
    w = gen.workload(2)
    idx = rb.Rambo(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    build_gpu(idx, w.docs, 0, w.K, 250)
    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    for c0 in range(0, w.K, 250):
        o.build_docs(w.docs.docs(c0, 250), w.docs.length, c0, 250)
    bits = o.bits()
    rng = np.random.default_rng(7)
    for k in rng.choice(w.R * w.B, 24, replace=False):
        r, b = divmod(int(k), w.B)
        assert np.array_equal(idx.dump_bfu(r, b), bits[r, b]), (r, b)
    q, src = gen.kmer_queries(w.docs, w.kmer_qseed, w.n_kmer_queries, 0.5)
    got = idx.query_kmers(to_dev(q))
    sample = rng.choice(q.size, 20_000, replace=False)
    want = o.query_kmers(q[sample], oracle.MODE_DEF)
    got_h = got.cpu().numpy().view(np.uint64)
    assert np.array_equal(got_h[sample], want)
    # every present query reports its source document
    pres = np.nonzero(src >= 0)[0]
    s = src[pres]
    srcbits = (got_h[pres, s >> 6] >> (s & 63).astype(np.uint64)) & np.uint64(1)
    assert srcbits.all()
    # either strand gives the same answers
    got_rc = idx.query_kmers(to_dev(_ref.revcomp_np(q)))
    assert torch.equal(got, got_rc)
    idx.close()


def test_k10000_reads_full():
    """K = 10,000 workload at full size (40 GiB index, 100,000 reads),
    plain and batched (autotuned) forms."""
    import torch
    w = gen.workload(3)
    idx = rb.Rambo(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    build_gpu(idx, w.docs, 0, w.K, 500)
    reads = gen.reads(w.docs, w.reads, w.n_reads)
    seqs, offs = to_dev(reads.seqs), to_dev(reads.offsets)
    idx.set_mode(rb.MODE_PLAIN)
    plain = idx.query_seqs(seqs, offs)
    idx.set_mode(rb.MODE_BATCHED)
    batched = idx.query_seqs(seqs, offs)  # autotunes, then runs the tuned shape
    batched = idx.query_seqs(seqs, offs)
    assert torch.equal(plain, batched)
    got = plain.cpu().numpy().view(np.uint64)
    # zero false negatives: a clean read reports its source document
    clean = np.nonzero((reads.src >= 0) & (reads.nerr == 0))[0]
    assert clean.size > 10_000
    for i in clean:
        d = int(reads.src[i])
        assert (got[i, d >> 6] >> np.uint64(d & 63)) & np.uint64(1), i
    # the oracle's whole answers for 10,000 sampled reads, and the answers of
    # sampled documents (covering all four 32-bit row words in every
    # repetition) on every read
    sample, ans, cols = load_golden("k10000", reads)
    assert sample.size == 10_000 and len(ans) > 1000 and len(cols) >= 32
    for i in sample:
        assert sorted(_ref.bits_to_ids(got[i], w.K)) == ans.get(int(i), []), int(i)
    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed, alloc_bits=False)
    phis = o.phis()
    for d, rs in cols.items():
        assert set(np.nonzero(bit_of(got, d))[0].tolist()) == rs, d
    assert {int(phis[r, d]) // 32 for d in cols for r in range(w.R)} == {0, 1, 2, 3}
    # whole BFUs of sampled cells, built by the oracle, and those documents'
    # answers on every read from them
    docs = [int(reads.src[clean[0]]), 4321, 9876]
    cells = [(r, int(phis[r, d])) for d in docs for r in range(w.R)]
    F = oracle_cells(o, w.docs, cells, w.docs.n_docs, phis)
    for (r, b), f in F.items():
        assert np.array_equal(idx.dump_bfu(r, b), f), (r, b)
    ans = doc_answers(o, F, phis, docs, reads)
    for d in docs:
        assert np.array_equal(bit_of(got, d), ans[d]), d
    assert ans[docs[0]].sum() > 0
    # strand invariance on a sample
    pick = np.arange(0, reads.n, 20)
    s2, o2 = make_reads([_ref.revcomp_seq(reads.read(i)) for i in pick])
    idx.set_mode(rb.MODE_PLAIN)
    rc = to_host_u64(idx.query_seqs(to_dev(s2), to_dev(o2)))
    assert np.array_equal(rc, got[pick])
    idx.close()


def test_k101000_streaming_and_id_lists_full():
    """K = 101,000 workload (96 GiB index): build of 100,000 documents,
    streaming insertion of 1,000 new ones, 10^6 reads answered as id lists."""
    import torch
    w = gen.workload(5)
    idx = rb.Rambo(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    build_gpu(idx, w.docs, 0, w.docs.n_docs, 2000)
    s0, ns = w.stream_docs
    # reads drawn from the streamed documents, error-free, before and after
    from dataclasses import replace
    rm_new = replace(w.reads, src_lo=s0, src_hi=s0 + ns, frac_doc=1.0, err_lo=0.0, err_hi=0.0,
                     qseed=w.reads.qseed + 1)
    new_reads = gen.reads(w.docs, rm_new, 2000)
    ns_, no_ = to_dev(new_reads.seqs), to_dev(new_reads.offsets)
    before = to_host_u64(idx.query_seqs(ns_, no_))
    src = new_reads.src
    hit_before = np.array([(before[i, d >> 6] >> np.uint64(d & 63)) & np.uint64(1) for i, d in enumerate(src)])
    build_gpu(idx, w.docs, s0, ns, 500)
    after = to_host_u64(idx.query_seqs(ns_, no_))
    hit_after = np.array([(after[i, d >> 6] >> np.uint64(d & 63)) & np.uint64(1) for i, d in enumerate(src)])
    assert hit_after.all()
    assert hit_before.sum() <= 2  # only false positives before the insertion
    # sampled cells after streaming, against the oracle
    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed, alloc_bits=False)
    phis = o.phis()
    docs = [int(src[0]), 12345]
    cells = [(r, int(phis[r, d])) for d in docs for r in range(w.R)]
    F = oracle_cells(o, w.docs, cells, s0 + ns, phis)
    for (r, b), f in F.items():
        assert np.array_equal(idx.dump_bfu(r, b), f), (r, b)
    # 10^6 reads in the batched form, as id lists
    reads = gen.reads(w.docs, w.reads, w.n_reads)
    seqs, offs = to_dev(reads.seqs), to_dev(reads.offsets)
    idx.set_mode(rb.MODE_BATCHED)
    scratch = torch.empty((reads.n, idx.W), dtype=torch.int64, device="cuda")
    ids, id_off = idx.query_seqs_ids(seqs, offs, ids_cap=50_000_000, scratch=scratch)
    ids, id_off = ids.cpu().numpy(), id_off.cpu().numpy()
    counts = np.diff(id_off)
    assert counts.sum() == ids.size
    # the id lists are the bitsets' set bits, ascending (rows of reads with
    # no id are not written in id-list mode)
    for i in np.nonzero(counts)[0][:2000]:
        lst = ids[id_off[i]:id_off[i + 1]]
        assert np.all(np.diff(lst) > 0)
        row = scratch[i].cpu().numpy().view(np.uint64)
        assert sorted(_ref.bits_to_ids(row, idx.K)) == lst.tolist()
    # and equal the bitset query's answers, read by read
    bits = to_host_u64(idx.query_seqs(seqs, offs))
    for i in range(0, reads.n, 97):
        assert ids[id_off[i]:id_off[i + 1]].tolist() == sorted(_ref.bits_to_ids(bits[i], idx.K)), i
    # sampled documents against the oracle, for every read
    ans = doc_answers(o, F, phis, docs, reads)
    read_of = np.repeat(np.arange(reads.n), counts)  # the read each listed id belongs to

    def column(d):
        col = np.zeros(reads.n, dtype=bool)
        col[read_of[ids == d]] = True
        return col
    for d in docs:
        assert np.array_equal(column(d), ans[d]), d
    # the oracle's whole answers for 10,000 sampled reads, and the answers of
    # sampled documents (covering all eight 16-byte row segments in every
    # repetition) on every read
    sample, gans, gcols = load_golden("k101000", reads)
    assert sample.size == 10_000 and len(gcols) >= 16
    for i in sample:
        assert ids[id_off[i]:id_off[i + 1]].tolist() == gans.get(int(i), []), int(i)
    for d, rs in gcols.items():
        assert set(np.nonzero(column(d))[0].tolist()) == rs, d
    assert {int(phis[r, d]) // 128 for d in gcols for r in range(w.R)} == set(range(8))
    clean = np.nonzero((reads.src >= 0) & (reads.nerr == 0))[0]
    assert clean.size > 1000
    for i in clean[:5000]:
        lst = ids[id_off[i]:id_off[i + 1]]
        assert int(reads.src[i]) in set(lst.tolist())
    idx.close()


@pytest.mark.parametrize("name", ["wiki", "clueweb"])
def test_web_term_workloads_full(name):
    """The two web-document term indexes at their full size (51-61 MB, which
    the oracle builds whole): every BFU bit, 20,000 single-term queries and
    5,000 term sets bit-exact; present terms and phrases find their source."""
    w = gen.term_workload(name)
    terms, offs = w.docs.docs()
    idx = rb.Rambo(w.K, w.B, w.R, w.m, w.eta, w.index_seed, opaque_terms=True)
    idx.insert_batch(to_dev(np.arange(w.K, dtype=np.uint64)), to_dev(offs), to_dev(terms))
    idx.sync()
    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    o.build_term_docs(terms, offs)
    assert np.array_equal(idx.bfu_major(), o.bits())
    q, src = w.docs.term_queries(w.qseed, 20_000, 0.5)
    want = o.query_terms(q, oracle.MODE_ALG2)
    got = to_host_u64(idx.query_kmers(to_dev(q)))
    assert np.array_equal(got, want)
    for i in np.nonzero(src >= 0)[0]:
        assert bit_of(got[i:i + 1], int(src[i]))[0]
    pt, po, ps = w.docs.phrases(w.qseed + 1, 5000, 2, 8, 0.5)
    want2, _ = o.query_termsets(pt, po, oracle.MODE_ALG2, early_exit=True)
    got2 = to_host_u64(idx.query_term_sets(to_dev(pt), to_dev(po)))
    assert np.array_equal(got2, want2)
    for i in np.nonzero(ps >= 0)[0]:
        assert bit_of(got2[i:i + 1], int(ps[i]))[0]
    idx.close()
