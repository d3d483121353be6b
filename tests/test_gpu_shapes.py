"""Index shapes away from the workloads': every B from a single cell to a
two-row-word split and past 1,024 (rows of 1 to 64 words), R from 1 to 8,
eta from 1 to 16 (the generic row loop above 3), m not a power of two (the
multiply-high range reduction), K not a multiple of 64 (result padding).
Every shape: the whole index against the oracle's bits on sampled BFUs, and
every read in both forms, every resolve strategy and schedule, with and
without early exit, against the oracle, as bitsets and (scout schedule) as
id lists."""
import numpy as np
import pytest

import gen
import oracle
from paper_1910_04358_amd import rambo as rb
from tests.gpu_util import build_gpu_seqs, build_oracle, reads_to_dev, to_host_u64

pytestmark = pytest.mark.gpu

# (K, B, R, m, eta)
SHAPES = [
    (70, 1, 3, 50_021, 2),        # one cell: every document in it
    (130, 3, 8, 100_003, 1),      # eight repetitions, one hash
    (257, 33, 2, 262_139, 4),     # two-word rows, eta = 4 (generic loop)
    (300, 129, 5, 300_007, 5),    # rows of 8 words, eta = 5
    (640, 300, 3, 1 << 19, 2),    # rows of 16 words (4 lanes per term)
    (900, 2048, 2, 400_009, 3),   # rows of 64 words (16 lanes per term)
    (200, 50, 3, 150_001, 16),    # the largest eta
    (96, 8192, 2, 1 << 18, 7),    # the largest B: rows of 256 words (64 lanes per term)
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "K%d-B%d-R%d-m%d-eta%d" % s)
def test_unusual_shapes_bit_exact(shape):
    K, B, R, m, eta = shape
    seed = 9000 + B
    dm = gen.DocModel(seed=B, n_docs=K, length=3_000, docs_per_anc=10, mu_lo=0.01, mu_hi=0.01)
    rm = gen.ReadModel(qseed=B + 1, src_lo=0, src_hi=K, len_kind=0, median=200, sigma=0.8, lo=31, hi=2_000,
                       err_lo=0.0, err_hi=0.01)
    idx = rb.Rambo(K, B, R, m, eta, seed)
    build_gpu_seqs(idx, dm, 0, K)
    o = build_oracle((K, B, R, m, eta, seed), dm)
    bits = o.bits()
    rng = np.random.default_rng(B)
    for r, b in {(int(rng.integers(R)), int(rng.integers(B))) for _ in range(12)}:
        assert np.array_equal(idx.dump_bfu(r, b), bits[r, b]), (r, b)
    reads = gen.reads(dm, rm, 400)
    want, _ = o.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2, early_exit=True)
    assert want.any(axis=1).sum() > 10
    want_bits = np.unpackbits(want.view(np.uint8), axis=1, bitorder="little")[:, :K]
    want_ids = [np.nonzero(row)[0].tolist() for row in want_bits]
    total = int(want_bits.sum())
    seqs, offs = reads_to_dev(reads)
    for mode in (rb.MODE_PLAIN, rb.MODE_BATCHED):
        idx.set_mode(mode)
        for resolve in (rb.RESOLVE_AUTO, rb.RESOLVE_DENSE, rb.RESOLVE_CANDIDATE):
            idx.set_resolve(resolve)
            for ee in (True, False):
                idx.set_early_exit(ee)
                for sched in (0, 1, 2):
                    t = idx.get_tune()
                    t.sched = sched
                    idx.set_tune(t)
                    got = to_host_u64(idx.query_seqs(seqs, offs))
                    bad = np.nonzero((got != want).any(axis=1))[0]
                    assert bad.size == 0, (mode, resolve, ee, sched, bad[:5])
                    if sched == 2:
                        # id lists (in the batched form the scout pass then
                        # walks each read one window per round)
                        ids, id_off = idx.query_seqs_ids(seqs, offs, ids_cap=total)
                        ids, id_off = ids.cpu().numpy(), id_off.cpu().numpy()
                        for i in range(reads.n):
                            assert ids[id_off[i]:id_off[i + 1]].tolist() == want_ids[i], (mode, resolve, ee, i)
    idx.set_early_exit(True)
    # single k-mer queries as well
    q, _ = gen.kmer_queries(dm, B + 2, 500, 0.5)
    idx.set_resolve(rb.RESOLVE_AUTO)
    assert np.array_equal(idx.query_kmers_host(q), o.query_kmers(q))
    idx.close()


@pytest.mark.parametrize("shape", [(640, 300, 3, 1 << 19, 2), (900, 2048, 2, 400_009, 3)],
                         ids=lambda s: "K%d-B%d" % s[:2])
def test_streaming_then_fold_wide_rows(shape):
    """Half the documents, then the rest streamed into the resident index
    (equal to the oracle's build of all), then two folds (rows shrink from 16
    to 4 words, or 64 to 16): every sampled BFU and every read equal the
    oracle's fold."""
    K, B, R, m, eta = shape
    seed = 9100 + B
    dm = gen.DocModel(seed=B + 7, n_docs=K, length=3_000, docs_per_anc=10, mu_lo=0.01, mu_hi=0.01)
    rm = gen.ReadModel(qseed=B + 8, src_lo=0, src_hi=K, len_kind=0, median=200, sigma=0.8, lo=31, hi=2_000,
                       err_lo=0.0, err_hi=0.01)
    idx = rb.Rambo(K, B, R, m, eta, seed)
    build_gpu_seqs(idx, dm, 0, K // 2)
    build_gpu_seqs(idx, dm, K // 2, K - K // 2)
    o = build_oracle((K, B, R, m, eta, seed), dm)
    reads = gen.reads(dm, rm, 300)
    seqs, offs = reads_to_dev(reads)
    rng = np.random.default_rng(B)
    for _ in range(2):
        idx.fold()
        o = o.fold()
        assert idx.B == o.B
        bits = o.bits()
        for r, b in {(int(rng.integers(R)), int(rng.integers(idx.B))) for _ in range(10)}:
            assert np.array_equal(idx.dump_bfu(r, b), bits[r, b]), (idx.B, r, b)
        want, _ = o.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2)
        for mode in (rb.MODE_PLAIN, rb.MODE_BATCHED):
            idx.set_mode(mode)
            assert np.array_equal(to_host_u64(idx.query_seqs(seqs, offs)), want), (idx.B, mode)
    idx.close()
