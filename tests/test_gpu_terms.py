"""Opaque-term indexes (documents as sets of word ids, the document indexing
setting of Section 5.4) and term-set queries, through the C ABI, bit-exact
against the oracle's term functions on the same generated inputs: the whole
index, single terms under every resolve strategy, term sets with and without
early exit, rows of 1 to 256 words, k-mer term sets on a k-mer index, and the
errors of the sequence entry points on a term index."""
import numpy as np
import pytest

import gen
import oracle
from paper_1910_04358_amd import rambo as rb
from tests import _ref
from tests.gpu_util import to_dev, to_host_u64

pytestmark = pytest.mark.gpu

# (K, B, R, m, eta, doc model): rows of 1, 4 and 256 words (B = 32, 100, 5000)
CASES = {
    "rw1": (400, 32, 3, 1 << 13, 2, gen.TermDocModel(seed=1301, n_docs=400, mean_terms=60, vocab=20_000)),
    "rw4": (1500, 100, 2, 1 << 14, 2, gen.TermDocModel(seed=1302, n_docs=1500, mean_terms=120, vocab=60_000)),
    "rw256": (3000, 5000, 3, 1 << 12, 2, gen.TermDocModel(seed=1303, n_docs=3000, mean_terms=45, vocab=40_000)),
}
_built = {}


def setup_case(name):
    if name in _built:
        return _built[name]
    K, B, R, m, eta, dm = CASES[name]
    seed = 6100 + len(_built)
    terms, offs = dm.docs()
    idx = rb.Rambo(K, B, R, m, eta, seed, opaque_terms=True)
    ids = np.arange(K, dtype=np.uint64)
    idx.insert_batch(to_dev(ids), to_dev(offs), to_dev(terms))
    idx.sync()
    o = oracle.Oracle(K, B, R, m, eta, seed)
    o.build_term_docs(terms, offs)
    _built[name] = (idx, o, dm, terms, offs)
    return _built[name]


@pytest.mark.parametrize("name", list(CASES))
def test_term_index_bits_match_oracle(name):
    idx, o, dm, terms, offs = setup_case(name)
    bits = o.bits()
    rng = np.random.default_rng(2)
    pairs = [(r, b) for r in range(idx.R) for b in range(idx.B)]
    if len(pairs) > 60:
        pairs = [pairs[i] for i in rng.choice(len(pairs), 60, replace=False)]
    for r, b in pairs:
        assert np.array_equal(idx.dump_bfu(r, b), bits[r, b]), (r, b)


@pytest.mark.parametrize("name", list(CASES))
def test_single_terms_every_resolve(name):
    idx, o, dm, terms, offs = setup_case(name)
    q, src = dm.term_queries(71, 3000, 0.5)
    q[:3] = [0, (1 << 64) - 1, 1 << 62]  # any 64-bit value is a term
    src[:3] = -1
    want = o.query_terms(q, oracle.MODE_ALG2)
    for resolve in (rb.RESOLVE_AUTO, rb.RESOLVE_DENSE, rb.RESOLVE_CANDIDATE):
        idx.set_resolve(resolve)
        got = to_host_u64(idx.query_kmers(to_dev(q)))
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, (name, resolve, bad[:5])
    idx.set_resolve(rb.RESOLVE_AUTO)
    idx.sync()  # no value was rejected
    for i in np.nonzero(src >= 0)[0][:200]:
        d = int(src[i])
        assert (got[i, d >> 6] >> np.uint64(d & 63)) & np.uint64(1)


@pytest.mark.parametrize("name", list(CASES))
def test_term_sets_equal_oracle(name):
    idx, o, dm, terms, offs = setup_case(name)
    pt, po, ps = dm.phrases(72, 1500, 1, 12, 0.6)
    # an empty set and a long set (several steps of 64 terms)
    extra = terms[offs[5]:offs[5] + 150]
    pt = np.concatenate([pt, extra])
    po = np.concatenate([po, [po[-1], po[-1] + extra.size]]).astype(np.uint64)
    want, _ = o.query_termsets(pt, po, oracle.MODE_ALG2, early_exit=True)
    assert _ref.bits_to_ids(want[-2], idx.K) == set(range(idx.K))
    for ee in (True, False):
        idx.set_early_exit(ee)
        for resolve in (rb.RESOLVE_AUTO, rb.RESOLVE_CANDIDATE):
            idx.set_resolve(resolve)
            got = to_host_u64(idx.query_term_sets(to_dev(pt), to_dev(po)))
            bad = np.nonzero((got != want).any(axis=1))[0]
            assert bad.size == 0, (name, ee, resolve, bad[:5])
    idx.set_early_exit(True)
    idx.set_resolve(rb.RESOLVE_AUTO)
    for i in np.nonzero(ps >= 0)[0][:200]:
        d = int(ps[i])
        assert (got[i, d >> 6] >> np.uint64(d & 63)) & np.uint64(1)


def test_term_sets_on_a_kmer_index():
    """On a k-mer index a term set is a set of 31-mer codes of either strand;
    a read's valid windows as a set answer what the read answers, and a
    value >= 4^31 empties its set and is reported."""
    from tests.test_gpu_parity import setup_case as kmer_case
    from tests.gpu_util import make_reads
    idx, o, dm, reads, want = kmer_case("rw4")
    sets, lens = [], []
    for i in range(300):
        codes = _ref.seq_terms(reads.read(i))
        if i % 2:
            codes = _ref.revcomp_np(codes)
        sets.append(codes)
        lens.append(codes.size)
    pt = np.concatenate(sets).astype(np.uint64)
    po = np.zeros(len(sets) + 1, dtype=np.uint64)
    po[1:] = np.cumsum(lens)
    got = to_host_u64(idx.query_term_sets(to_dev(pt), to_dev(po)))
    assert np.array_equal(got, want[:300])
    bad = np.array([5, 1 << 62, 9], dtype=np.uint64)
    got2 = to_host_u64(idx.query_term_sets(to_dev(bad), to_dev(np.array([0, 3], dtype=np.uint64))))
    assert not got2.any()
    with pytest.raises(rb.RamboError) as e:
        idx.sync()
    assert e.value.status == rb.EINVAL


def test_term_index_rejects_sequence_entry_points():
    idx, o, dm, terms, offs = setup_case("rw1")
    s = to_dev(np.frombuffer(b"ACGT" * 20, dtype=np.uint8).copy())
    off = to_dev(np.array([0, 80], dtype=np.uint64))
    with pytest.raises(rb.RamboError) as e:
        idx.query_seqs(s, off)
    assert e.value.status == rb.EINVAL
    with pytest.raises(rb.RamboError):
        idx.insert_seqs(to_dev(np.array([0], dtype=np.uint64)), s, off)
    with pytest.raises(rb.RamboError):
        rb.Server(idx)
    # host insertion takes any 64-bit value on a term index
    idx2 = rb.Rambo(10, 4, 2, 1 << 10, 2, 5, opaque_terms=True)
    o2 = oracle.Oracle(10, 4, 2, 1 << 10, 2, 5)
    vals = np.array([0, 1 << 62, (1 << 64) - 1, 12345], dtype=np.uint64)
    idx2.insert(3, vals)
    o2.insert_terms(3, vals)
    assert np.array_equal(idx2.bfu_major(), o2.bits())
    idx2.close()
