"""Pins of the CPU oracle against what the paper and the mathematics fix:
hand-derived encodings, published SplitMix64 outputs, brute-force set
membership, the Bloom filter occupancy and false-positive laws (Section 2.1,
Lemma 4.1), Algorithm 2 versus the per-document definition, streaming
insertion, strand invariance and folding (Section 5.3)."""
import math
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import twin
from tests import _ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P61 = (1 << 61) - 1


# ---------------------------------------------------------------- encoding
def test_encoding_golden():
    n = 0
    for line in open(os.path.join(GOLDEN, "kmer_canonical.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        w, c = line.split()
        got = oracle.window(w.encode())
        if c == "-":
            assert got is None, w
        else:
            assert got == int(c.translate(str.maketrans("ACGT", "0123")), 4), w
        n += 1
    assert n >= 10


def test_revcomp_identities():
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 1 << 62, size=2000, dtype=np.uint64)
    rcs = _ref.revcomp_np(xs)
    for x, r in zip(xs[:300].tolist(), rcs[:300].tolist()):
        assert oracle.revcomp(x) == r
        assert oracle.revcomp(r) == x
        assert oracle.canon(x) == oracle.canon(r) == min(x, r)
        assert x != r  # odd k: no 31-mer is its own reverse complement


def test_generator_codes_vs_oracle_windows():
    dm = gen.DocModel(seed=5, n_docs=1, length=2000)
    s = dm.doc(0)
    codes = dm.window_codes(0)
    canon = _ref.canon_np(codes)
    for p in range(0, 1970, 37):
        assert oracle.window(s, p) == int(canon[p])
    assert np.array_equal(_ref.seq_terms(s), canon)


# ---------------------------------------------------------------- hashing
def test_parameters_drawn_from_published_splitmix_outputs():
    v = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
         if l.strip() and not l.startswith("#")]
    o = oracle.Oracle(10, 4, 1, 1 << 20, 1, 1234567)
    p = o.params()
    assert int(p["pa"][0]) == 1 + v[0] % (P61 - 1)
    assert int(p["pb"][0]) == v[1] % P61
    assert int(p["Alo"][0]) == v[2] and int(p["Ahi"][0]) == v[3] and int(p["Clo"][0]) == v[4]


def test_phi_two_universal():
    """Carter-Wegman: for fixed d1 != d2, over random seeds, the collision
    probability is about 1/B; every cell gets about K/B documents."""
    B, trials, hits = 16, 4000, 0
    for s in range(trials):
        o = oracle.Oracle(1000, B, 1, 64, 1, 10_000 + s, alloc_bits=False)
        hits += o.phi(0, 3) == o.phi(0, 977)
    assert abs(hits / trials - 1 / B) < 4 * math.sqrt((1 / B) * (1 - 1 / B) / trials)
    o = oracle.Oracle(100_000, 100, 3, 64, 1, 7, alloc_bits=False)
    for r in range(3):
        cnt = np.bincount([o.phi(r, d) for d in range(0, 100_000, 7)], minlength=100)
        exp = cnt.sum() / 100
        chi2 = ((cnt - exp) ** 2 / exp).sum()
        assert chi2 < 99 + 6 * math.sqrt(2 * 99)


def test_h_strongly_universal_small_range():
    """Multiply-add-shift: for fixed x != y, over random parameters, the pair
    (h(x), h(y)) is uniform on [m]^2; with m = 16 collisions occur with
    probability 1/16 and each value with probability 1/16."""
    m, trials = 16, 6000
    coll, val = 0, np.zeros(m, dtype=np.int64)
    x, y = 0x123456789ABCDEF & ((1 << 62) - 1), 0x3ABCDEF012345678 & ((1 << 62) - 1)
    for s in range(trials):
        o = oracle.Oracle(10, 2, 1, m, 1, 50_000 + s, alloc_bits=False)
        hx, hy = o.h(0, 0, x), o.h(0, 0, y)
        coll += hx == hy
        val[hx] += 1
    assert abs(coll / trials - 1 / m) < 4 * math.sqrt((1 / m) * (1 - 1 / m) / trials)
    exp = trials / m
    assert ((val - exp) ** 2 / exp).sum() < 15 + 6 * math.sqrt(30)


def test_h_positions_uniform_and_in_range():
    o = oracle.Oracle(10, 2, 2, 1000, 2, 3, alloc_bits=False)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 1 << 62, size=20000, dtype=np.uint64).tolist()
    pos = np.array([o.h(1, 1, x) for x in xs])
    assert pos.min() >= 0 and pos.max() < 1000
    cnt = np.bincount(pos // 50, minlength=20)
    exp = 1000
    assert ((cnt - exp) ** 2 / exp).sum() < 19 + 6 * math.sqrt(38)


def test_twin_agrees_on_hashes_and_queries():
    K, B, R, m, eta = 12, 3, 2, 4096, 2
    o = oracle.Oracle(K, B, R, m, eta, 77)
    t = twin.Twin(K, B, R, m, eta, 77)
    rng = np.random.default_rng(2)
    for x in rng.integers(0, 1 << 62, size=50, dtype=np.uint64).tolist():
        for r in range(R):
            for j in range(eta):
                assert o.h(r, j, x) == t.h(r, j, x)
    for d in range(K):
        for r in range(R):
            assert o.phi(r, d) == t.phi(r, d)
    dm = gen.DocModel(seed=8, n_docs=K, length=120, docs_per_anc=3, mu_lo=0.05, mu_hi=0.05)
    for d in range(K):
        s = dm.doc(d)
        o.insert_seq(d, s)
        t.insert_terms(d, twin.kmer_terms(s))
    bits = o.bits()
    for r in range(R):
        for b in range(B):
            got = set(np.nonzero(np.unpackbits(bits[r, b].view(np.uint8), bitorder="little")[:m])[0].tolist())
            assert got == t.bfu[r][b]
    for d in range(0, K, 2):
        s = dm.doc(d, 10, 40)
        assert _ref.bits_to_ids(o.query_seq(s), K) == t.query_terms(twin.kmer_terms(s))


# ---------------------------------------------------------------- structure
def _small_index(K=40, B=5, R=3, m=1 << 26, eta=2, L=300, seed=21):
    dm = gen.DocModel(seed=seed, n_docs=K, length=L, docs_per_anc=4, mu_lo=0.03, mu_hi=0.03)
    o = oracle.Oracle(K, B, R, m, eta, seed + 1)
    docs = dm.docs(0, K)
    o.build_docs(docs, L, 0, K, nthreads=4)
    table = _ref.KmerTable({d: _ref.seq_terms(docs[d * L:(d + 1) * L].tobytes()) for d in range(K)})
    return dm, o, table


def test_exact_partition_brute_force():
    """With m far above the number of inserted terms, Bloom filters make no
    errors w.h.p., so the answer must equal RAMBO over exact sets: d is kept
    iff, in every repetition, the union of the sets of d's cell holds every
    term (Section 3: union within a repetition, intersection across). The
    truth (documents containing every term) must be inside it."""
    K, B, R = 40, 5, 3
    dm, o, table = _small_index(K=K, B=B, R=R)
    phis = o.phis()
    cell_sets = {(r, b): set().union(*[table.sets[d] for d in range(K) if phis[r, d] == b])
                 for r in range(R) for b in range(B)}
    rng = np.random.default_rng(3)
    n_nonempty = 0
    for q in range(200):
        d = int(rng.integers(K))
        st = int(rng.integers(0, 300 - 40))
        s = dm.doc(d, st, int(rng.integers(31, 40)))
        Q = set(_ref.seq_terms(s).tolist())
        ex = {e for e in range(K) if all(Q <= cell_sets[(r, phis[r, e])] for r in range(R))}
        truth = table.truth_seq(np.array(sorted(Q), dtype=np.uint64), K)
        got = _ref.bits_to_ids(o.query_seq(s), K)
        assert truth <= ex
        assert got == ex, (q, d)
        n_nonempty += len(got) > 0
    assert n_nonempty == 200
    # single terms, through both the definition and Algorithm 2
    for x in list(table.sets[0])[:50]:
        ex = {e for e in range(K) if all(x in cell_sets[(r, phis[r, e])] for r in range(R))}
        assert _ref.bits_to_ids(o.query_kmer(x), K) == ex
        assert _ref.bits_to_ids(o.query_kmer(x, oracle.MODE_ALG2), K) == ex


@pytest.fixture(scope="module")
def c1():
    w = gen.workload(1)
    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed)
    docs = w.docs.docs(0, w.docs.n_docs)
    L = w.docs.length
    o.build_docs(docs, L, 0, w.docs.n_docs)
    table = _ref.KmerTable({d: _ref.seq_terms(docs[d * L:(d + 1) * L].tobytes()) for d in range(w.K)})
    q, src = gen.kmer_queries(w.docs, w.kmer_qseed, w.n_kmer_queries, 0.5)
    res = o.query_kmers(q, oracle.MODE_DEF)
    return w, o, docs, table, q, src, res


def test_c1_zero_false_negatives(c1):
    w, o, docs, table, q, src, res = c1
    cq = _ref.canon_np(q)
    for i in range(q.size):
        truth = set(table.docs_with(int(cq[i])).tolist())
        got = _ref.bits_to_ids(res[i], w.K)
        assert truth <= got
        if src[i] >= 0:
            assert int(src[i]) in truth


def test_c1_alg2_equals_definition(c1):
    w, o, docs, table, q, src, res = c1
    res2 = o.query_kmers(q[:3000], oracle.MODE_ALG2)
    assert np.array_equal(res2, res[:3000])
    # padding bits above K stay zero
    assert np.all(res[:, -1] >> np.uint64(w.K & 63) == 0)


def test_c1_bloom_occupancy_law(c1):
    """Section 2.1: after inserting n distinct keys with eta hashes into m
    bits, the expected number of set bits is m (1 - (1 - 1/m)^(eta n))."""
    w, o, docs, table, q, src, res = c1
    phis = o.phis()
    for r in range(w.R):
        for b in range(w.B):
            n_b = len(set().union(*[table.sets[d] for d in range(w.K) if phis[r, d] == b]))
            exp = w.m * (1 - (1 - 1 / w.m) ** (w.eta * n_b))
            q_ = exp / w.m
            sd = math.sqrt(w.m * q_ * (1 - q_))
            assert abs(o.bfu_popcount(r, b) - exp) < 6 * sd, (r, b)


def test_c1_false_positive_law(c1):
    """Fresh terms (absent from every document): document d is reported with
    probability prod_r fill(r, phi_r(d))^eta (Section 2.1 per BFU, independent
    repetitions), and on average about p^R (Lemma 4.1 with V = 0)."""
    w, o, docs, table, q, src, res = c1
    cq = _ref.canon_np(q)
    fresh = np.nonzero((src < 0) & (table.multiplicity(cq) == 0))[0]
    assert fresh.size > 4500
    phis = o.phis()
    fill = np.array([[o.bfu_popcount(r, b) / w.m for b in range(w.B)] for r in range(w.R)])
    pdoc = np.prod([fill[r, phis[r]] ** w.eta for r in range(w.R)], axis=0)
    bits = np.unpackbits(res[fresh].view(np.uint8), axis=1, bitorder="little")[:, :w.K]
    observed = bits.sum()
    expected = fresh.size * pdoc.sum()
    assert abs(observed - expected) < max(8 * math.sqrt(expected), 0.08 * expected), (observed, expected)
    p = (fill ** w.eta).mean()
    lemma = fresh.size * w.K * p ** w.R
    assert abs(observed - lemma) < 0.2 * lemma, (observed, lemma)


def test_c1_lemma_4_1_multiplicity_one(c1):
    """Present terms of multiplicity V = 1 (i.i.d. documents): a document that
    does not hold the term is reported iff, in every repetition, it shares the
    true document's cell or its own BFU gives a false positive. Sharp form
    with the realised cells and fills; Lemma 4.1's F_p on average."""
    w, o, docs, table, q, src, res = c1
    cq = _ref.canon_np(q)
    mult = table.multiplicity(cq)
    pres = np.nonzero((src >= 0) & (mult == 1))[0]
    phis = o.phis()
    fill = np.array([[o.bfu_popcount(r, b) / w.m for b in range(w.B)] for r in range(w.R)])
    obs = exp = 0.0
    for i in pres:
        t = int(src[i])
        pr = np.ones(w.K)
        for r in range(w.R):
            same = phis[r] == phis[r, t]
            pr *= np.where(same, 1.0, fill[r, phis[r]] ** w.eta)
        pr[t] = 0
        got = _ref.bits_to_ids(res[i], w.K) - {t}
        obs += len(got)
        exp += pr.sum()
    assert abs(obs - exp) < max(8 * math.sqrt(exp), 0.08 * exp), (obs, exp)
    p = (fill ** w.eta).mean()
    Fp = (p * (1 - 1 / w.B) + 1 - (1 - 1 / w.B)) ** w.R
    lemma = pres.size * (w.K - 1) * Fp
    assert abs(obs - lemma) < 0.35 * lemma, (obs, lemma)


# ---------------------------------------------------------------- invariants
def test_streaming_insert_equals_batch_build_and_order_independent():
    K, B, R, m, eta, L = 30, 4, 3, 1 << 16, 2, 500
    dm = gen.DocModel(seed=31, n_docs=K, length=L, docs_per_anc=5, mu_lo=0.02, mu_hi=0.02)
    docs = dm.docs(0, K)
    full = oracle.Oracle(K, B, R, m, eta, 9)
    full.build_docs(docs, L, 0, K)
    part = oracle.Oracle(K, B, R, m, eta, 9)
    part.build_docs(docs, L, 0, 20)
    probe = dm.doc(25, 100, 60)
    before = _ref.bits_to_ids(part.query_seq(probe), K)
    for d in range(20, K):
        part.insert_seq(d, docs[d * L:(d + 1) * L].tobytes())
    assert np.array_equal(part.bits(), full.bits())
    after = _ref.bits_to_ids(part.query_seq(probe), K)
    assert 25 in after and 25 not in before
    perm = oracle.Oracle(K, B, R, m, eta, 9)
    for d in np.random.default_rng(4).permutation(K):
        perm.insert_seq(int(d), docs[d * L:(d + 1) * L].tobytes())
    assert np.array_equal(perm.bits(), full.bits())
    # the same document given as k-mer codes (either strand) sets the same bits
    km = oracle.Oracle(K, B, R, m, eta, 9)
    for d in range(K):
        codes = dm.window_codes(d)
        if d % 2:
            codes = _ref.revcomp_np(codes)
        km.insert_kmers(d, codes)
    assert np.array_equal(km.bits(), full.bits())


def test_bfu_is_union_of_document_filters():
    """Section 3: BFU(r, b) is the Bloom filter of the union of its
    documents' sets, i.e. the OR of the single-document filters."""
    K, B, R, m, eta, L = 16, 3, 2, 1 << 14, 2, 300
    dm = gen.DocModel(seed=41, n_docs=K, length=L)
    full = oracle.Oracle(K, B, R, m, eta, 5)
    acc = np.zeros((R, B, full.wpb), dtype=np.uint64)
    for d in range(K):
        s = dm.doc(d)
        full.insert_seq(d, s)
        one = oracle.Oracle(K, B, R, m, eta, 5)
        one.insert_seq(d, s)
        acc |= one.bits()
    assert np.array_equal(acc, full.bits())


def test_strand_invariance_and_empty_queries():
    dm, o, table = _small_index(K=20, B=4, R=2, m=1 << 16, L=400, seed=51)
    rng = np.random.default_rng(5)
    for _ in range(30):
        d = int(rng.integers(20))
        s = dm.doc(d, int(rng.integers(0, 300)), int(rng.integers(31, 100)))
        a = o.query_seq(s)
        assert np.array_equal(a, o.query_seq(_ref.revcomp_seq(s)))
        assert np.array_equal(a, o.query_seq(s.lower()))
        assert np.array_equal(a, o.query_seq(s, oracle.MODE_ALG2, early_exit=True))
        assert np.array_equal(a, o.query_seq(s, oracle.MODE_ALG2, early_exit=False))
    everyone = _ref.ids_to_bits(range(20), 20)
    for s in (b"", b"ACGT" * 7, b"N" * 100, b"ACGTN" * 20):
        assert np.array_equal(o.query_seq(s), everyone)
        assert np.array_equal(o.query_seq(s, oracle.MODE_ALG2), everyone)


def test_invalid_inputs_rejected():
    o = oracle.Oracle(10, 2, 2, 1024, 2, 1)
    with pytest.raises(ValueError):
        o.insert_kmers(0, np.array([1 << 62], dtype=np.uint64))
    with pytest.raises(ValueError):
        o.insert_kmers(10, np.array([5], dtype=np.uint64))
    assert not o.bits().any()


def test_fold_equals_rebuild_with_half_the_cells():
    """Section 5.3 folding: OR-ing BFU(r, b + B/2) onto BFU(r, b) gives the
    index built directly with B/2 cells (same seeds, phi mod B/2)."""
    K, B, R, m, eta, L = 40, 8, 3, 1 << 16, 2, 400
    dm = gen.DocModel(seed=61, n_docs=K, length=L, docs_per_anc=4, mu_lo=0.02, mu_hi=0.02)
    docs = dm.docs(0, K)
    big = oracle.Oracle(K, B, R, m, eta, 13)
    big.build_docs(docs, L, 0, K)
    half = oracle.Oracle(K, B // 2, R, m, eta, 13)
    half.build_docs(docs, L, 0, K)
    f = big.fold()
    assert np.array_equal(f.bits(), half.bits())
    s = dm.doc(7, 50, 80)
    assert np.array_equal(f.query_seq(s), half.query_seq(s))
    assert _ref.bits_to_ids(big.query_seq(s), K) <= _ref.bits_to_ids(f.query_seq(s), K)


# ---------------------------------------------------------------- word terms
# Document indexing with opaque word terms (Section 5.4): the same method with
# the terms taken as they are.
def _term_index(K, B, R, m, eta=2, seed=77, mean=40, vocab=2000, dseed=1201):
    dm = gen.TermDocModel(seed=dseed, n_docs=K, mean_terms=mean, vocab=vocab)
    terms, offs = dm.docs()
    o = oracle.Oracle(K, B, R, m, eta, seed)
    o.build_term_docs(terms, offs)
    sets = [set(terms[offs[d]:offs[d + 1]].tolist()) for d in range(K)]
    return dm, o, terms, offs, sets


def test_terms_equal_kmers_on_canonical_codes():
    """On canonical k-mer codes the term functions are the k-mer functions:
    insertion of canonical codes as terms gives the same bits, and a term
    query of canon(x) answers the k-mer query of x."""
    dm = gen.DocModel(seed=9, n_docs=12, length=3000)
    ok = oracle.Oracle(12, 4, 3, 1 << 16, 2, 31)
    ot = oracle.Oracle(12, 4, 3, 1 << 16, 2, 31)
    for d in range(12):
        codes = dm.window_codes(d)
        ok.insert_kmers(d, _ref.revcomp_np(codes) if d % 2 else codes)
        ot.insert_terms(d, _ref.canon_np(codes))
    assert np.array_equal(ok.bits(), ot.bits())
    q, _ = gen.kmer_queries(dm, 5, 300, 0.5)
    assert np.array_equal(ok.query_kmers(q), ot.query_terms(_ref.canon_np(q)))


def test_terms_exact_partition_brute_force():
    """Word-term documents with m far above the inserted terms (no Bloom
    errors w.h.p.): single terms and term sets give RAMBO over exact sets
    (d kept iff every term is in the union of d's cell in every repetition),
    which contains the truth; Algorithm 2 equals the definition."""
    K, B, R = 60, 7, 3
    dm, o, terms, offs, sets = _term_index(K, B, R, 1 << 24)
    phis = o.phis()
    cell = {(r, b): set().union(*[sets[d] for d in range(K) if phis[r, d] == b]) for r in range(R) for b in range(B)}
    q, src = dm.term_queries(11, 400, 0.5)
    res = o.query_terms(q)
    res2 = o.query_terms(q, oracle.MODE_ALG2)
    assert np.array_equal(res, res2)
    strict = 0
    for i, x in enumerate(q.tolist()):
        ex = {e for e in range(K) if all(x in cell[(r, phis[r, e])] for r in range(R))}
        truth = {e for e in range(K) if x in sets[e]}
        got = _ref.bits_to_ids(res[i], K)
        assert truth <= ex and got == ex, i
        if src[i] >= 0:
            assert int(src[i]) in got
        strict += ex != truth
    assert strict > 0  # the partition does produce false positives here
    pt, po, ps = dm.phrases(12, 200, 2, 6, 0.7)
    got, _ = o.query_termsets(pt, po, oracle.MODE_ALG2, early_exit=True)
    for i in range(200):
        Q = set(pt[po[i]:po[i + 1]].tolist())
        ex = {e for e in range(K) if all(Q <= cell[(r, phis[r, e])] for r in range(R))}
        assert _ref.bits_to_ids(got[i], K) == ex, i
        assert np.array_equal(o.query_termset(pt[po[i]:po[i + 1]], oracle.MODE_DEF), got[i])
        if ps[i] >= 0:
            assert int(ps[i]) in ex


def test_term_sets_are_the_and_of_their_terms():
    """Section 3.3.1 for term sets: the answer is the intersection of the
    terms' answers, whatever their order; the empty set is every document."""
    K = 300
    dm, o, terms, offs, sets = _term_index(K, 20, 2, 1 << 12, mean=60, vocab=5000)
    pt, po, ps = dm.phrases(13, 150, 1, 8, 0.6)
    got, _ = o.query_termsets(pt, po)
    single = o.query_terms(pt)
    rng = np.random.default_rng(4)
    for i in range(150):
        a, b = int(po[i]), int(po[i + 1])
        want = np.bitwise_and.reduce(single[a:b], axis=0)
        assert np.array_equal(got[i], want), i
        perm = pt[a:b][rng.permutation(b - a)]
        assert np.array_equal(o.query_termset(perm, oracle.MODE_ALG2), want)
    allk = o.query_termset(np.zeros(0, dtype=np.uint64), oracle.MODE_ALG2)
    assert _ref.bits_to_ids(allk, K) == set(range(K))


def test_terms_false_positive_law():
    """Fresh terms on a loaded term index: document d is reported with
    probability prod_r fill(r, phi_r(d))^eta (Section 2.1, independent
    repetitions), about p^R on average (Lemma 4.1, V = 0)."""
    K, B, R, m, eta = 400, 10, 2, 4096, 2
    dm, o, terms, offs, sets = _term_index(K, B, R, m, eta=eta, mean=80, vocab=100_000)
    phis = o.phis()
    fill = np.array([[o.bfu_popcount(r, b) / m for b in range(B)] for r in range(R)])
    pdoc = np.prod([fill[r, phis[r]] ** eta for r in range(R)], axis=0)
    allterms = set(terms.tolist())
    q, src = dm.term_queries(14, 4000, 0.0)
    assert all(x not in allterms for x in q.tolist())
    res = o.query_terms(q)
    bits = np.unpackbits(res.view(np.uint8), axis=1, bitorder="little")[:, :K]
    observed, expected = bits.sum(), q.size * pdoc.sum()
    assert abs(observed - expected) < max(8 * math.sqrt(expected), 0.08 * expected), (observed, expected)
    p = (fill ** eta).mean()
    lemma = q.size * K * p ** R
    assert abs(observed - lemma) < 0.2 * lemma, (observed, lemma)


def test_lemma_4_1_across_multiplicities():
    """Lemma 4.1 for any multiplicity V (the curve of Figure 4): a term held
    by V documents is reported for a document that does not hold it with
    probability (1 - (1 - p)(1 - 1/B)^V)^R -- in each repetition the
    document's cell holds one of the V holders, or its Bloom filter errs.
    Documents shaped like the K=1,000 workload (mutant families of one
    ancestor with 1 % substitutions; B=32, R=4, eta=3), in families of 5, 20
    and 50 so that present terms are held by 1 to 50 documents, shorter and
    with a smaller m so that false positives are frequent enough to count at
    V = 1. Present terms are bucketed by their exact V (brute force); per
    bucket the observed count must match the sharp prediction with the
    realised cells and fills, and the lemma with the mean p."""
    B, R, eta, L, m = 32, 4, 3, 2000, 1 << 18
    families = [gen.DocModel(seed=1402 + k, n_docs=500, length=L, docs_per_anc=fam, mu_lo=0.01, mu_hi=0.01)
                for k, fam in enumerate((5, 20, 50))]
    K = 500 * len(families)
    o = oracle.Oracle(K, B, R, m, eta, 2402)
    docs = np.concatenate([dm.docs(0, 500) for dm in families])
    o.build_docs(docs, L, 0, K)
    table = _ref.KmerTable({d: _ref.seq_terms(docs[d * L:(d + 1) * L].tobytes()) for d in range(K)})
    q = np.concatenate([gen.kmer_queries(dm, 3402 + k, 4000, 1.0)[0] for k, dm in enumerate(families)])
    cq = _ref.canon_np(q)
    res = o.query_kmers(cq)
    phis = o.phis()
    fill = np.array([[o.bfu_popcount(r, b) / m for b in range(B)] for r in range(R)])
    fe = fill ** eta                                   # per-BFU false-positive rate of an absent term
    p = fe.mean()
    bits = np.unpackbits(res.view(np.uint8), axis=1, bitorder="little")[:, :K].astype(bool)
    buckets = [(1, 1), (2, 5), (6, 24), (25, 50)]
    stats = {bk: [0.0, 0.0, 0.0] for bk in buckets}    # observed, sharp prediction, lemma
    for i in range(q.size):
        holders = table.docs_with(int(cq[i]))
        V = holders.size
        bk = next((b for b in buckets if b[0] <= V <= b[1]), None)
        if bk is None:
            continue
        assert bits[i, holders].all()                  # no false negative
        non = np.ones(K, dtype=bool)
        non[holders] = False
        pr = np.ones(K)
        for r in range(R):
            hc = np.zeros(B, dtype=bool)
            hc[phis[r, holders]] = True
            pr *= np.where(hc[phis[r]], 1.0, fe[r, phis[r]])
        st = stats[bk]
        st[0] += bits[i, non].sum()
        st[1] += pr[non].sum()
        st[2] += (K - V) * (1 - (1 - p) * (1 - 1 / B) ** V) ** R
    for bk, (obs, sharp, lemma) in stats.items():
        assert sharp > 50, (bk, sharp)
        assert abs(obs - sharp) < max(8 * math.sqrt(sharp), 0.05 * sharp), (bk, obs, sharp)
        assert abs(obs - lemma) < 0.15 * lemma, (bk, obs, lemma)


# ------------------------------------------- sampled BFUs and one repetition
def _reads_with_edges(dm, rm, n):
    reads = gen.reads(dm, rm, n)
    extra = [b"", b"N" * 50, b"ACGT" * 7, dm.doc(3, 10, 31), dm.doc(5, 0, 200).lower()]
    seqs = [reads.read(i) for i in range(reads.n)] + extra
    offs = np.zeros(len(seqs) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(s) for s in seqs])
    return np.frombuffer(b"".join(seqs), dtype=np.uint8).copy(), offs


def test_single_bfu_functions_reproduce_the_oracle():
    """The functions that check sampled documents of indexes too large for
    the oracle -- one BFU built from the documents of its cell, a read tested
    against one filter of repetition r -- reproduce the whole oracle: the
    filter built from cell (r, b)'s documents is BFU(r, b), and ANDing over r
    the tests of document d's filters gives d's answer from the
    per-document definition (Section 3.3.1), for every document and read
    (reads without a term pass vacuously). A filter tested with another
    repetition's hash functions gives other answers, so that slip would
    fail here."""
    K, B, R, m, eta, L = 40, 5, 3, 1 << 14, 2, 600
    dm = gen.DocModel(seed=131, n_docs=K, length=L, docs_per_anc=4, mu_lo=0.02, mu_hi=0.02)
    o = oracle.Oracle(K, B, R, m, eta, 55)
    docs = dm.docs(0, K)
    o.build_docs(docs, L, 0, K)
    bits, phis = o.bits(), o.phis()
    F = {}
    for r in range(R):
        for b in range(B):
            f = o.new_bfu()
            for d in np.nonzero(phis[r] == b)[0]:
                o.bfu_insert_seq(r, f, docs[d * L:(d + 1) * L])
            assert np.array_equal(f, bits[r, b]), (r, b)
            F[(r, b)] = f
    rm = gen.ReadModel(qseed=132, src_lo=0, src_hi=K, len_kind=1, lo=31, hi=200, err_lo=0.0, err_hi=0.02)
    seqs, offs = _reads_with_edges(dm, rm, 300)
    want, _ = o.query_seqs(seqs, offs, oracle.MODE_DEF)
    wbits = np.unpackbits(want.view(np.uint8), axis=1, bitorder="little")[:, :K].astype(bool)
    assert 10 < wbits.sum() < wbits.size
    slip = False
    for d in range(K):
        keep = np.ones(offs.size - 1, dtype=bool)
        for r in range(R):
            t = o.bfu_test_seqs(r, F[(r, int(phis[r, d]))], seqs, offs)
            keep &= t
            other = o.bfu_test_seqs((r + 1) % R, F[(r, int(phis[r, d]))], seqs, offs)
            slip |= not np.array_equal(other, t)
        assert np.array_equal(keep, wbits[:, d]), d
        for i in (0, offs.size - 2, offs.size - 4):
            s = seqs[int(offs[i]):int(offs[i + 1])].tobytes()
            one = all(o.bfu_test_seq(r, F[(r, int(phis[r, d]))], s) for r in range(R))
            assert one == wbits[i, d]
    assert slip
    assert o.bfu_test_seq(0, o.new_bfu(), b"N" * 40)       # no term: vacuously in any filter
    assert not o.bfu_test_seq(0, o.new_bfu(), dm.doc(1, 0, 31))


def test_one_repetition_at_a_time_equals_the_whole_oracle():
    """Algorithm 1 restricted to one repetition, over documents given in
    chunks, fills exactly that repetition's filters; Algorithm 2 taken one
    repetition at a time (each repetition's union of positive cells,
    intersected into the answer) gives the whole oracle's answers in both
    modes, including reads without a term; with m far above the number of
    terms it gives RAMBO over exact sets (brute force)."""
    for (K, B, R, m, eta, L) in ((60, 7, 3, 1 << 13, 2, 500), (50, 4, 2, 1 << 24, 3, 300)):
        dm = gen.DocModel(seed=K + B, n_docs=K, length=L, docs_per_anc=5, mu_lo=0.02, mu_hi=0.02)
        o = oracle.Oracle(K, B, R, m, eta, 71)
        docs = dm.docs(0, K)
        o.build_docs(docs, L, 0, K)
        rm = gen.ReadModel(qseed=K, src_lo=0, src_hi=K, len_kind=1, lo=31, hi=150, err_lo=0.0, err_hi=0.02)
        seqs, offs = _reads_with_edges(dm, rm, 400)
        n = offs.size - 1
        out = np.zeros((n, o.W), dtype=np.uint64)
        bits = o.bits()
        for r in range(R):
            rep = o.new_rep()
            for c0 in range(0, K, 17):                    # documents in chunks
                c1 = min(K, c0 + 17)
                o.build_rep(r, rep, docs[c0 * L:c1 * L], L, c0, c1 - c0)
            assert np.array_equal(rep, bits[r]), r
            o.alg2_rep(r, rep, seqs, offs, out, first=(r == 0))
        want_def, _ = o.query_seqs(seqs, offs, oracle.MODE_DEF)
        want_alg2, _ = o.query_seqs(seqs, offs, oracle.MODE_ALG2, early_exit=True)
        assert np.array_equal(out, want_def)
        assert np.array_equal(out, want_alg2)
        everyone = _ref.ids_to_bits(range(K), K)
        assert np.array_equal(out[n - 4], everyone) and np.array_equal(out[n - 5], everyone)
        if m >= 1 << 20:
            table = _ref.KmerTable({d: _ref.seq_terms(docs[d * L:(d + 1) * L].tobytes()) for d in range(K)})
            phis = o.phis()
            cell = {(r, b): set().union(*[table.sets[d] for d in range(K) if phis[r, d] == b])
                    for r in range(R) for b in range(B)}
            for i in range(n):
                Q = set(_ref.seq_terms(seqs[int(offs[i]):int(offs[i + 1])].tobytes()).tolist())
                ex = {e for e in range(K) if all(Q <= cell[(r, phis[r, e])] for r in range(R))}
                assert _ref.bits_to_ids(out[i], K) == ex, i
    with pytest.raises(ValueError):
        o.build_rep(R, o.new_rep(), docs, L, 0, 1)


# ------------------------------------------------ routing and stacking
def test_two_level_partition_equals_stacked_shards():
    """Section 5.3: documents are routed to G shards by a random hash tau,
    each shard is an independent RAMBO of b cells over its documents with the
    same seeds (so the same Bloom hash functions and the same node-local
    partition phi_r of the global document id), and the shards stacked are
    the RAMBO built directly with the two-level partition
    b * tau(d) + phi_r(d) over B = G * b cells. Checked on the oracle: every
    BFU of the two-level index is the BFU of its shard, and each document's
    answer in the two-level index is its answer in its shard, for every read
    (so the K_g-document answers of the shards, put back in global id order,
    are the whole answer). An index given phi_r itself as its table equals
    the plain oracle."""
    K, G, b, R, m, eta, L, seed, rseed = 300, 4, 6, 3, 1 << 16, 2, 400, 77, 5151
    dm = gen.DocModel(seed=161, n_docs=K, length=L, docs_per_anc=10, mu_lo=0.02, mu_hi=0.02)
    docs = dm.docs(0, K)
    tau = oracle.route(rseed, G, range(K))
    assert set(tau.tolist()) == set(range(G))
    local = oracle.Oracle(K, b, R, m, eta, seed, alloc_bits=False)   # phi_r over b cells, global ids
    phi = local.phis()
    two = oracle.Oracle(K, G * b, R, m, eta, seed, cells=b * tau[None, :] + phi)
    two.build_docs(docs, L, 0, K)
    rm = gen.ReadModel(qseed=162, src_lo=0, src_hi=K, len_kind=1, lo=31, hi=150, err_lo=0.0, err_hi=0.01)
    reads = gen.reads(dm, rm, 400)
    want, _ = two.query_seqs(reads.seqs, reads.offsets, oracle.MODE_DEF)
    assert want.any(axis=1).sum() > 50
    tbits = two.bits()
    got = np.zeros_like(want)
    for g in range(G):
        gid = np.nonzero(tau == g)[0]
        sh = oracle.Oracle(gid.size, b, R, m, eta, seed, cells=phi[:, gid])
        for l, d in enumerate(gid):
            sh.insert_seq(l, docs[d * L:(d + 1) * L])
        sbits = sh.bits()
        for r in range(R):
            for c in range(b):
                assert np.array_equal(sbits[r, c], tbits[r, b * g + c]), (g, r, c)
        ans, _ = sh.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2)
        abits = np.unpackbits(ans.view(np.uint8), axis=1, bitorder="little")[:, :gid.size]
        for l, d in enumerate(gid):       # local document l is global document d
            got[:, d >> 6] |= abits[:, l].astype(np.uint64) << np.uint64(d & 63)
    assert np.array_equal(got, want)
    plain = oracle.Oracle(K, b, R, m, eta, seed)
    table = oracle.Oracle(K, b, R, m, eta, seed, cells=phi)
    plain.build_docs(docs, L, 0, K)
    table.build_docs(docs, L, 0, K)
    assert np.array_equal(plain.bits(), table.bits())
    assert np.array_equal(table.cells(), phi)


def test_two_level_partition_is_two_universal():
    """Section 5.3's claim: the two-level hash b * tau(d) + phi(d) keeps the
    collision probability of any two documents at 1/B for B = G * b cells.
    Over random seeds (routing and index), a fixed pair of document ids
    collides at that rate; the routing itself spreads documents evenly."""
    G, b, trials = 4, 8, 6000
    hits = 0
    for s in range(trials):
        t = oracle.route(90_000 + s, G, [17, 901])
        o = oracle.Oracle(1000, b, 1, 64, 1, 70_000 + s, alloc_bits=False)
        hits += b * t[0] + o.phi(0, 17) == b * t[1] + o.phi(0, 901)
    B = G * b
    assert abs(hits / trials - 1 / B) < 4 * math.sqrt((1 / B) * (1 - 1 / B) / trials), hits / trials
    cnt = np.bincount(oracle.route(5, G, range(0, 40_000, 3)), minlength=G)
    exp = cnt.sum() / G
    assert ((cnt - exp) ** 2 / exp).sum() < G - 1 + 6 * math.sqrt(2 * (G - 1))
