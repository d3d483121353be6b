"""The seeded input generators: determinism and the workload structure the
documentation promises (related genomes, reads copied from documents)."""
import os

import numpy as np

import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    want = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert gen.splitmix64(1234567, len(want)) == want


def test_docs_deterministic_and_random_access():
    dm = gen.DocModel(seed=7, n_docs=6, length=5000, docs_per_anc=3, mu_lo=0.01, mu_hi=0.02)
    a = dm.docs(0, 6)
    b = dm.docs(0, 6)
    assert np.array_equal(a, b)
    assert set(np.unique(a).tolist()) <= set(b"ACGT")
    # any slice of any document regenerates alone
    assert dm.doc(4, 1234, 100) == a[4 * 5000 + 1234: 4 * 5000 + 1334].tobytes()
    assert dm.docs(2, 3).tobytes() == a[2 * 5000: 5 * 5000].tobytes()


def test_mutants_share_ancestor():
    dm = gen.DocModel(seed=9, n_docs=4, length=200_000, docs_per_anc=2, mu_lo=0.01, mu_hi=0.01)
    d = dm.docs(0, 4).reshape(4, -1)
    same = (d[0] == d[1]).mean()      # siblings: each differs from the ancestor at ~1%
    other = (d[0] == d[2]).mean()     # unrelated: ~1/4 agreement
    assert 0.975 < same < 0.985
    assert 0.24 < other < 0.26


def test_iid_docs_uniform():
    dm = gen.DocModel(seed=1, n_docs=2, length=100_000)
    d = dm.docs(0, 2)
    counts = np.bincount(d, minlength=256)[[65, 67, 71, 84]] / d.size
    assert np.all(np.abs(counts - 0.25) < 0.01)


def test_window_codes_match_bases():
    dm = gen.DocModel(seed=3, n_docs=2, length=400, docs_per_anc=2, mu_lo=0.02, mu_hi=0.02)
    codes = dm.window_codes(1)
    s = dm.doc(1)
    assert codes.size == 400 - 30
    for p in (0, 17, 369):
        w = s[p:p + 31].decode().translate(str.maketrans("ACGT", "0123"))
        assert int(codes[p]) == int(w, 4)


def _rc(s: bytes) -> bytes:
    return s[::-1].translate(bytes.maketrans(b"ACGT", b"TGCA"))


def test_reads_structure():
    dm = gen.DocModel(seed=11, n_docs=20, length=30_000, docs_per_anc=10, mu_lo=0.01, mu_hi=0.01)
    rm = gen.ReadModel(qseed=5, src_lo=0, src_hi=20, frac_doc=0.7, len_kind=0, median=300, sigma=1.0,
                       lo=31, hi=10_000, err_lo=0.0, err_hi=0.01)
    r = gen.reads(dm, rm, 2000)
    r2 = gen.reads(dm, rm, 2000)
    assert np.array_equal(r.seqs, r2.seqs) and np.array_equal(r.offsets, r2.offsets)
    L = np.diff(r.offsets.astype(np.int64))
    assert L.min() >= 31 and L.max() <= 10_000
    assert 250 < np.median(L) < 350
    frac = (r.src >= 0).mean()
    assert 0.66 < frac < 0.74
    assert 0.45 < r.rc[r.src >= 0].mean() < 0.55
    # a read regenerates alone (random access by index)
    one = gen.reads(dm, rm, 1, i0=123)
    assert one.read(0) == r.read(123)
    # doc-derived reads: after undoing the strand, differ from the source window
    # in exactly nerr positions
    for i in np.nonzero(r.src >= 0)[0][:200]:
        s = r.read(i)
        if r.rc[i]:
            s = _rc(s)
        w = dm.doc(int(r.src[i]), int(r.start[i]), len(s))
        diff = sum(a != b for a, b in zip(s, w))
        assert diff == r.nerr[i]


def test_uniform_lengths():
    dm = gen.DocModel(seed=12, n_docs=5, length=5000)
    rm = gen.ReadModel(qseed=6, src_lo=0, src_hi=5, len_kind=1, lo=100, hi=1000, err_lo=0.01, err_hi=0.01)
    r = gen.reads(dm, rm, 3000)
    L = np.diff(r.offsets.astype(np.int64))
    assert L.min() >= 100 and L.max() <= 1000 and abs(L.mean() - 550) < 20


def test_kmer_queries():
    dm = gen.DocModel(seed=13, n_docs=10, length=1000)
    q, src = gen.kmer_queries(dm, 99, 1000, 0.5)
    assert np.all(q < (1 << 62))
    assert 0.4 < (src >= 0).mean() < 0.6
    for i in np.nonzero(src >= 0)[0][:20]:
        codes = dm.window_codes(int(src[i]))
        assert int(q[i]) in set(codes.tolist())


def test_poisson_arrivals():
    t = gen.poisson_arrivals(4000, 1000.0, 20000)
    gaps = np.diff(t)
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1e-3) < 5e-5


def test_term_documents_regenerate_and_have_their_shape():
    dm = gen.TermDocModel(seed=3, n_docs=500, mean_terms=100, vocab=10_000)
    terms, offs = dm.docs()
    lens = np.diff(offs.astype(np.int64))
    assert lens.min() >= 50 and lens.max() <= 150
    for d in (0, 17, 499):
        assert np.array_equal(dm.doc(d), terms[offs[d]:offs[d + 1]])
    t2, o2 = dm.docs(200, 50)
    assert np.array_equal(t2, terms[offs[200]:offs[250]])
    # Zipf: the most frequent word is about 1/H_V of all draws
    vals, counts = np.unique(terms, return_counts=True)
    top = counts.max() / terms.size
    hv = sum(1.0 / (k + 1) for k in range(10_000))
    assert abs(top - 1 / hv) < 0.2 / hv
    cdf = dm.cdf()
    assert np.all(np.diff(cdf) > 0) and cdf[-1] == 1.0


def test_term_queries_and_phrases_come_from_their_sources():
    dm = gen.TermDocModel(seed=4, n_docs=200, mean_terms=60, vocab=5000)
    terms, offs = dm.docs()
    q, src = dm.term_queries(9, 1000, 0.5)
    assert 400 < (src >= 0).sum() < 600
    for i in np.nonzero(src >= 0)[0][:200]:
        d = int(src[i])
        assert q[i] in set(terms[offs[d]:offs[d + 1]].tolist())
    pt, po, ps = dm.phrases(10, 300, 2, 6, 0.5)
    lens = np.diff(po.astype(np.int64))
    assert lens.min() >= 2 and lens.max() <= 6
    for i in np.nonzero(ps >= 0)[0][:100]:
        d = int(ps[i])
        doc = terms[offs[d]:offs[d + 1]]
        ph = pt[po[i]:po[i + 1]]
        # consecutive terms of the document (cyclically)
        starts = [s for s in range(doc.size) if doc[s] == ph[0]]
        assert any(all(doc[(s + k) % doc.size] == ph[k] for k in range(ph.size)) for s in starts)
