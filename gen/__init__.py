"""Seeded synthetic inputs (genomes, reads, k-mer queries) shared by tests,
benchmark and oracle.

Input plumbing only: no canonical form, hashing or filter arithmetic lives
here. The C core (``gen.c``) is built into ``libgen.so`` beside this file.

Workloads follow the paper's genomic setting (k = 31 over ACGT; documents are
genomes, queries are k-mers or reads; Sections 5.1-5.2), scaled to one GPU.
The ENA archive the paper indexes is not available; these seeded generators
stand in for it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgen.so")
_lib = None

K_MER = 31


def build(force: bool = True) -> str:
    """Compile libgen.so with gcc (OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        u64, i64, dbl, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        vp = ctypes.c_void_p
        L.gen_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
        L.gen_splitmix64_next.restype = u64
        L.gen_doc.argtypes = [u64, u64, u64, dbl, dbl, u64, u64, u64, vp]
        L.gen_docs.argtypes = [u64, u64, u64, dbl, dbl, u64, u64, vp, i32]
        L.gen_doc_window_codes.argtypes = [u64, u64, u64, dbl, dbl, u64, ctypes.c_uint32, vp]
        L.gen_kmer_queries.argtypes = [u64, u64, u64, dbl, dbl, u64, u64, dbl, ctypes.c_uint32, u64,
                                       vp, vp, i32]
        L.gen_read_offsets.argtypes = [u64, u64, u64, u64, u64, dbl, i32, dbl, dbl, u64, u64, dbl,
                                       dbl, u64, u64, vp]
        L.gen_read_fill.argtypes = [u64, u64, u64, dbl, dbl, u64, u64, u64, dbl, i32, dbl, dbl, u64,
                                    u64, dbl, dbl, u64, u64, vp, vp, vp, vp, vp, vp, i32]
        L.gen_poisson_arrivals.argtypes = [u64, dbl, u64, vp]
        L.gen_term_id.argtypes = [u64, u64]
        L.gen_term_id.restype = u64
        L.gen_term_doc_len.argtypes = [u64, u64, u64]
        L.gen_term_doc_len.restype = u64
        L.gen_zipf_cdf.argtypes = [u64, dbl, vp]
        L.gen_term_docs.argtypes = [u64, u64, vp, u64, u64, vp, vp, i32]
        L.gen_term_queries.argtypes = [u64, u64, vp, u64, u64, u64, dbl, u64, vp, vp, i32]
        L.gen_term_phrase_lens.argtypes = [u64, u64, u64, u64, vp]
        L.gen_term_phrases.argtypes = [u64, u64, vp, u64, u64, u64, dbl, u64, vp, vp, vp, i32]
        for f in ("gen_doc", "gen_docs", "gen_doc_window_codes", "gen_kmer_queries",
                  "gen_read_offsets", "gen_read_fill", "gen_poisson_arrivals", "gen_zipf_cdf",
                  "gen_term_docs", "gen_term_queries", "gen_term_phrase_lens", "gen_term_phrases"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def nthreads() -> int:
    n = os.environ.get("OMP_NUM_THREADS")
    if n and n.isdigit():
        return max(1, int(n))
    return max(1, min(16, os.cpu_count() or 1))


def splitmix64(seed: int, n: int) -> list[int]:
    s = ctypes.c_uint64(seed)
    return [lib().gen_splitmix64_next(ctypes.byref(s)) for _ in range(n)]


@dataclass(frozen=True)
class DocModel:
    """Documents: ``n_docs`` genomes of ``length`` bases. Document d copies
    ancestor d // docs_per_anc and substitutes each base independently with
    probability mu_d, mu_d uniform in [mu_lo, mu_hi]. docs_per_anc = 1 with
    mu = 0 gives i.i.d. uniform documents."""
    seed: int
    n_docs: int
    length: int
    docs_per_anc: int = 1
    mu_lo: float = 0.0
    mu_hi: float = 0.0

    def _a(self):
        return (self.seed, self.length, self.docs_per_anc, self.mu_lo, self.mu_hi)

    def doc(self, d: int, start: int = 0, n: int | None = None) -> bytes:
        n = self.length - start if n is None else n
        buf = ctypes.create_string_buffer(n)
        lib().gen_doc(*self._a(), d, start, n, buf)
        return buf.raw

    def docs(self, d0: int, nd: int, out: np.ndarray | None = None) -> np.ndarray:
        """nd whole documents, concatenated, as a uint8 array."""
        if out is None:
            out = np.empty(nd * self.length, dtype=np.uint8)
        assert out.dtype == np.uint8 and out.size >= nd * self.length and out.flags.c_contiguous
        lib().gen_docs(*self._a(), d0, nd, _ptr(out), nthreads())
        return out

    def window_codes(self, d: int, k: int = K_MER) -> np.ndarray:
        """Forward 2-bit codes (first base most significant; A0 C1 G2 T3) of
        every length-k window of document d; not canonical."""
        out = np.empty(max(0, self.length - k + 1), dtype=np.uint64)
        if out.size:
            lib().gen_doc_window_codes(*self._a(), d, k, _ptr(out))
        return out


@dataclass(frozen=True)
class ReadModel:
    """Reads: a fraction ``frac_doc`` copied from a uniform document in
    [src_lo, src_hi) at a uniform start, with per-base substitution errors at
    a per-read rate uniform in [err_lo, err_hi] and reverse-complemented with
    probability 1/2; the rest i.i.d. uniform ACGT. Length: log-normal
    round(median * exp(sigma * Z)) clipped to [lo, hi] (len_kind 0) or uniform
    in [lo, hi] (len_kind 1)."""
    qseed: int
    src_lo: int
    src_hi: int
    frac_doc: float = 0.7
    len_kind: int = 0
    median: float = 300.0
    sigma: float = 1.0
    lo: int = 31
    hi: int = 10000
    err_lo: float = 0.0
    err_hi: float = 0.01


@dataclass
class Reads:
    seqs: np.ndarray      # uint8, concatenated
    offsets: np.ndarray   # uint64, n+1
    src: np.ndarray       # int64, source document or -1
    start: np.ndarray     # int64
    nerr: np.ndarray      # int64
    rc: np.ndarray        # int8

    @property
    def n(self) -> int:
        return self.offsets.size - 1

    def read(self, i: int) -> bytes:
        return self.seqs[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def n_windows(self, k: int = K_MER) -> int:
        L = np.diff(self.offsets.astype(np.int64))
        return int(np.maximum(L - (k - 1), 0).sum())


def reads(dm: DocModel, rm: ReadModel, n: int, i0: int = 0) -> Reads:
    L = lib()
    offs = np.empty(n + 1, dtype=np.uint64)
    ra = (rm.qseed, rm.src_lo, rm.src_hi, rm.frac_doc, rm.len_kind, rm.median, rm.sigma, rm.lo,
          rm.hi, rm.err_lo, rm.err_hi)
    L.gen_read_offsets(dm.seed, dm.length, *ra, i0, n, _ptr(offs))
    seqs = np.empty(int(offs[-1]), dtype=np.uint8)
    src = np.empty(n, dtype=np.int64)
    start = np.empty(n, dtype=np.int64)
    nerr = np.empty(n, dtype=np.int64)
    rc = np.empty(n, dtype=np.int8)
    L.gen_read_fill(*dm._a(), *ra, i0, n, _ptr(offs), _ptr(seqs), _ptr(src), _ptr(start),
                    _ptr(nerr), _ptr(rc), nthreads())
    return Reads(seqs, offs, src, start, nerr, rc)


def kmer_queries(dm: DocModel, qseed: int, n: int, frac_present: float = 0.5, k: int = K_MER):
    """n single k-mer queries as forward 2-bit codes: a fraction drawn as a
    window of a uniform document (source id returned), the rest uniform
    random 2k-bit codes (source -1)."""
    out = np.empty(n, dtype=np.uint64)
    src = np.empty(n, dtype=np.int64)
    lib().gen_kmer_queries(*dm._a(), dm.n_docs, qseed, frac_present, k, n, _ptr(out), _ptr(src),
                           nthreads())
    return out, src


def poisson_arrivals(aseed: int, lam: float, n: int) -> np.ndarray:
    t = np.empty(n, dtype=np.float64)
    lib().gen_poisson_arrivals(aseed, lam, n, _ptr(t))
    return t


# ---------------------------------------------------------------------------
# Word-term documents (the web-document setting): a document is a set of
# opaque 64-bit term ids (hashes of word unigrams), drawn from a Zipf
# vocabulary; see gen.c.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class TermDocModel:
    seed: int
    n_docs: int
    mean_terms: int      # terms per document uniform in [mean/2, 3 mean/2]
    vocab: int = 200_000
    zipf_s: float = 1.0

    def cdf(self) -> np.ndarray:
        key = (self.vocab, self.zipf_s)
        c = _CDF.get(key)
        if c is None:
            c = np.empty(self.vocab, dtype=np.float64)
            lib().gen_zipf_cdf(self.vocab, self.zipf_s, _ptr(c))
            _CDF[key] = c
        return c

    def doc_len(self, d: int) -> int:
        return int(lib().gen_term_doc_len(self.seed, self.mean_terms, d))

    def docs(self, d0: int = 0, nd: int | None = None):
        """(terms uint64, offsets uint64[nd+1]) of documents d0 .. d0+nd-1."""
        nd = self.n_docs - d0 if nd is None else nd
        lens = np.array([self.doc_len(d0 + k) for k in range(nd)], dtype=np.uint64)
        offs = np.zeros(nd + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        out = np.empty(int(offs[-1]), dtype=np.uint64)
        lib().gen_term_docs(self.seed, self.vocab, _ptr(self.cdf()), d0, nd, _ptr(offs), _ptr(out), nthreads())
        return out, offs

    def doc(self, d: int) -> np.ndarray:
        return self.docs(d, 1)[0]

    def term_queries(self, qseed: int, n: int, frac_present: float = 0.5):
        out = np.empty(n, dtype=np.uint64)
        src = np.empty(n, dtype=np.int64)
        lib().gen_term_queries(self.seed, self.vocab, _ptr(self.cdf()), self.mean_terms, self.n_docs, qseed,
                               frac_present, n, _ptr(out), _ptr(src), nthreads())
        return out, src

    def phrases(self, qseed: int, n: int, lo: int = 2, hi: int = 8, frac_doc: float = 0.5):
        """n term-set queries: (terms, offsets[n+1], source doc or -1)."""
        lens = np.empty(n, dtype=np.uint64)
        lib().gen_term_phrase_lens(qseed, lo, hi, n, _ptr(lens))
        offs = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        out = np.empty(int(offs[-1]), dtype=np.uint64)
        src = np.empty(n, dtype=np.int64)
        lib().gen_term_phrases(self.seed, self.vocab, _ptr(self.cdf()), self.mean_terms, self.n_docs, qseed,
                               frac_doc, n, _ptr(offs), _ptr(out), _ptr(src), nthreads())
        return out, offs, src


_CDF: dict = {}


@dataclass(frozen=True)
class TermWorkload:
    name: str
    K: int
    B: int
    R: int
    m: int
    eta: int
    docs: TermDocModel
    index_seed: int
    n_queries: int
    qseed: int


def term_workload(name: str) -> TermWorkload:
    """The paper's two web-document index shapes (Section 5.4, document
    indexing) on synthetic term sets: Wiki-dump-like (17,618 documents of
    ~650 terms, B=1,000, R=2, 200,000-bit BFUs) and ClueWeb09-like (50,000
    documents of ~450 terms, B=5,000, R=3, 20,000-bit BFUs); eta = 2."""
    if name == "wiki":
        dm = TermDocModel(seed=1101, n_docs=17_618, mean_terms=650, vocab=200_000)
        return TermWorkload("wiki-K17618-B1000-R2-m200000", 17_618, 1000, 2, 200_000, 2, dm, 2101, 1_000_000, 3101)
    if name == "clueweb":
        dm = TermDocModel(seed=1102, n_docs=50_000, mean_terms=450, vocab=500_000)
        return TermWorkload("clueweb-K50000-B5000-R3-m20000", 50_000, 5000, 3, 20_000, 2, dm, 2102, 1_000_000,
                            3102)
    raise ValueError(name)


# ---------------------------------------------------------------------------
# The five workloads (index parameters + inputs). Seeds: data 1000+c,
# index 2000+c, queries 3000+c, arrivals 4000+rate index.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    K: int            # document capacity of the index
    B: int
    R: int
    m: int
    eta: int
    docs: DocModel    # documents built into the index
    index_seed: int
    reads: ReadModel | None = None
    n_reads: int = 0
    n_kmer_queries: int = 0
    kmer_qseed: int = 0
    stream_docs: tuple = field(default=())   # (first id, count) inserted after the build

    @property
    def n_built(self) -> int:
        return self.docs.n_docs


def workload(c: int) -> Workload:
    """Workload c (1..5) as described by its index and input parameters."""
    if c == 1:
        dm = DocModel(seed=1001, n_docs=100, length=20000)
        return Workload("tiny-K100-B10-R3", 100, 10, 3, 1 << 20, 2, dm, 2001,
                        n_kmer_queries=10_000, kmer_qseed=3001)
    if c == 2:
        dm = DocModel(seed=1002, n_docs=1000, length=200_000, docs_per_anc=50, mu_lo=0.01, mu_hi=0.01)
        return Workload("K1000-B32-R4-m2^26", 1000, 32, 4, 1 << 26, 3, dm, 2002,
                        n_kmer_queries=10_000_000, kmer_qseed=3002)
    if c in (3, 4):
        dm = DocModel(seed=1003, n_docs=10_000, length=500_000, docs_per_anc=100, mu_lo=0.005,
                      mu_hi=0.02)
        rm = ReadModel(qseed=3003, src_lo=0, src_hi=10_000, frac_doc=0.7, len_kind=0, median=300.0,
                       sigma=1.0, lo=31, hi=10_000, err_lo=0.0, err_hi=0.01)
        return Workload("K10000-B100-R5-m2^29" + ("-served" if c == 4 else ""), 10_000, 100, 5,
                        1 << 29, 2, dm, 2003, reads=rm, n_reads=100_000)
    if c == 5:
        dm = DocModel(seed=1005, n_docs=100_000, length=100_000, docs_per_anc=100, mu_lo=0.01,
                      mu_hi=0.01)
        rm = ReadModel(qseed=3005, src_lo=0, src_hi=101_000, frac_doc=0.7, len_kind=1, lo=100,
                       hi=1000, err_lo=0.01, err_hi=0.01)
        return Workload("K101000-B1000-R6-m2^27", 101_000, 1000, 6, 1 << 27, 2, dm, 2005, reads=rm,
                        n_reads=1_000_000, stream_docs=(100_000, 1000))
    raise ValueError(c)
