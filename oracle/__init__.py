"""RAMBO CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``oracle.c`` (plain C, BFU-major, written from the paper's
definitions: Section 2.1 Bloom filters, Section 3 / Algorithm 1 construction,
Section 3.3 / Algorithm 2 query, Section 3.3.1 sequence query, Section 5.3
folding). Only ``tests/``, the package ``smoke()`` check and the benchmark's
CPU-baseline leg may import it; the GPU library never does.

``twin.py`` beside it is an independent pure-Python restatement for tiny
inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

KMER = 31
MODE_DEF, MODE_ALG2 = 0, 1


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
        sig = {
            "orc_new": ([u64, u32, u32, u64, u32, u64, i32], vp),
            "orc_new_cells": ([u64, u32, u32, u64, u32, u64, vp, i32], vp),
            "orc_route": ([u64, u32, u64], u32),
            "orc_cells": ([vp, vp], None),
            "orc_free": ([vp], None),
            "orc_bits": ([vp], vp),
            "orc_wpb": ([vp], u64),
            "orc_result_words": ([vp], u64),
            "orc_params": ([vp, vp, vp, vp, vp, vp, vp], None),
            "orc_phi": ([vp, u32, u64], u32),
            "orc_h": ([vp, u32, u32, u64], u64),
            "orc_revcomp": ([u64], u64),
            "orc_canon": ([u64], u64),
            "orc_window": ([vp, u64, vp], i32),
            "orc_insert_kmers": ([vp, u64, vp, u64], i32),
            "orc_insert_seq": ([vp, u64, vp, u64], i32),
            "orc_build_docs": ([vp, vp, u64, u64, u64, i32], i32),
            "orc_bfu_insert_seq": ([vp, u32, vp, vp, u64], None),
            "orc_bfu_test_seq": ([vp, u32, vp, vp, u64], i32),
            "orc_popcount_bfu": ([vp, u32, u32], u64),
            "orc_bfu_test_seqs": ([vp, u32, vp, vp, vp, u64, vp, i32], None),
            "orc_build_rep": ([vp, u32, vp, vp, u64, u64, u64, i32], i32),
            "orc_alg2_rep": ([vp, u32, vp, vp, vp, u64, vp, i32, i32], None),
            "orc_query_kmer_def": ([vp, u64, vp], None),
            "orc_query_kmer_alg2": ([vp, u64, vp], None),
            "orc_query_seq_def": ([vp, vp, u64, vp], None),
            "orc_query_seq_alg2": ([vp, vp, u64, vp, i32], u64),
            "orc_query_kmers": ([vp, vp, u64, vp, i32, i32], None),
            "orc_query_seqs": ([vp, vp, vp, u64, vp, i32, i32, i32], u64),
            "orc_fold": ([vp], vp),
            "orc_insert_terms": ([vp, u64, vp, u64], i32),
            "orc_build_term_docs": ([vp, vp, vp, u64, u64, i32], i32),
            "orc_query_termset_def": ([vp, vp, u64, vp], None),
            "orc_query_termset_alg2": ([vp, vp, u64, vp, i32], u64),
            "orc_query_terms": ([vp, vp, u64, vp, i32, i32], None),
            "orc_query_termsets": ([vp, vp, vp, u64, vp, i32, i32, i32], u64),
        }
        for name, (a, r) in sig.items():
            f = getattr(L, name)
            f.argtypes, f.restype = a, r
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _nthreads():
    n = os.environ.get("OMP_NUM_THREADS")
    if n and n.isdigit():
        return max(1, int(n))
    return max(1, min(16, os.cpu_count() or 1))


def canon(x: int) -> int:
    return int(lib().orc_canon(x))


def revcomp(x: int) -> int:
    return int(lib().orc_revcomp(x))


def window(seq: bytes, p: int = 0):
    """Canonical code of the 31-window at p, or None if it holds a non-ACGT byte."""
    out = ctypes.c_uint64(0)
    ok = lib().orc_window(seq, p, ctypes.byref(out))
    return int(out.value) if ok else None


def route(route_seed: int, G: int, ids) -> np.ndarray:
    """tau(d) for each document id: the shard of Section 5.3's routing."""
    return np.array([lib().orc_route(route_seed, G, int(d)) for d in ids], dtype=np.int64)


class Oracle:
    """A RAMBO index on the CPU: R x B Bloom filters of m bits (BFU-major).
    With `cells` (an (R, K) table of cells < B), the partition is that table
    instead of phi_r (the two-level partition of Section 5.3)."""

    def __init__(self, K, B, R, m, eta, seed, alloc_bits=True, _handle=None, cells=None):
        self.K, self.B, self.R, self.m, self.eta, self.seed = K, B, R, m, eta, seed
        L = lib()
        if _handle is None and cells is not None:
            c = np.ascontiguousarray(cells, dtype=np.uint32)
            assert c.shape == (R, K)
            _handle = L.orc_new_cells(K, B, R, m, eta, seed, _p(c), int(alloc_bits))
            if not _handle:
                raise ValueError("cell table out of range")
        self._h = _handle if _handle is not None else L.orc_new(K, B, R, m, eta, seed, int(alloc_bits))
        if not self._h:
            raise MemoryError("oracle allocation failed")
        self.wpb = int(L.orc_wpb(self._h))
        self.W = int(L.orc_result_words(self._h))
        self.has_bits = bool(L.orc_bits(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # -- hash functions and parameters
    def phi(self, r: int, d: int) -> int:
        return int(lib().orc_phi(self._h, r, d))

    def phis(self) -> np.ndarray:
        """phi_r(d) for every r and d: the partition hash (see cells())."""
        return np.array([[self.phi(r, d) for d in range(self.K)] for r in range(self.R)], dtype=np.int64)

    def cells(self) -> np.ndarray:
        """The cell of every document in every repetition, shape (R, K): phi_r,
        or the explicit table the index was created with."""
        out = np.zeros((self.R, self.K), dtype=np.uint32)
        lib().orc_cells(self._h, _p(out))
        return out.astype(np.int64)

    def h(self, r: int, j: int, x: int) -> int:
        return int(lib().orc_h(self._h, r, j, x))

    def params(self):
        R, E = self.R, self.R * self.eta
        arrs = [np.zeros(R, np.uint64), np.zeros(R, np.uint64)] + [np.zeros(E, np.uint64) for _ in range(4)]
        lib().orc_params(self._h, *[_p(a) for a in arrs])
        return dict(zip(("pa", "pb", "Alo", "Ahi", "Clo", "Chi"), arrs))

    # -- construction
    def insert_kmers(self, d: int, kmers: np.ndarray) -> None:
        k = np.ascontiguousarray(kmers, dtype=np.uint64)
        if lib().orc_insert_kmers(self._h, d, _p(k), k.size) != 0:
            raise ValueError("invalid document id or k-mer value")

    def insert_seq(self, d: int, seq) -> None:
        s = np.frombuffer(bytes(seq), dtype=np.uint8) if not isinstance(seq, np.ndarray) else seq
        s = np.ascontiguousarray(s, dtype=np.uint8)
        if lib().orc_insert_seq(self._h, d, _p(s), s.size) != 0:
            raise ValueError("invalid document id")

    def build_docs(self, docs: np.ndarray, doc_len: int, d0: int, nd: int, nthreads=None) -> None:
        docs = np.ascontiguousarray(docs, dtype=np.uint8)
        assert docs.size >= nd * doc_len
        if lib().orc_build_docs(self._h, _p(docs), doc_len, d0, nd, nthreads or _nthreads()) != 0:
            raise ValueError("document range exceeds K")

    # -- opaque terms (word ids; no k-mer encoding)
    def insert_terms(self, d: int, terms: np.ndarray) -> None:
        t = np.ascontiguousarray(terms, dtype=np.uint64)
        if lib().orc_insert_terms(self._h, d, _p(t), t.size) != 0:
            raise ValueError("invalid document id")

    def build_term_docs(self, terms: np.ndarray, offsets: np.ndarray, d0: int = 0, nthreads=None) -> None:
        t = np.ascontiguousarray(terms, dtype=np.uint64)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        if lib().orc_build_term_docs(self._h, _p(t), _p(o), d0, o.size - 1, nthreads or _nthreads()) != 0:
            raise ValueError("document range exceeds K")

    def query_terms(self, xs: np.ndarray, mode=MODE_DEF, nthreads=None) -> np.ndarray:
        xs = np.ascontiguousarray(xs, dtype=np.uint64)
        out = np.zeros((xs.size, self.W), dtype=np.uint64)
        lib().orc_query_terms(self._h, _p(xs), xs.size, _p(out), mode, nthreads or _nthreads())
        return out

    def query_termset(self, terms, mode=MODE_DEF, early_exit=True) -> np.ndarray:
        t = np.ascontiguousarray(terms, dtype=np.uint64)
        out = np.zeros(self.W, dtype=np.uint64)
        if mode == MODE_DEF:
            lib().orc_query_termset_def(self._h, _p(t), t.size, _p(out))
        else:
            lib().orc_query_termset_alg2(self._h, _p(t), t.size, _p(out), int(early_exit))
        return out

    def query_termsets(self, terms: np.ndarray, offsets: np.ndarray, mode=MODE_ALG2, early_exit=True,
                       nthreads=None):
        """(results [n][W], single-term Bloom tests performed)."""
        t = np.ascontiguousarray(terms, dtype=np.uint64)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = o.size - 1
        out = np.zeros((n, self.W), dtype=np.uint64)
        tests = lib().orc_query_termsets(self._h, _p(t), _p(o), n, _p(out), mode, int(early_exit),
                                         nthreads or _nthreads())
        return out, int(tests)

    # -- index contents
    def bits(self) -> np.ndarray:
        """Copy of the BFU-major bit array, shape (R, B, wpb) uint64."""
        ptr = lib().orc_bits(self._h)
        n = self.R * self.B * self.wpb
        buf = (ctypes.c_uint64 * n).from_address(ptr)
        return np.frombuffer(buf, dtype=np.uint64, count=n).reshape(self.R, self.B, self.wpb).copy()

    def bfu_popcount(self, r: int, b: int) -> int:
        return int(lib().orc_popcount_bfu(self._h, r, b))

    # -- single sampled BFUs of a large index
    def new_bfu(self) -> np.ndarray:
        return np.zeros(self.wpb, dtype=np.uint64)

    def bfu_insert_seq(self, r: int, f: np.ndarray, seq: np.ndarray) -> None:
        s = np.ascontiguousarray(seq, dtype=np.uint8)
        lib().orc_bfu_insert_seq(self._h, r, _p(f), _p(s), s.size)

    def bfu_test_seq(self, r: int, f: np.ndarray, seq) -> bool:
        s = np.frombuffer(bytes(seq), dtype=np.uint8) if not isinstance(seq, np.ndarray) else seq
        s = np.ascontiguousarray(s, dtype=np.uint8)
        return bool(lib().orc_bfu_test_seq(self._h, r, _p(f), _p(s), s.size))

    def bfu_test_seqs(self, r: int, f: np.ndarray, seqs: np.ndarray, offsets: np.ndarray, nthreads=None):
        """For every read: 1 iff each of its terms passes filter f of repetition r."""
        seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = offsets.size - 1
        out = np.zeros(n, dtype=np.uint8)
        lib().orc_bfu_test_seqs(self._h, r, _p(f), _p(seqs), _p(offsets), n, _p(out), nthreads or _nthreads())
        return out.astype(bool)

    # -- one repetition at a time (indexes too large for host memory)
    def new_rep(self) -> np.ndarray:
        """Zeroed filters of one repetition, shape (B, wpb) uint64."""
        return np.zeros((self.B, self.wpb), dtype=np.uint64)

    def build_rep(self, r: int, rep_bits: np.ndarray, docs: np.ndarray, doc_len: int, d0: int, nd: int,
                  nthreads=None) -> None:
        """Algorithm 1 for repetition r only: documents d0..d0+nd-1 into rep_bits."""
        assert rep_bits.shape == (self.B, self.wpb) and rep_bits.dtype == np.uint64 and rep_bits.flags.c_contiguous
        docs = np.ascontiguousarray(docs, dtype=np.uint8)
        assert docs.size >= nd * doc_len
        if lib().orc_build_rep(self._h, r, _p(rep_bits), _p(docs), doc_len, d0, nd, nthreads or _nthreads()) != 0:
            raise ValueError("repetition or document range out of range")

    def alg2_rep(self, r: int, rep_bits: np.ndarray, seqs: np.ndarray, offsets: np.ndarray, out: np.ndarray,
                 first: bool, nthreads=None) -> None:
        """Repetition r of Algorithm 2 for every read, intersected into out (n, W)."""
        assert rep_bits.shape == (self.B, self.wpb) and rep_bits.dtype == np.uint64
        seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = offsets.size - 1
        assert out.shape == (n, self.W) and out.dtype == np.uint64 and out.flags.c_contiguous
        lib().orc_alg2_rep(self._h, r, _p(rep_bits), _p(seqs), _p(offsets), n, _p(out), int(first),
                           nthreads or _nthreads())

    # -- queries
    def query_kmer(self, x: int, mode=MODE_DEF) -> np.ndarray:
        out = np.zeros(self.W, dtype=np.uint64)
        (lib().orc_query_kmer_def if mode == MODE_DEF else lib().orc_query_kmer_alg2)(self._h, x, _p(out))
        return out

    def query_kmers(self, xs: np.ndarray, mode=MODE_DEF, nthreads=None) -> np.ndarray:
        xs = np.ascontiguousarray(xs, dtype=np.uint64)
        out = np.zeros((xs.size, self.W), dtype=np.uint64)
        lib().orc_query_kmers(self._h, _p(xs), xs.size, _p(out), mode, nthreads or _nthreads())
        return out

    def query_seq(self, seq, mode=MODE_DEF, early_exit=True) -> np.ndarray:
        s = np.frombuffer(bytes(seq), dtype=np.uint8)
        s = np.ascontiguousarray(s)
        out = np.zeros(self.W, dtype=np.uint64)
        if mode == MODE_DEF:
            lib().orc_query_seq_def(self._h, _p(s), s.size, _p(out))
        else:
            lib().orc_query_seq_alg2(self._h, _p(s), s.size, _p(out), int(early_exit))
        return out

    def query_seqs(self, seqs: np.ndarray, offsets: np.ndarray, mode=MODE_ALG2, early_exit=True,
                   nthreads=None):
        """Returns (results (n, W) uint64, number of single-term Bloom tests)."""
        seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = offsets.size - 1
        out = np.zeros((n, self.W), dtype=np.uint64)
        t = lib().orc_query_seqs(self._h, _p(seqs), _p(offsets), n, _p(out), mode, int(early_exit),
                                 nthreads or _nthreads())
        return out, int(t)

    def fold(self) -> "Oracle":
        h = lib().orc_fold(self._h)
        if not h:
            raise ValueError("fold needs an even B and a built index")
        return Oracle(self.K, self.B // 2, self.R, self.m, self.eta, self.seed, _handle=h)


def bitset_to_ids(row: np.ndarray, K: int) -> list[int]:
    bits = np.unpackbits(row.view(np.uint8), bitorder="little")[:K]
    return np.nonzero(bits)[0].tolist()


def ids_to_bitset(ids, K: int) -> np.ndarray:
    W = (K + 63) // 64
    bits = np.zeros(W * 64, dtype=np.uint8)
    bits[list(ids)] = 1
    return np.packbits(bits, bitorder="little").view(np.uint64)
