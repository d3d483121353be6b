"""Test-side helpers: brute-force set membership with numpy, independent of
both the oracle's and the GPU library's arithmetic.

The reverse complement here works on whole words (complement all bits, then
reverse the order of the 2-bit groups with byte swaps and in-byte shuffles),
a different route from the oracle's base-by-base loop.
"""
from __future__ import annotations

import numpy as np

MASK62 = np.uint64((1 << 62) - 1)


def revcomp_np(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    y = (~x) & MASK62                      # complement every base (A<->T, C<->G)
    y = y.byteswap()                       # reverse byte order
    # reverse the four 2-bit groups inside each byte
    y = ((y >> np.uint64(4)) & np.uint64(0x0F0F0F0F0F0F0F0F)) | ((y & np.uint64(0x0F0F0F0F0F0F0F0F)) << np.uint64(4))
    y = ((y >> np.uint64(2)) & np.uint64(0x3333333333333333)) | ((y & np.uint64(0x3333333333333333)) << np.uint64(2))
    return y >> np.uint64(2)               # 32 groups reversed; drop the empty one


def canon_np(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    return np.minimum(x, revcomp_np(x))


def seq_terms(seq: bytes, k: int = 31) -> np.ndarray:
    """Canonical codes of the valid windows of an ASCII sequence (numpy)."""
    s = np.frombuffer(seq, dtype=np.uint8)
    lut = np.full(256, 255, dtype=np.uint8)
    for i, c in enumerate(b"ACGT"):
        lut[c] = i
        lut[c + 32] = i
    c = lut[s]
    n = s.size - k + 1
    if n <= 0:
        return np.zeros(0, dtype=np.uint64)
    bad = (c == 255).astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(bad)])
    valid = (cs[k:] - cs[:-k]) == 0
    cc = np.where(c == 255, 0, c).astype(np.uint64)
    fwd = np.zeros(n, dtype=np.uint64)
    for i in range(k):
        fwd = (fwd << np.uint64(2)) | cc[i:i + n]
    return canon_np(fwd[valid])


class KmerTable:
    """Exact k-mer sets of documents: sorted (canonical k-mer, document) pairs."""

    def __init__(self, doc_terms: dict[int, np.ndarray]):
        ks, ds = [], []
        for d, t in doc_terms.items():
            u = np.unique(t)
            ks.append(u)
            ds.append(np.full(u.size, d, dtype=np.int64))
        k = np.concatenate(ks) if ks else np.zeros(0, np.uint64)
        d = np.concatenate(ds) if ds else np.zeros(0, np.int64)
        o = np.lexsort((d, k))
        self.k, self.d = k[o], d[o]
        self.sets = {d: set(np.unique(t).tolist()) for d, t in doc_terms.items()}

    def docs_with(self, x: int) -> np.ndarray:
        lo = np.searchsorted(self.k, np.uint64(x), "left")
        hi = np.searchsorted(self.k, np.uint64(x), "right")
        return self.d[lo:hi]

    def multiplicity(self, xs: np.ndarray) -> np.ndarray:
        xs = np.asarray(xs, dtype=np.uint64)
        return np.searchsorted(self.k, xs, "right") - np.searchsorted(self.k, xs, "left")

    def truth_seq(self, terms: np.ndarray, K: int) -> set[int]:
        """Documents containing every term (all documents if there is none)."""
        if terms.size == 0:
            return set(range(K))
        out = None
        for x in np.unique(terms):
            s = set(self.docs_with(int(x)).tolist())
            out = s if out is None else out & s
            if not out:
                break
        return out


def bits_to_ids(row: np.ndarray, K: int) -> set[int]:
    b = np.unpackbits(np.ascontiguousarray(row, dtype=np.uint64).view(np.uint8), bitorder="little")[:K]
    return set(np.nonzero(b)[0].tolist())


def ids_to_bits(ids, K: int) -> np.ndarray:
    W = (K + 63) // 64
    b = np.zeros(W * 64, dtype=np.uint8)
    b[list(ids)] = 1
    return np.packbits(b, bitorder="little").view(np.uint64)


def revcomp_seq(s: bytes) -> bytes:
    return s[::-1].translate(bytes.maketrans(b"ACGTacgt", b"TGCAtgca"))
