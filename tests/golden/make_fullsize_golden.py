"""Write the expected answers of the full-size read workloads (K=10,000 and
K=101,000 documents) for seeded samples of their reads, with the CPU oracle
only -- test infrastructure, run by hand when the oracle or the generator
changes:

    python tests/golden/make_fullsize_golden.py [k10000|k101000 ...]

The oracle cannot hold these indexes whole (40 and 96 GiB as bits), so it
takes them one repetition at a time: Algorithm 1 restricted to repetition r
over every document, then repetition r of Algorithm 2 (the union of the
documents of the cells whose BFU holds every term of the read), intersected
into each sampled read's answer. With the same filters it also tests every
read of the workload against the cells of a set of sampled documents, which
gives those documents' answers on every read (a document is reported iff
its cell passes in every repetition).

Sampled documents: enough that, in every repetition, the cells of the
sampled documents fall in every 32-bit row word (K=10,000: 100 cells, four
words) or in every 16-byte segment of the row (K=101,000: 1,000 cells,
eight segments of 128 cells), plus sources of error-free reads, plus random
ones.

Output: tests/golden/<name>_answers.txt (text; see write()).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

# name: (workload, sampled reads, sampled documents, cells per covered unit, seed)
SPECS = {
    "k10000": (3, 10_000, 32, 32, 7001),
    "k101000": (5, 10_000, 16, 128, 7002),
}


def log(*a):
    print("[golden %7.1fs]" % (time.time() - T0), *a, flush=True)


T0 = time.time()


def reads_sha256(reads) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(reads.offsets, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(reads.seqs, dtype=np.uint8).tobytes())
    return h.hexdigest()


def pick_docs(phis, n_docs, want, unit, rng, reads, sample):
    """Documents whose cells cover every (repetition, unit of `unit` cells)
    pair, then sources of error-free sampled reads, then random ones, up to
    `want` (more if the cover needs more)."""
    R, K = phis.shape
    n_units = (int(phis.max()) + unit) // unit
    need = {(r, u) for r in range(R) for u in range(n_units)}
    chosen = []
    for d in rng.permutation(n_docs):
        d = int(d)
        new = {(r, int(phis[r, d]) // unit) for r in range(R)} & need
        if new:
            chosen.append(d)
            need -= new
        if not need:
            break
    assert not need, "cover incomplete"
    clean = [i for i in sample if reads.src[i] >= 0 and reads.nerr[i] == 0]
    for i in clean[:4]:
        if int(reads.src[i]) not in chosen:
            chosen.append(int(reads.src[i]))
    while len(chosen) < want:
        d = int(rng.integers(n_docs))
        if d not in chosen:
            chosen.append(d)
    return sorted(chosen)


def build(name: str) -> str:
    c, n_sample, n_docs_sample, unit, seed = SPECS[name]
    w = gen.workload(c)
    dm = w.docs
    n_docs = dm.n_docs + (w.stream_docs[1] if w.stream_docs else 0)  # built + streamed documents
    reads = gen.reads(dm, w.reads, w.n_reads)
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(reads.n, n_sample, replace=False))
    o = oracle.Oracle(w.K, w.B, w.R, w.m, w.eta, w.index_seed, alloc_bits=False)
    phis = o.phis()
    docs_s = pick_docs(phis, n_docs, n_docs_sample, unit, rng, reads, sample)
    log(name, "documents", n_docs, "reads", reads.n, "sample", n_sample, "sampled documents", len(docs_s))
    # the sampled reads, packed
    lens = (reads.offsets[sample + 1] - reads.offsets[sample]).astype(np.uint64)
    s_offs = np.zeros(n_sample + 1, dtype=np.uint64)
    np.cumsum(lens, out=s_offs[1:])
    s_seqs = np.concatenate([reads.seqs[int(reads.offsets[i]):int(reads.offsets[i + 1])] for i in sample])
    answers = np.zeros((n_sample, o.W), dtype=np.uint64)
    cols = {d: np.ones(reads.n, dtype=bool) for d in docs_s}
    chunk = max(1, (2_000_000_000 // dm.length))
    buf = np.empty(chunk * dm.length, dtype=np.uint8)
    for r in range(w.R):
        rep = o.new_rep()
        for c0 in range(0, n_docs, chunk):
            c1 = min(n_docs, c0 + chunk)
            dm.docs(c0, c1 - c0, out=buf[: (c1 - c0) * dm.length])
            o.build_rep(r, rep, buf, dm.length, c0, c1 - c0)
        log(name, "repetition", r, "built")
        o.alg2_rep(r, rep, s_seqs, s_offs, answers, first=(r == 0))
        for b in sorted({int(phis[r, d]) for d in docs_s}):
            ok = o.bfu_test_seqs(r, np.ascontiguousarray(rep[b]), reads.seqs, reads.offsets)
            for d in docs_s:
                if int(phis[r, d]) == b:
                    cols[d] &= ok
        log(name, "repetition", r, "queried")
        del rep
    return write(name, w, reads, sample, answers, docs_s, cols)


def write(name, w, reads, sample, answers, docs_s, cols) -> str:
    """Lines: '#' comments; 'key value' header lines; 'sample i0 i1 ...' (the
    sampled read indices, ascending); 'A <read index> <doc> <doc> ...' for
    every sampled read with a non-empty answer (ascending ids; a sampled read
    without an A line answers no document); 'D <doc> <read> <read> ...' for
    every sampled document (the reads, over the whole workload, that report
    it)."""
    path = os.path.join(HERE, "%s_answers.txt" % name)
    K = w.K
    with open(path, "w") as f:
        f.write("# Expected answers of workload %s for a seeded sample of its reads, computed by\n"
                "# tests/golden/make_fullsize_golden.py with the CPU oracle only (one repetition at a time).\n"
                % w.name)
        f.write("workload %s\nK %d\nreads %d\nreads_sha256 %s\n" % (w.name, K, reads.n, reads_sha256(reads)))
        f.write("sample %s\n" % " ".join(str(int(i)) for i in sample))
        nonempty = 0
        for k, i in enumerate(sample):
            bits = np.unpackbits(answers[k].view(np.uint8), bitorder="little")[:K]
            ids = np.nonzero(bits)[0]
            if ids.size:
                nonempty += 1
                f.write("A %d %s\n" % (int(i), " ".join(str(int(d)) for d in ids)))
        for d in docs_s:
            f.write("D %d %s\n" % (d, " ".join(str(int(i)) for i in np.nonzero(cols[d])[0])))
    log(name, "wrote", path, "non-empty sampled answers", nonempty)
    return path


if __name__ == "__main__":
    names = sys.argv[1:] or list(SPECS)
    for nm in names:
        build(nm)
