"""Helpers for GPU tests: upload generator inputs, build indexes through the
C ABI, and build the matching oracle on the CPU from the same inputs."""
from __future__ import annotations

import numpy as np

import gen
import oracle


def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(cuda())


def to_host_u64(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def build_gpu_seqs(idx, dm: gen.DocModel, d0: int, nd: int, chunk: int = 256):
    """Insert documents d0..d0+nd-1 as sequences, chunk documents per call."""
    import torch
    for c0 in range(d0, d0 + nd, chunk):
        c1 = min(d0 + nd, c0 + chunk)
        docs = dm.docs(c0, c1 - c0)
        offs = np.arange(c1 - c0 + 1, dtype=np.uint64) * np.uint64(dm.length)
        ids = np.arange(c0, c1, dtype=np.uint64)
        idx.insert_seqs(to_dev(ids), to_dev(docs), to_dev(offs))
    torch.cuda.synchronize()
    idx.sync()


def build_oracle(w_or_params, dm: gen.DocModel, nd: int | None = None) -> oracle.Oracle:
    K, B, R, m, eta, seed = w_or_params
    o = oracle.Oracle(K, B, R, m, eta, seed)
    nd = dm.n_docs if nd is None else nd
    step = 512
    for c0 in range(0, nd, step):
        c1 = min(nd, c0 + step)
        o.build_docs(dm.docs(c0, c1 - c0), dm.length, c0, c1 - c0)
    return o


def reads_to_dev(r: gen.Reads):
    return to_dev(r.seqs), to_dev(r.offsets)


def make_reads(seqs: list[bytes]):
    """Ragged read batch from a list of byte strings."""
    offs = np.zeros(len(seqs) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(s) for s in seqs])
    buf = np.frombuffer(b"".join(seqs), dtype=np.uint8) if seqs and offs[-1] else np.zeros(1, np.uint8)
    return buf.copy(), offs
