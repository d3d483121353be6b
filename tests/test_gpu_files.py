"""Index files (rambo_save / rambo_load): a loaded index equals the saved one
byte for byte and answers every read as the oracle does, in both forms; a
folded index keeps its folded partition and an opaque-term index its flag;
missing, foreign, short, long, corrupted and altered files are refused."""
import numpy as np
import pytest

import gen
import oracle
from paper_1910_04358_amd import rambo as rb
from tests.gpu_util import build_gpu_seqs, build_oracle, reads_to_dev, to_host_u64

pytestmark = pytest.mark.gpu

HEADER = 96


def test_save_load_round_trip(tmp_path):
    K, B, R, m, eta, seed = 1000, 100, 5, 1 << 20, 2, 777
    dm = gen.DocModel(seed=72, n_docs=K, length=20_000, docs_per_anc=100, mu_lo=0.005, mu_hi=0.02)
    rm = gen.ReadModel(qseed=82, src_lo=0, src_hi=K, len_kind=0, median=300, sigma=1.0, lo=31, hi=10_000,
                       err_lo=0.0, err_hi=0.01)
    idx = rb.Rambo(K, B, R, m, eta, seed)
    build_gpu_seqs(idx, dm, 0, K)
    o = build_oracle((K, B, R, m, eta, seed), dm)
    reads = gen.reads(dm, rm, 1500)
    seqs, offs = reads_to_dev(reads)
    want, _ = o.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2)
    assert want.any(axis=1).sum() > 20
    p = tmp_path / "a.rambo"
    idx.save(p)
    assert p.stat().st_size == idx.index_bytes + HEADER
    ld = rb.Rambo.load(p)
    assert (ld.K, ld.B, ld.R, ld.m, ld.eta, ld.seed, ld.opaque_terms) == (K, B, R, m, eta, seed, False)
    assert np.array_equal(ld.copy_rows(), idx.copy_rows())
    for mode in (rb.MODE_PLAIN, rb.MODE_BATCHED):
        ld.set_mode(mode)
        assert np.array_equal(to_host_u64(ld.query_seqs(seqs, offs)), want), mode
    # a folded index is stored with its folded B, which derives the folded
    # partition: the loaded copy answers as the oracle's fold
    idx.fold()
    o2 = o.fold()
    idx.save(p)
    ld2 = rb.Rambo.load(p)
    assert ld2.B == B // 2 and ld2.index_bytes == idx.index_bytes
    want2, _ = o2.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2)
    assert np.array_equal(to_host_u64(ld2.query_seqs(seqs, offs)), want2)
    for x in (idx, ld, ld2):
        x.close()


def test_bad_files_are_refused(tmp_path):
    dm = gen.DocModel(seed=5, n_docs=200, length=2_000, docs_per_anc=20, mu_lo=0.01, mu_hi=0.01)
    idx = rb.Rambo(200, 40, 3, 1 << 16, 2, 99)
    build_gpu_seqs(idx, dm, 0, 200)
    p = tmp_path / "b.rambo"
    idx.save(p)
    raw = bytearray(p.read_bytes())
    corrupt = bytearray(raw)
    corrupt[HEADER + len(raw) // 2] ^= 0x10
    altered = bytearray(raw)
    altered[32] ^= 1  # the seed: other hash functions for the same rows
    cases = {"missing": None, "foreign": b"NOTRAMBO" + bytes(raw[8:]), "short": bytes(raw[:-4]),
             "long": bytes(raw) + b"\0", "corrupt": bytes(corrupt), "altered": bytes(altered),
             "header only": bytes(raw[:HEADER])}
    for name, data in cases.items():
        q = tmp_path / (name.replace(" ", "_") + ".rambo")
        if data is not None:
            q.write_bytes(data)
        with pytest.raises(rb.RamboError) as e:
            rb.Rambo.load(q)
        assert e.value.status == rb.EIO, name
    # the intact file still loads after the refusals
    ok = rb.Rambo.load(p)
    assert np.array_equal(ok.copy_rows(), idx.copy_rows())
    # an opaque-term index keeps its flag
    t = rb.Rambo(50, 10, 2, 4096, 2, 3, opaque_terms=True)
    t.save(tmp_path / "t.rambo")
    t2 = rb.Rambo.load(tmp_path / "t.rambo")
    assert t2.opaque_terms
    for x in (idx, ok, t, t2):
        x.close()
