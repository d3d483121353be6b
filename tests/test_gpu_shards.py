"""Sharding by document on one GPU (Section 5.3, Figure 3): routing with the
device hash tau, G shards built on the same device from the documents routed
to them (local ids, cells of their global ids), queried in both forms, and
their answers stacked at the global ids -- equal, bit for bit, to the
oracle's index built directly with the two-level partition b * tau(d) +
phi_r(d) over G * b cells. Shard files keep the global ids."""
import os
import tempfile

import numpy as np
import pytest

import gen
import oracle
from paper_1910_04358_amd import rambo as rb
from tests.gpu_util import make_reads, reads_to_dev, to_dev, to_host_u64

pytestmark = pytest.mark.gpu

K, G, b, R, m, eta, SEED, RSEED = 1200, 4, 25, 5, 1 << 21, 2, 6060, 424242
DM = gen.DocModel(seed=171, n_docs=K, length=8_000, docs_per_anc=40, mu_lo=0.005, mu_hi=0.02)
RM = gen.ReadModel(qseed=172, src_lo=0, src_hi=K, len_kind=0, median=300, sigma=1.0, lo=31, hi=3000,
                   err_lo=0.0, err_hi=0.01)


def test_routed_shards_stack_to_the_two_level_index():
    import torch
    ids = np.arange(K, dtype=np.uint64)
    tau = rb.route(to_dev(ids), G, RSEED).cpu().numpy().astype(np.int64)
    assert np.array_equal(tau, oracle.route(RSEED, G, range(K)))
    # the oracle's index with the two-level partition over G * b cells
    phi = oracle.Oracle(K, b, R, m, eta, SEED, alloc_bits=False).phis()
    two = oracle.Oracle(K, G * b, R, m, eta, SEED, cells=b * tau[None, :] + phi)
    docs = DM.docs(0, K)
    two.build_docs(docs, DM.length, 0, K)
    tbits = two.bits()
    reads = gen.reads(DM, RM, 2000)
    want, _ = two.query_seqs(reads.seqs, reads.offsets, oracle.MODE_ALG2)
    assert want.any(axis=1).sum() > 100
    seqs, offs = reads_to_dev(reads)
    W = (K + 63) // 64
    stacked = {mode: torch.zeros((reads.n, W), dtype=torch.int64, device="cuda")
               for mode in (rb.MODE_PLAIN, rb.MODE_BATCHED)}
    shards = []
    for g in range(G):
        gid = np.nonzero(tau == g)[0].astype(np.uint64)
        sh = rb.Rambo.shard(gid, b, R, m, eta, SEED)
        assert sh.is_shard and np.array_equal(sh.shard_ids(), gid)
        assert np.array_equal(sh.phi_table().astype(np.int64), phi[:, gid.astype(np.int64)])
        # local document l is global document gid[l]
        L = DM.length
        sel = np.concatenate([docs[int(d) * L:(int(d) + 1) * L] for d in gid])
        sh.insert_seqs(to_dev(np.arange(gid.size, dtype=np.uint64)), to_dev(sel),
                       to_dev(np.arange(gid.size + 1, dtype=np.uint64) * np.uint64(L)))
        sh.sync()
        # every BFU of the shard is the two-level index's BFU b * g + c
        for r in range(R):
            for c in range(b):
                assert np.array_equal(sh.dump_bfu(r, c), tbits[r, b * g + c]), (g, r, c)
        for mode, out in stacked.items():
            sh.set_mode(mode)
            sl = sh.query_seqs(seqs, offs)
            sh.stack_slice(sl, out)
        shards.append(sh)
    for mode, out in stacked.items():
        assert np.array_equal(to_host_u64(out), want), mode
    # a shard file keeps the global ids and answers the same after loading
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "shard1.rambo")
        shards[1].save(path)
        back = rb.Rambo.load(path)
        assert back.is_shard and np.array_equal(back.shard_ids(), shards[1].shard_ids())
        assert np.array_equal(back.copy_rows(), shards[1].copy_rows())
        a = to_host_u64(back.query_seqs(seqs, offs))
        assert np.array_equal(a, to_host_u64(shards[1].query_seqs(seqs, offs)))
        # a flipped global id is refused by the checksum
        raw = bytearray(open(path, "rb").read())
        raw[96] ^= 1
        open(path, "wb").write(bytes(raw))
        with pytest.raises(rb.RamboError) as e:
            rb.Rambo.load(path)
        assert e.value.status == rb.EIO
        back.close()
    # stacking refuses an output too narrow for the global ids, and ordinary indexes
    narrow = torch.zeros((reads.n, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(rb.RamboError):
        shards[0].stack_slice(shards[0].query_seqs(seqs, offs), narrow)
    plain = rb.Rambo(10, 2, 1, 1024, 1, 1)
    with pytest.raises(rb.RamboError):
        plain.stack_slice(torch.zeros((1, 1), dtype=torch.int64, device="cuda"), narrow[:1])
    plain.close()
    for sh in shards:
        sh.close()
    e_s, e_o = make_reads([])
    assert rb.route(to_dev(np.zeros(0, dtype=np.uint64)), G, RSEED).numel() == 0
