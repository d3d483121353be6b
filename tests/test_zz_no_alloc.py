"""rambo_query_seqs_ids_noalloc, the id-list query for callers that cannot
allocate, against rambo_query_seqs_ids (the entry point it varies) and the
oracle on the same inputs: id lists, offsets and status equal, on two calls
in a row, the second with a smaller batch, so that what the first call left
in the library's fixed scratch array cannot leak into the second."""
import ctypes

import numpy as np
import pytest

import gen
import oracle
from paper_1910_04358_amd import rambo as rb
from tests import _ref
from tests.gpu_util import build_gpu_seqs, build_oracle, make_reads, to_dev

pytestmark = pytest.mark.gpu

K, B, R, M, ETA, SEED = 400, 100, 5, 1 << 21, 2, 8080
DM = gen.DocModel(seed=91, n_docs=K, length=10_000, docs_per_anc=40, mu_lo=0.005, mu_hi=0.02)
RM = gen.ReadModel(qseed=92, src_lo=0, src_hi=K, len_kind=0, median=300, sigma=1.0, lo=31, hi=4000,
                   err_lo=0.0, err_hi=0.01)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def noalloc(idx, seqs, offs, n, bits, cap):
    import torch
    ids = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    id_off = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
    st = rb.lib().rambo_query_seqs_ids_noalloc(idx._h, _p(seqs), _p(offs), n, _p(bits), _p(ids), _p(id_off), cap,
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, ids, id_off


def lists(ids, id_off):
    ids, id_off = ids.cpu().numpy(), id_off.cpu().numpy()
    return [ids[id_off[i]:id_off[i + 1]].tolist() for i in range(id_off.size - 1)]


def test_noalloc_ids_equal_the_allocating_entry_point():
    import torch
    idx = rb.Rambo(K, B, R, M, ETA, SEED)
    build_gpu_seqs(idx, DM, 0, K)
    o = build_oracle((K, B, R, M, ETA, SEED), DM)
    big = gen.reads(DM, RM, 2500)
    d3 = DM.doc(3)
    small_list = [big.read(i) for i in range(0, 700)] + [b"N" * 80, d3[500:900]]
    batches = [(big.seqs, big.offsets, None), (*make_reads(small_list), small_list)]
    for k, (s_np, o_np, lst) in enumerate(batches):
        n = o_np.size - 1
        if lst is None:
            want, _ = o.query_seqs(s_np, o_np, oracle.MODE_ALG2)
        else:
            want = np.stack([o.query_seq(x) for x in lst])
        want_lists = [sorted(_ref.bits_to_ids(want[i], K)) for i in range(n)]
        seqs, offs = to_dev(s_np), to_dev(o_np)
        bits = torch.full((n, idx.W), -1, dtype=torch.int64, device="cuda")
        st, ids, id_off = noalloc(idx, seqs, offs, n, bits, 200_000)
        torch.cuda.synchronize()
        assert st == (rb.OK_EMPTYQ if lst is not None else rb.OK), (k, st, rb.lib().rambo_last_error())
        got = lists(ids, id_off)
        assert got == want_lists, k
        for mode in (rb.MODE_PLAIN, rb.MODE_BATCHED):
            idx.set_mode(mode)
            ref_ids, ref_off = idx.query_seqs_ids(seqs, offs, ids_cap=200_000)
            assert idx.last_status == st
            assert np.array_equal(ref_off.cpu().numpy(), id_off.cpu().numpy()), (k, mode)
            assert lists(ref_ids, ref_off) == got, (k, mode)
        idx.set_mode(rb.MODE_PLAIN)
        # too small an id buffer: ETRUNC with the required size, ids untouched
        total = int(id_off[-1].item())
        if total:
            st2, ids2, off2 = noalloc(idx, seqs, offs, n, bits, total - 1)
            assert st2 == rb.ETRUNC and int(off2[-1].item()) == total
            assert bool((ids2 == -7).all())
    # limits and the empty batch
    e_s, e_o = make_reads([])
    bits = torch.empty((1, idx.W), dtype=torch.int64, device="cuda")
    st, ids, id_off = noalloc(idx, to_dev(e_s), to_dev(e_o), 0, bits, 0)
    assert st == rb.OK and id_off.cpu().tolist() == [0]
    one = to_dev(np.zeros(1, dtype=np.uint8))
    offs_big = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = rb.lib().rambo_query_seqs_ids_noalloc(idx._h, _p(one), _p(offs_big), (1 << 20) + 1, _p(bits), _p(bits),
                                               _p(offs_big), 0, None)
    assert st == rb.EINVAL and b"limit" in rb.lib().rambo_last_error()
    idx.close()
