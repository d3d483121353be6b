"""Python binding of librambo.so (the C ABI in include/rambo.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI. Device buffers are torch tensors on the GPU
(int64 tensors carry uint64 bit patterns); streams are torch.cuda streams.
Importing works without a GPU; creating an index needs one and fails loudly
if the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librambo.so")
_lib = None

OK, EINVAL, ENOMEM, EDEVICE, ETRUNC, EBUSY, EIO = 0, -1, -2, -3, -4, -5, -6
OK_EMPTYQ = 1  # success; some query held no term (answered with every document)
MODE_PLAIN, MODE_BATCHED = 0, 1
RESOLVE_AUTO, RESOLVE_DENSE, RESOLVE_CANDIDATE = 0, 1, 2
TERMS_OPAQUE, SHARD = 1, 2
MAX_R, MAX_ETA, MAX_B = 8, 16, 8192

# every function the C ABI exports, with its ctypes signature
_u64, _u32, _i32, _vp, _cp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_char_p


class Layout(ctypes.Structure):
    _fields_ = [("K", _u64), ("m", _u64), ("seed", _u64), ("B", _u32), ("R", _u32), ("eta", _u32),
                ("row_words", _u32), ("W", _u64), ("index_bytes", _u64), ("rows", _vp), ("flags", _u32)]


class TuneC(ctypes.Structure):
    _fields_ = [("seg", _i32), ("tile", _i32), ("waves_per_cu", _i32), ("wpb", _i32), ("grab", _i32),
                ("sched", _i32), ("tuned", _i32)]


SIGNATURES = {
    "rambo_create": ([_u64, _u32, _u32, _u64, _u32, _u64], _vp),
    "rambo_create_ex": ([_u64, _u32, _u32, _u64, _u32, _u64, _u32], _vp),
    "rambo_query_term_sets": ([_vp, _vp, _vp, _u64, _vp, _vp], _i32),
    "rambo_destroy": ([_vp], None),
    "rambo_last_error": ([], _cp),
    "rambo_last_status": ([], _i32),
    "rambo_sync": ([_vp, _vp], _i32),
    "rambo_layout": ([_vp, ctypes.POINTER(Layout)], _i32),
    "rambo_result_words": ([_vp], _u64),
    "rambo_index_bytes": ([_vp], _u64),
    "rambo_hash_params": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "rambo_phi_table": ([_vp, _vp], _i32),
    "rambo_dump_bfu": ([_vp, _u32, _u32, _vp], _i32),
    "rambo_copy_rows": ([_vp, _u64, _u64, _vp], _i32),
    "rambo_save": ([_vp, ctypes.c_char_p], _i32),
    "rambo_load": ([ctypes.c_char_p], _vp),
    "rambo_fold": ([_vp], _i32),
    "rambo_insert": ([_vp, _u64, _vp, _u64], _i32),
    "rambo_insert_batch": ([_vp, _vp, _vp, _vp, _u64, _vp], _i32),
    "rambo_insert_seqs": ([_vp, _vp, _vp, _vp, _u64, _vp], _i32),
    "rambo_query_kmers": ([_vp, _vp, _u64, _vp, _vp], _i32),
    "rambo_query_seqs": ([_vp, _vp, _vp, _u64, _vp, _vp], _i32),
    "rambo_query_seqs_ids": ([_vp, _vp, _vp, _u64, _vp, _vp, _vp, _u64, _vp], _i32),
    "rambo_query_seqs_ids_noalloc": ([_vp, _vp, _vp, _u64, _vp, _vp, _vp, _u64, _vp], _i32),
    "rambo_route": ([_vp, _u64, _u32, _u64, _vp, _vp], _i32),
    "rambo_create_shard": ([_u64, _u32, _u32, _u64, _u32, _u64, _vp], _vp),
    "rambo_shard_ids": ([_vp, _vp], _i32),
    "rambo_stack_slice": ([_vp, _vp, _u64, _vp, _u64, _vp], _i32),
    "rambo_set_mode": ([_vp, _i32], _i32),
    "rambo_set_resolve": ([_vp, _i32], _i32),
    "rambo_set_early_exit": ([_vp, _i32], _i32),
    "rambo_set_probe_counter": ([_vp, _vp], _i32),
    "rambo_set_sparse_counter": ([_vp, _vp], _i32),
    "rambo_autotune": ([_vp, _vp, _vp, _u64, _vp, _vp], _i32),
    "rambo_get_tune": ([_vp, ctypes.POINTER(TuneC)], _i32),
    "rambo_set_tune": ([_vp, ctypes.POINTER(TuneC)], _i32),
    "rambo_last_batch_ms": ([_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)], _i32),
    "rambo_clock": ([], ctypes.c_double),
    "rambo_server_start": ([_vp, _vp], _vp),
    "rambo_server_submit": ([_vp, _vp, _u64, _u64, ctypes.c_double], _i32),
    "rambo_server_submit_schedule": ([_vp, _vp, _vp, _u64, _vp, _u64], _i32),
    "rambo_server_poll": ([_vp, _vp, _vp, _u32, ctypes.c_double], _i32),
    "rambo_server_stats": ([_vp, _vp], _i32),
    "rambo_server_stop": ([_vp], _i32),
}

SERVE_CONTINUOUS, SERVE_SERIAL = 0, 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", _u64), ("slots", _u32), ("max_batch_reads", _u32), ("max_batch_bytes", _u64),
                ("policy", _u32), ("queue_cap", _u32), ("direct_below", _u32), ("batch_wait_us", _u32)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", _u64), ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int32), ("batch_reads", _u32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, _u64) for n in ("submitted", "completed", "rejected", "batches", "max_batch_reads",
                                     "max_inflight_bytes", "backpressure_waits", "pending", "inflight_bytes")]


class RamboError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


def lib():
    """Load librambo.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librambo.so is not built (python -m paper_1910_04358_amd.build)")
        # torch ships its own HIP runtime under the same soname as the system
        # one; it must be loaded first so that both share one runtime (and one
        # view of device memory and streams).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, res
        _lib = L
    return _lib


def _check(st: int):
    if st < 0:
        raise RamboError(st, lib().rambo_last_error().decode(errors="replace"))
    return st


def _dptr(t, name, dtypes=None):
    """Device pointer of a contiguous CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _i64():
    import torch
    return (torch.int64, torch.uint64) if hasattr(torch, "uint64") else (torch.int64,)


@dataclass
class Tune:
    seg: int
    tile: int
    waves_per_cu: int
    wpb: int
    grab: int
    sched: int = 2  # the library's default: scout schedule
    tuned: bool = False


class Rambo:
    """A RAMBO index resident on the current GPU."""

    def __init__(self, K: int, B: int, R: int, m: int, eta: int, seed: int, opaque_terms: bool = False):
        """opaque_terms: documents are sets of opaque 64-bit terms (word ids)
        instead of 31-mers; see rambo_create_ex."""
        L = lib()
        self._adopt(L.rambo_create_ex(K, B, R, m, eta, seed, TERMS_OPAQUE if opaque_terms else 0))

    @classmethod
    def shard(cls, global_ids, B: int, R: int, m: int, eta: int, seed: int) -> "Rambo":
        """A shard (Section 5.3) of len(global_ids) local documents; local
        document l stands for global document global_ids[l]."""
        g = np.ascontiguousarray(global_ids, dtype=np.uint64)
        obj = cls.__new__(cls)
        obj._h = None
        obj._adopt(lib().rambo_create_shard(g.size, B, R, m, eta, seed, ctypes.c_void_p(g.ctypes.data)))
        return obj

    def shard_ids(self) -> np.ndarray:
        out = np.zeros(self.K, dtype=np.uint64)
        _check(lib().rambo_shard_ids(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def stack_slice(self, slice_, out, stream=None) -> None:
        """OR this shard's answer rows (local ids) into out at the documents'
        global ids (out: (n, out_words) int64 device tensor, zeroed by the
        caller before the first shard)."""
        n = out.shape[0]
        if slice_.numel() < n * self.W:
            raise ValueError("slice too small")
        _check(lib().rambo_stack_slice(self._h, _dptr(slice_, "slice", _i64()), n, _dptr(out, "out", _i64()),
                                       out.shape[1], _stream(stream)))

    def _adopt(self, h):
        if not h:
            L = lib()
            raise RamboError(L.rambo_last_status(), L.rambo_last_error().decode(errors="replace"))
        self._h = h
        lay = self.layout()
        self.K, self.B, self.R, self.m = int(lay.K), int(lay.B), int(lay.R), int(lay.m)
        self.eta, self.seed = int(lay.eta), int(lay.seed)
        self.opaque_terms = bool(lay.flags & TERMS_OPAQUE)
        self.is_shard = bool(lay.flags & SHARD)
        self.W, self.row_words, self.index_bytes = int(lay.W), int(lay.row_words), int(lay.index_bytes)

    # -- index files
    def save(self, path) -> None:
        """Write the index to a file (header, then the row array; see rambo_save)."""
        _check(lib().rambo_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path) -> "Rambo":
        """An index read from a file written by save(), on the current GPU;
        raises RamboError (status EIO) for a missing, foreign or corrupted file."""
        obj = cls.__new__(cls)
        obj._h = None
        obj._adopt(lib().rambo_load(os.fsencode(path)))
        return obj

    def close(self):
        if getattr(self, "_h", None):
            lib().rambo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- introspection
    def layout(self) -> Layout:
        lay = Layout()
        _check(lib().rambo_layout(self._h, ctypes.byref(lay)))
        return lay

    def hash_params(self) -> dict:
        R, E = self.R, self.R * self.eta
        arrs = [np.zeros(R, np.uint64), np.zeros(R, np.uint64)] + [np.zeros(E, np.uint64) for _ in range(4)]
        _check(lib().rambo_hash_params(self._h, *[ctypes.c_void_p(a.ctypes.data) for a in arrs]))
        return dict(zip(("pa", "pb", "Alo", "Ahi", "Clo", "Chi"), arrs))

    def phi_table(self) -> np.ndarray:
        out = np.zeros((self.R, self.K), dtype=np.uint32)
        _check(lib().rambo_phi_table(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def dump_bfu(self, r: int, b: int) -> np.ndarray:
        out = np.zeros((self.m + 63) // 64, dtype=np.uint64)
        _check(lib().rambo_dump_bfu(self._h, r, b, ctypes.c_void_p(out.ctypes.data)))
        return out

    def copy_rows(self, offset: int = 0, nbytes: int | None = None) -> np.ndarray:
        nbytes = self.index_bytes - offset if nbytes is None else nbytes
        out = np.zeros(nbytes // 4, dtype=np.uint32)
        _check(lib().rambo_copy_rows(self._h, offset, nbytes, ctypes.c_void_p(out.ctypes.data)))
        return out

    def bfu_major(self) -> np.ndarray:
        """The whole index as (R, B, ceil(m/64)) uint64 Bloom filters (small indexes)."""
        rows = self.copy_rows().reshape(self.R, self.m, self.row_words)
        out = np.zeros((self.R, self.B, (self.m + 63) // 64), dtype=np.uint64)
        for b in range(self.B):
            col = ((rows[:, :, b >> 5] >> np.uint32(b & 31)) & np.uint32(1)).astype(np.uint8)
            pad = (-self.m) % 64
            if pad:
                col = np.concatenate([col, np.zeros((self.R, pad), np.uint8)], axis=1)
            out[:, b, :] = np.packbits(col, axis=1, bitorder="little").view(np.uint64)
        return out

    def fold(self) -> None:
        """Fold B -> B/2 cells in place (Section 5.3)."""
        _check(lib().rambo_fold(self._h))
        lay = self.layout()
        self.B, self.row_words, self.index_bytes = int(lay.B), int(lay.row_words), int(lay.index_bytes)

    # -- construction
    def insert(self, doc_id: int, kmers) -> None:
        k = np.ascontiguousarray(kmers, dtype=np.uint64)
        _check(lib().rambo_insert(self._h, doc_id, ctypes.c_void_p(k.ctypes.data), k.size))

    def insert_batch(self, doc_ids, kmer_offsets, kmers, stream=None) -> None:
        ok = _i64()
        n = doc_ids.numel()
        if kmer_offsets.numel() != n + 1:
            raise ValueError("kmer_offsets must have len(doc_ids) + 1 entries")
        _check(lib().rambo_insert_batch(self._h, _dptr(doc_ids, "doc_ids", ok), _dptr(kmer_offsets, "kmer_offsets", ok),
                                        _dptr(kmers, "kmers", ok), n, _stream(stream)))

    def insert_seqs(self, doc_ids, seqs, offsets, stream=None) -> None:
        import torch
        ok = _i64()
        n = doc_ids.numel()
        if offsets.numel() != n + 1:
            raise ValueError("offsets must have len(doc_ids) + 1 entries")
        _check(lib().rambo_insert_seqs(self._h, _dptr(doc_ids, "doc_ids", ok), _dptr(seqs, "seqs", (torch.uint8,)),
                                       _dptr(offsets, "offsets", ok), n, _stream(stream)))

    # -- queries
    def query_kmers(self, kmers, out=None, stream=None):
        import torch
        n = kmers.numel()
        if out is None:
            out = torch.empty((n, self.W), dtype=torch.int64, device=kmers.device)
        if out.numel() < n * self.W:
            raise ValueError("out too small")
        if n:
            _check(lib().rambo_query_kmers(self._h, _dptr(kmers, "kmers", _i64()), n, _dptr(out, "out", _i64()),
                                           _stream(stream)))
        return out

    def query_kmers_host(self, kmers) -> np.ndarray:
        """Single k-mer queries from a host array (synchronous copy in and
        out); returns a host [n][W] uint64 array."""
        k = np.ascontiguousarray(kmers, dtype=np.uint64)
        out = np.zeros((k.size, self.W), dtype=np.uint64)
        if k.size:
            _check(lib().rambo_query_kmers(self._h, ctypes.c_void_p(k.ctypes.data), k.size,
                                           ctypes.c_void_p(out.ctypes.data), None))
        return out

    def query_term_sets(self, terms, offsets, out=None, stream=None, check=True):
        """Term-set queries: set i is terms[offsets[i] .. offsets[i+1])
        (device int64 tensors); returns out [n][W]."""
        import torch
        n = offsets.numel() - 1
        if check:
            check_offsets(offsets, terms.numel())
        if out is None:
            out = torch.empty((max(n, 0), self.W), dtype=torch.int64, device=offsets.device)
        if out.numel() < n * self.W:
            raise ValueError("out too small")
        if n > 0:
            if terms.numel() == 0:
                terms = torch.zeros(1, dtype=torch.int64, device=offsets.device)
            _check(lib().rambo_query_term_sets(self._h, _dptr(terms, "terms", _i64()), _dptr(offsets, "offsets", _i64()),
                                               n, _dptr(out, "out", _i64()), _stream(stream)))
        return out

    def query_seqs(self, seqs, offsets, out=None, stream=None, check=True):
        import torch
        n = offsets.numel() - 1
        if check:
            check_offsets(offsets, seqs.numel())
        if out is None:
            out = torch.empty((max(n, 0), self.W), dtype=torch.int64, device=seqs.device)
        if out.numel() < n * self.W:
            raise ValueError("out too small")
        if n > 0:
            _check(lib().rambo_query_seqs(self._h, _dptr(seqs, "seqs", (torch.uint8,)), _dptr(offsets, "offsets", _i64()),
                                          n, _dptr(out, "out", _i64()), _stream(stream)))
        return out

    def query_seqs_ids(self, seqs, offsets, ids_cap: int, scratch=None, stream=None, check=True):
        """Returns (ids int32 tensor, id_offsets int64 tensor); raises
        RamboError(ETRUNC) with .required set if ids_cap is too small. The
        call's status (OK, or OK_EMPTYQ if some read held no valid window) is
        left in self.last_status."""
        import torch
        n = offsets.numel() - 1
        if check:
            check_offsets(offsets, seqs.numel())
        dev = seqs.device
        if scratch is None:
            scratch = torch.empty((max(n, 1), self.W), dtype=torch.int64, device=dev)
        ids = torch.empty(max(ids_cap, 1), dtype=torch.int32, device=dev)
        id_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        st = lib().rambo_query_seqs_ids(self._h, _dptr(seqs, "seqs", (torch.uint8,)), _dptr(offsets, "offsets", _i64()), n,
                                        _dptr(scratch, "scratch", _i64()), _dptr(ids, "ids", (torch.int32,)),
                                        _dptr(id_off, "id_offsets", _i64()), ids_cap, _stream(stream))
        if st == ETRUNC:
            e = RamboError(st, lib().rambo_last_error().decode())
            e.required = int(id_off[-1].item())
            raise e
        self.last_status = _check(st)
        return ids[: int(id_off[-1].item())], id_off

    # -- options
    def set_mode(self, mode: int) -> None:
        _check(lib().rambo_set_mode(self._h, mode))

    def set_resolve(self, resolve: int) -> None:
        _check(lib().rambo_set_resolve(self._h, resolve))

    def set_early_exit(self, on: bool) -> None:
        _check(lib().rambo_set_early_exit(self._h, int(bool(on))))

    def set_probe_counter(self, counter) -> None:
        ptr = None if counter is None else _dptr(counter, "counter", _i64())
        _check(lib().rambo_set_probe_counter(self._h, ptr))

    def set_sparse_counter(self, counters) -> None:
        """RAMBO+ tallies (6 int64 words on the device; None disables); see
        rambo_set_sparse_counter."""
        ptr = None
        if counters is not None:
            if counters.numel() < 6:
                raise ValueError("the sparse counter needs 6 words")
            ptr = _dptr(counters, "counters", _i64())
        _check(lib().rambo_set_sparse_counter(self._h, ptr))

    def sync(self, stream=None) -> int:
        """Wait for the handle's work on the stream; returns OK, or OK_EMPTYQ if
        a query without a term ran since the last sync (raises on errors)."""
        return _check(lib().rambo_sync(self._h, _stream(stream)))

    def autotune(self, seqs, offsets, out, stream=None) -> Tune:
        import torch
        n = offsets.numel() - 1
        _check(lib().rambo_autotune(self._h, _dptr(seqs, "seqs", (torch.uint8,)), _dptr(offsets, "offsets", _i64()), n,
                                    _dptr(out, "out", _i64()), _stream(stream)))
        return self.get_tune()

    def last_batch_ms(self):
        """(graph_ms, kernel_ms) of the most recent batched launch."""
        g, k = ctypes.c_float(), ctypes.c_float()
        _check(lib().rambo_last_batch_ms(self._h, ctypes.byref(g), ctypes.byref(k)))
        return g.value, k.value

    def get_tune(self) -> Tune:
        t = TuneC()
        _check(lib().rambo_get_tune(self._h, ctypes.byref(t)))
        return Tune(t.seg, t.tile, t.waves_per_cu, t.wpb, t.grab, t.sched, bool(t.tuned))

    def set_tune(self, tune: Tune) -> None:
        t = TuneC(tune.seg, tune.tile, tune.waves_per_cu, tune.wpb, tune.grab, tune.sched, 1)
        _check(lib().rambo_set_tune(self._h, ctypes.byref(t)))


def route(doc_ids, G: int, route_seed: int, stream=None):
    """tau(d) of each document id (device int64 tensor): its shard, as an
    int32 device tensor (Section 5.3 routing; see rambo_route)."""
    import torch
    out = torch.empty(doc_ids.numel(), dtype=torch.int32, device=doc_ids.device)
    _check(lib().rambo_route(_dptr(doc_ids, "doc_ids", _i64()), doc_ids.numel(), G, route_seed,
                             _dptr(out, "shard", (torch.int32,)), _stream(stream)))
    return out


def clock() -> float:
    return lib().rambo_clock()


class Server:
    """Continuous-batching server over a resident index (RAMBO_SERVE_*)."""

    def __init__(self, idx: "Rambo", budget_bytes=4 << 30, slots=4, max_batch_reads=8192,
                 max_batch_bytes=8 << 20, policy=SERVE_CONTINUOUS, queue_cap=1 << 20, direct_below=65,
                 batch_wait_us=0):
        self.idx = idx
        cfg = ServerConfig(budget_bytes, slots, max_batch_reads, max_batch_bytes, policy, queue_cap, direct_below,
                           batch_wait_us)
        self._s = lib().rambo_server_start(idx._h, ctypes.byref(cfg))
        if not self._s:
            raise RamboError(lib().rambo_last_status(), lib().rambo_last_error().decode(errors="replace"))
        self._keep = []

    def submit(self, read: bytes, tag: int, t_arrival: float | None = None) -> int:
        t = clock() if t_arrival is None else t_arrival
        return lib().rambo_server_submit(self._s, read, len(read), tag, t)

    def submit_schedule(self, seqs: np.ndarray, offsets: np.ndarray, t_arrival: np.ndarray, tag0: int = 0):
        seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        t = np.ascontiguousarray(t_arrival, dtype=np.float64)
        _check(lib().rambo_server_submit_schedule(self._s, ctypes.c_void_p(seqs.ctypes.data),
                                                  ctypes.c_void_p(offsets.ctypes.data), offsets.size - 1,
                                                  ctypes.c_void_p(t.ctypes.data), tag0))

    def poll(self, max_n=4096, timeout_s=0.05, results=True):
        comp = (Completion * max_n)()
        res = np.zeros((max_n, self.idx.W), dtype=np.uint64) if results else None
        k = _check(lib().rambo_server_poll(self._s, comp, ctypes.c_void_p(res.ctypes.data) if results else None,
                                           max_n, timeout_s))
        return comp[:k], (res[:k] if results else None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().rambo_server_stats(self._s, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}

    def stop(self):
        if getattr(self, "_s", None):
            s, self._s = self._s, None
            _check(lib().rambo_server_stop(s))

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def check_offsets(offsets, nbytes: int) -> None:
    """Host-side check that offsets are non-decreasing and inside the buffer
    (the kernels trust them)."""
    o = offsets.detach().to("cpu").numpy().astype(np.uint64) if hasattr(offsets, "detach") else np.asarray(offsets)
    if o.size == 0:
        raise ValueError("offsets must have n+1 >= 1 entries")
    if np.any(o[1:] < o[:-1]) or int(o[-1]) > nbytes:
        raise ValueError("offsets must be non-decreasing and within the sequence buffer")
