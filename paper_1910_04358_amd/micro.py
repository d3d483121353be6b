"""Random-access microbenchmarks (libmicro.so): the empirical ceiling of
uniformly random row reads and random atomic ORs over HBM-sized buffers.

python -m paper_1910_04358_amd.micro [--sizes-gib 1,8,40,96] [--rows 4,16,64,128]
prints one JSON line per case.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(_HERE, "libmicro.so")


def lib():
    import torch  # noqa: F401  (shares torch's HIP runtime)
    if not os.path.exists(SO):
        raise RuntimeError("libmicro.so is not built (python -m paper_1910_04358_amd.build)")
    L = ctypes.CDLL(SO)
    L.micro_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
    L.micro_run.restype = ctypes.c_double
    L.micro_per_lane.argtypes = [ctypes.c_int, ctypes.c_int]
    L.micro_per_lane.restype = ctypes.c_uint32
    L.micro_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32]
    L.micro_copy.restype = ctypes.c_double
    return L


def copy(nbytes: int = 1 << 30) -> float:
    """Run the plain copy kernel over nbytes (multiple of 16); returns ms."""
    import torch
    L = lib()
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    ms = L.micro_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), nbytes, n_cu * 16)
    if ms < 0:
        raise RuntimeError("micro_copy failed")
    return ms


def run(sizes_gib, rows, iters=16, reps=3, atomics=True, coop_rows=(32, 64, 128, 256)):
    """Every case on buffers of each size; one JSON line per case."""
    import torch
    L = lib()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = n_cu * 16
    sink = torch.zeros(1024 * 4, dtype=torch.int32, device="cuda")
    out = []
    for gib in sizes_gib:
        nbytes = int(gib * (1 << 30))
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        cases = [(0, rb) for rb in rows] + [(2, rb) for rb in coop_rows] + ([(1, 4)] if atomics else [])
        for kind, rb in cases:
            best = None
            for rep in range(reps):
                ms = L.micro_run(kind, ctypes.c_void_p(buf.data_ptr()), nbytes, rb, blocks, iters, 1234 + rep,
                                 ctypes.c_void_p(sink.data_ptr()))
                if ms < 0:
                    raise RuntimeError("micro_run failed (%g)" % ms)
                best = ms if best is None else min(best, ms)
            n = blocks * 256 * iters * L.micro_per_lane(kind, rb)
            if kind == 2:
                n //= rb // 16  # rows: rb/16 lanes share one
            rec = {"kind": ("gather", "atomic_or", "coop_gather")[kind], "buffer_GiB": gib, "row_bytes": rb,
                   "ops": n, "ms": best, "ops_per_s": n / best * 1e3,
                   "useful_GBps": n * rb / best / 1e6, "line_GBps_at_128B": n * max(128, rb) / best / 1e6}
            print(json.dumps(rec), flush=True)
            out.append(rec)
        del buf
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes-gib", default="1,8,40,96")
    ap.add_argument("--rows", default="4,16,64,128")
    ap.add_argument("--coop-rows", default="32,64,128,256")
    ap.add_argument("--iters", type=int, default=16)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--no-atomics", action="store_true", help="leave out the atomic OR case")
    ap.add_argument("--copy-gib", type=float, default=0,
                    help="also run the plain copy kernel over this many GiB (scale for byte counters)")
    a = ap.parse_args()
    if a.copy_gib:
        nbytes = int(a.copy_gib * (1 << 30)) // 16 * 16
        print(json.dumps({"kind": "copy", "bytes": nbytes, "ms": copy(nbytes)}), flush=True)
    run([float(s) for s in a.sizes_gib.split(",") if s], [int(r) for r in a.rows.split(",") if r], iters=a.iters,
        reps=a.reps, atomics=not a.no_atomics, coop_rows=[int(r) for r in a.coop_rows.split(",") if r])


if __name__ == "__main__":
    sys.exit(main())
