"""RAMBO (Repeated And Merged BloOm filter) hot path on AMD Instinct MI355X.

The index and every step of building and querying it run in hand-written HIP
kernels behind the C ABI of ``librambo.so`` (``include/rambo.h``); this
package is the thin Python binding (``rambo.py``) and its build script.
"""
from .rambo import (EBUSY, EDEVICE, EINVAL, EIO, ENOMEM, ETRUNC, MODE_BATCHED, MODE_PLAIN, OK, OK_EMPTYQ, RESOLVE_AUTO,
                    RESOLVE_CANDIDATE, RESOLVE_DENSE, SERVE_CONTINUOUS, SERVE_SERIAL, SHARD, TERMS_OPAQUE, Rambo,
                    RamboError, Server, Tune, check_offsets, clock, lib, route)

__all__ = ["Rambo", "RamboError", "Server", "Tune", "lib", "check_offsets", "clock", "SERVE_CONTINUOUS",
           "SERVE_SERIAL", "MODE_PLAIN", "MODE_BATCHED", "RESOLVE_AUTO",
           "RESOLVE_DENSE", "RESOLVE_CANDIDATE", "TERMS_OPAQUE", "SHARD", "route", "OK", "OK_EMPTYQ", "EINVAL", "ENOMEM", "EDEVICE", "ETRUNC", "EBUSY",
           "EIO"]
