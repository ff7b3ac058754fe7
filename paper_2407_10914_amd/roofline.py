"""The practical HBM ceiling of the device, measured with the library's own
streaming kernels (cg_stream_probe): plain read, write and copy streams of
float4 elements over a few GiB, swept over grid and block sizes with and
without non-temporal hints.  The best rate of each kind is the ceiling a
bandwidth-bound kernel is compared with, beside the published peak."""
from __future__ import annotations

import ctypes as C

from . import lib as L

KINDS = {"read": 0, "write": 1, "copy": 2}


def probe(kind, src, dst, nbytes, grid, block, nontemporal, reps=5):
    """Mean milliseconds per launch of one streaming kernel (torch tensors or
    raw device addresses)."""
    import torch

    ms = C.c_float()
    sp = src.data_ptr() if hasattr(src, "data_ptr") else src
    dp = dst.data_ptr() if hasattr(dst, "data_ptr") else dst
    L.check(L.load().cg_stream_probe(KINDS[kind], sp, dp, int(nbytes), int(grid), int(block),
                                     1 if nontemporal else 0, torch.cuda.current_stream().cuda_stream, int(reps),
                                     C.byref(ms)))
    return ms.value


def stream_ceiling(gib=4.0, reps=5, grids=None, blocks=(256, 512, 1024), log=None):
    """Sweep every kind x non-temporal x grid x block over `gib` GiB per buffer;
    returns {kind: best record} and the list of all records.  A record holds
    the rate in GB/s of bytes moved (read + written)."""
    import torch

    nbytes = int(gib * (1 << 30)) // 16 * 16
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    if grids is None:
        grids = [cus * m for m in (1, 2, 4, 8, 16, 32, 64)]
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    recs = []
    for kind in ("read", "write", "copy"):
        moved = nbytes * (2 if kind == "copy" else 1)
        for nt in (False, True):
            for block in blocks:
                for grid in grids:
                    ms = probe(kind, a, b, nbytes, grid, block, nt, reps)
                    r = dict(kind=kind, nontemporal=nt, grid=grid, block=block, ms=round(ms, 4),
                             gbs=round(moved / (ms * 1e-3) / 1e9, 1))
                    recs.append(r)
                    if log:
                        log(r)
    del a, b
    torch.cuda.empty_cache()
    best = {}
    for r in recs:
        if r["kind"] not in best or r["gbs"] > best[r["kind"]]["gbs"]:
            best[r["kind"]] = r
    return best, recs
