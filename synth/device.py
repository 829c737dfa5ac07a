"""Transport of generated blocks to a device tensor (no method arithmetic).

A block too large to hold twice on the host (1024 complex bands of a
120x120x160 grid are 37.7 GB) is generated chunk by chunk on host threads
and copied into one preallocated device tensor through two pinned staging
buffers, so that generation of one chunk overlaps the copy of the previous.
"""
import sys

import numpy as np


def block_to_device(s, device, dtype=None, chunk_bytes=1 << 30):
    """[nb][Ng] device tensor holding the block of system s (lazy or not),
    converted to dtype (default: float64 / complex128) on the host side of
    the copy."""
    import torch
    cplx = s.is_complex
    if dtype is None:
        dtype = torch.complex128 if cplx else torch.float64
    nb, ng = s.nb, s.ng
    out = torch.empty((nb, ng), dtype=dtype, device=device)
    src_bytes = ng * (16 if cplx else 8)
    chunk = max(1, min(nb, chunk_bytes // src_bytes))
    stream = torch.cuda.Stream(device=device)
    pinned = [torch.empty((chunk, ng), dtype=dtype, pin_memory=True) for _ in range(2)]
    done = [None, None]
    nchunks = (nb + chunk - 1) // chunk
    for i, lo in enumerate(range(0, nb, chunk)):
        hi = min(nb, lo + chunk)
        if nchunks >= 8 and i % max(1, nchunks // 8) == 0:
            # progress on stderr: a large block takes minutes to generate
            print(f"[synth] bands {lo}..{hi} of {nb}", file=sys.stderr, flush=True)
        slot = i % 2
        if done[slot] is not None:
            done[slot].synchronize()
        host = np.ascontiguousarray(s.bands(lo, hi).reshape(hi - lo, ng))
        buf = pinned[slot][:hi - lo]
        buf.copy_(torch.from_numpy(host))
        with torch.cuda.stream(stream):
            out[lo:hi].copy_(buf, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        done[slot] = ev
    stream.synchronize()
    return out
