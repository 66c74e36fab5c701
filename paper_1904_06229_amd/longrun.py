"""Long permanents in slices, with progress and resume.

A permanent of size n has 2^(n-1) Gray terms; at n = 48 one launch runs for
minutes.  ``run_sliced`` cuts [0, 2^(n-1)) into equal power-of-two slices
(App. A, distribute, with aligned boundaries), evaluates each with
``perm_partial`` (the paper's subpermanent over that range), and adds the
slice sums in slice order.  Each slice is an independent unit of work: a
checkpoint file records every finished slice (JSON lines: slice index, the
double-double partial, the matrix fingerprint), so an interrupted run resumes
where it stopped and, because the order of the final sum is fixed, finishes
with the same bits.  This is also how the range would be divided between
devices.

The slice sums are combined by the library's perm_combine (App. A,
permanent: per = 2(-1)^n sum_k S_k, the parts added in slice order in
double-double, or as 128-bit integers for 0/1 input); this module only runs
the slices and keeps the checkpoint.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import binding as B


def fingerprint(A) -> str:
    """Hash of a device matrix's values and the layout the library sees."""
    import numpy as np
    a = A.detach().cpu().numpy()
    h = hashlib.sha256()
    h.update(str((a.shape, a.dtype.str, A.stride())).encode())
    h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:24]


def run_sliced(A, slices: int = 16, checkpoint: str | None = None, progress=None, **opts):
    """per(A) from `slices` perm_partial launches.  Returns (result, info).

    result: the library's Result of perm_combine over the slices (``.value``;
    ``.exact`` for 0/1 input).  info: per-slice seconds and walk-kernel
    milliseconds of the slices run now, and the number resumed.
    `opts` go to perm_partial (blocks, log2_chunk, precision, stream).
    """
    import torch
    n = A.shape[0]
    if n < 1:
        raise ValueError("n >= 1")
    T = 1 << (n - 1) if n < 64 else 1 << 63
    if slices < 1 or slices & (slices - 1) or slices > T:
        raise ValueError("slices must be a power of two no larger than 2^(n-1)")
    kind = {torch.float64: "real", torch.complex128: "complex", torch.uint8: "int01"}[A.dtype]
    width = T // slices
    fp = fingerprint(A)
    done = {}
    if checkpoint and os.path.exists(checkpoint):
        with open(checkpoint) as f:
            for line in f:
                rec = json.loads(line)
                if rec.get("fingerprint") == fp and rec.get("slices") == slices:
                    done[rec["slice"]] = rec
    resumed = len(done)
    secs, kms = [], []
    for k in range(slices):
        if k in done:
            continue
        t0 = time.perf_counter()
        r = B.perm_partial(A, k * width, width, **opts)
        dt = time.perf_counter() - t0
        secs.append(dt)
        kms.append(r.kernel_ms)
        rec = {"slice": k, "slices": slices, "fingerprint": fp, "kind": kind,
               "re": [r.re_hi, r.re_lo], "im": [r.im_hi, r.im_lo],
               "exact": None if r.exact is None else str(r.exact), "seconds": dt,
               "kernel_ms": r.kernel_ms, "max_drift": r.max_drift, "terms": r.terms,
               "chunks": r.chunks, "log2_chunk": r.log2_chunk, "blocks": r.blocks}
        done[k] = rec
        if checkpoint:
            with open(checkpoint, "a") as f:
                f.write(json.dumps(rec) + "\n")
        if progress:
            progress(f"slice {k + 1}/{slices} done in {dt:.1f} s")
    parts = []
    for k in range(slices):
        rec = done[k]
        parts.append(B.Result(rec["re"][0], rec["re"][1], rec["im"][0], rec["im"][1],
                              None if rec["exact"] is None else int(rec["exact"]),
                              rec.get("max_drift", -1.0), rec.get("terms", width),
                              rec.get("chunks", 0), rec.get("log2_chunk", 0),
                              rec.get("blocks", 0), rec.get("kernel_ms", 0.0),
                              1e3 * rec.get("seconds", 0.0)))
    result = B.perm_combine(kind, n, parts)
    return result, {"seconds": secs, "kernel_ms": kms, "resumed": resumed}
