"""Measured choice of the FLASH parallelism P for a given batch.

The library's own choice for P <= 0 is a closed-form rule (the largest
power of two with P <= T/16 for the median length).  This helper instead
decodes the actual batch once per candidate P on the current stream, timed
with device events, and returns the fastest; results are memoised per
(model shape, method, length profile).  Every candidate gives the same
paths and scores (FLASH is exact for every P), so tuning never changes a
result.
"""
from __future__ import annotations

import hashlib

import numpy as np
import torch

from .decode import Batch, decode_batch

_cache: dict = {}


def _key(log_a, batch: Batch, method: str) -> str:
    shape = (log_a.K, "csr") if hasattr(log_a, "trans") else tuple(log_a.shape)
    lens = np.sort(np.asarray(batch.lengths, np.int64))
    h = hashlib.sha1(lens.tobytes()).hexdigest()[:16]
    return f"{shape}:{method}:{batch.n}:{h}"


def best_parallelism(log_a, batch: Batch, log_pi=None, candidates=(16, 32, 64, 128, 256, 512),
                     method: str = "flash", repeats: int = 1) -> tuple[int, dict]:
    """(best P, {P: ms}) for decoding `batch` with FLASH.  The batch's outputs
    hold the last candidate's (identical) results afterwards."""
    key = _key(log_a, batch, method)
    if key in _cache:
        return _cache[key]
    times, ws = {}, None
    for P in candidates:
        ws = decode_batch(log_a, batch, log_pi, method=method, P=P, ws=ws)   # warm-up, sizes ws
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(repeats):
            ws = decode_batch(log_a, batch, log_pi, method=method, P=P, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        times[P] = e0.elapsed_time(e1) / repeats
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return best, times
