"""Launch-shape tuning of the fused apply and of batches.

The timing and the JSON cache live in the library (mf_tune, mf_batch_tune of
include/mfmv.h); this module only supplies the default cache location.  The
candidate shapes are the analogue of the paper's sweep of its GPU kernel's
batch size and thread-block shape (Sec. 4, tbl:batchsizeStudy): tile of
columns per workgroup, columns per thread and threads per workgroup, one-shot
or persistent grid, chosen per degree, column count and precision.
"""
from __future__ import annotations

import os
from typing import Optional, Sequence

from . import mfmv

DEFAULT_CACHE = os.environ.get("MFMV_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "mfmv_tune.json"))


def _cache(cache: Optional[str]) -> Optional[str]:
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    return cache


def tune_operator(op: mfmv.Operator, nvec: int, precision: str = "fp64",
                  cache: Optional[str] = DEFAULT_CACHE) -> dict:
    """Fastest launch shape of `op` for nvec columns in this precision (kept on the
    operator); {"cfg": shape, "ms": {shape: median ms}} ("ms" empty if cached)."""
    return op.tune(nvec, precision, _cache(cache))


def tune_batch(batch: mfmv.Batch, Xs: Sequence, Ys: Sequence,
               cache: Optional[str] = DEFAULT_CACHE) -> dict:
    """Fastest launch shape of a batch on these buffers (kept on the batch)."""
    return {"cfg": batch.tune(Xs, Ys, _cache(cache))}
