"""Autotuner for the launch shapes of the fused apply kernels.

Single operators: every built launch shape of the kernel the operator uses
(FP64 box-cell shapes 0..9, mixed-precision shapes 0..6, the FP32 vector shapes 4..6
for FP32 only) is timed with the
library's per-launch HIP events (mf_timing) on the caller's buffers, and the
fastest is set on the operator.  Batches: every persistent-kernel shape (0..2)
is timed with events around mf_batch_apply.  Results are kept in a JSON cache
keyed by (GPU architecture, p, q, cells, columns, precision), so a later
process reuses the choice without timing.

The candidate shapes are the analogue of the paper's (b, alpha) sweep of its
GPU kernel (Sec. 4, tbl:batchsizeStudy): tile of columns per workgroup and
threads per workgroup, chosen per degree and column count.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence

from . import mfmv

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mfmv_tune.json")
N_BOX, N_MIXED, N_BATCH = mfmv.BOX_CFGS, mfmv.MIXED_CFGS, mfmv.BATCH_CFGS


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _load(path: str) -> dict:
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def _save(path: str, db: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    json.dump(db, open(tmp, "w"), indent=1, sort_keys=True)
    os.replace(tmp, path)


def operator_key(op: mfmv.Operator, nvec: int, precision: str) -> str:
    return f"{_arch()}/p{op.p}q{op.q}/cells{op.ncells}/nvec{nvec}/{precision}"


def _set(op: mfmv.Operator, precision: str, cfg: int) -> None:
    if precision == "fp64":
        op.set_launch(False, cfg)
    else:
        op.set_launch_mixed(cfg)


def tune_operator(op: mfmv.Operator, X, Y, precision: str = "fp64", reps: int = 10,
                  warmup: int = 2, cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> dict:
    """Pick the fastest launch shape for Y := A X at this column count; returns
    {"cfg": best, "ms": {cfg: kernel ms}} and leaves the choice set on `op`."""
    import torch
    key = operator_key(op, X.shape[1], precision)
    db = _load(cache) if cache else {}
    if not force and key in db:
        _set(op, precision, db[key]["cfg"])
        return db[key]
    times = {}
    n = N_BOX if precision == "fp64" else (N_MIXED if precision == "fp32" else mfmv.MIXED_MFMA_CFGS)
    for cfg in range(n):
        try:
            _set(op, precision, cfg)
        except mfmv.MfError:
            continue  # shape does not fit this degree
        for _ in range(warmup):
            op.apply(X, Y, precision=precision)
        torch.cuda.synchronize()
        op.timing(reps)
        for _ in range(reps):
            op.apply(X, Y, precision=precision)
        n, _z, k = op.timing_read()
        op.timing(0)
        times[cfg] = k / max(n, 1)
    best = min(times, key=times.get)
    _set(op, precision, best)
    rec = {"cfg": best, "ms": {str(c): t for c, t in times.items()}}
    if cache:
        db = _load(cache)
        db[key] = rec
        _save(cache, db)
    return rec


def tune_batch(batch: mfmv.Batch, Xs: Sequence, Ys: Sequence, reps: int = 5, warmup: int = 1) -> dict:
    """Pick the fastest persistent-kernel shape for this batch; returns
    {"cfg": best, "ms": {cfg: ms per batched apply}} and leaves it set."""
    import torch
    times = {}
    for cfg in range(N_BATCH):
        batch.set_launch(cfg)
        for _ in range(warmup):
            batch.apply(Xs, Ys)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            batch.apply(Xs, Ys)
        b.record()
        torch.cuda.synchronize()
        times[cfg] = a.elapsed_time(b) / reps
    best = min(times, key=times.get)
    batch.set_launch(best)
    return {"cfg": best, "ms": {str(c): t for c, t in times.items()}}
