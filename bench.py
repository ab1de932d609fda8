"""Benchmark of the matrix-free product Y = A X on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
                    [--workload c2|c3|c5] [--nvec N] [--no-cpu-baseline]

A step is one full product Y := A X (zero fill of Y, then the fused
extraction / sum-factorised cell operator / assembly kernel) over a batch of
nvec synthetic columns already resident in HBM.  Prints one JSON line.

The default workload is the periodic [0,10]^3 box with 16^3 cells, p = 6,
q = 7 (884,736 dofs), eight seeded Gaussian wells, nvec = 64, FP64.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "A·X GDoF·vec/s, FP64 vs mixed precision at ≤1e-6 rel err; %roofline"
UNIT = "GDoF·vec/s"
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (= FP64 matrix) peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_f64_traffic.json")
KERNEL_SOURCES = ["paper_2208_07129_amd/csrc/apply_box.hip", "paper_2208_07129_amd/csrc/sf_common.h",
                  "paper_2208_07129_amd/csrc/sf_tables.h"]


def flops_per_cell_vector(p: int, q: int) -> int:
    """Algorithmic FP64 flops of the sum-factorised cell operator, per cell and column:
    N and N^T stages 4(np^3 nq + np^2 nq^2 + np nq^3), Dt and Dt^T stages 12 nq^4,
    3x3 scaling and mass term 18 nq^3."""
    n, m = p + 1, q
    return 4 * (n ** 3 * m + n ** 2 * m ** 2 + n * m ** 3) + 12 * m ** 4 + 18 * m ** 3


def executed_flops_per_cell_vector(p: int, q: int, box: bool) -> int:
    """FP64 flops the axis-aligned-cell kernel executes per cell and column: N and N^T
    stages as above, one collapsed symmetric contraction per direction 6 nq^4, and
    7 nq^3 for the per-point scaling and sums (exact-zero coefficients not discounted)."""
    n, m = p + 1, q
    if not box:
        return flops_per_cell_vector(p, q)
    return 4 * (n ** 3 * m + n ** 2 * m ** 2 + n * m ** 3) + 6 * m ** 4 + 7 * m ** 3


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def workload(name: str, nvec: int | None):
    if name == "c2":
        w = W.config2()
    elif name == "c3":
        w = W.config3(nvec or 64)
    elif name == "c5":
        w = W.config5()
    else:
        raise SystemExit(f"unknown workload {name}")
    if nvec:
        w.nvec = nvec
    return w


def traffic_for(wname: str, nvec: int, precision: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or
    None if they were taken on a different kernel source or workload."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    key = f"{wname}/nvec{nvec}/{precision}"
    rec = t.get(key)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline_leg(w, Y_gpu_rows_fn, sample_cells: int):
    """Time the CPU oracle (as it stands) on a bounded sample of the same workload, and
    compare sampled GPU output rows with it.  The only place this script uses the oracle."""
    from oracle import fe_oracle as fo
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    cells = np.arange(min(sample_cells, orc.E))
    t1 = time.perf_counter()
    Ae = orc.element_matrices(cells)
    t2 = time.perf_counter()
    X = w.X()
    times = []
    for _ in range(3):
        ta = time.perf_counter()
        orc.apply(X, cells=cells, Ae=Ae)
        times.append(time.perf_counter() - ta)
    t_apply = float(np.median(times))
    owned = cells.size * w.p ** 3 if w.mesh.bc == W.BC_PERIODIC else cells.size * (w.p + 1) ** 3
    rate = owned * w.nvec / t_apply / 1e9
    # sampled-row parity of the GPU result measured above
    rows = np.random.default_rng(12345).choice(orc.ndofs, 8, replace=False)
    Yref = orc.apply_rows(X, rows)
    Yg = Y_gpu_rows_fn(rows)
    rel = float(np.linalg.norm(Yg - Yref) / np.linalg.norm(Yref))
    return {
        "value": rate, "unit": UNIT, "cores": int(threads), "kind": "oracle",
        "sample": (f"cell-matrix apply (numpy/OpenBLAS FP64) of {cells.size} of {orc.E} cells, "
                   f"all {w.nvec} columns, element matrices precomputed "
                   f"({t2 - t1:.1f} s for the sample; setup {t1 - t0:.1f} s); rate counts the "
                   f"{owned} dofs the sampled cells own; median of 3"),
    }, rel


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c5"])
    ap.add_argument("--nvec", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-cells", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of X into Y (known bytes), for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU's partition only; --gpus {a.gpus} is not supported "
              f"(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        return 2

    import torch
    from paper_2208_07129_amd import mfmv

    if not torch.cuda.is_available():
        raise SystemExit("no HIP device")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = workload(a.workload, a.nvec)
    prec = mfmv.PRECISIONS[a.precision]
    op = mfmv.Operator.from_workload(w)
    nvec = w.nvec
    X = torch.from_numpy(w.X()).to(dev)
    Y = torch.empty_like(X)
    free = int(op.ndofs - mfmv.constrained_mask(w.mesh, w.p).sum())
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream
    if a.calibrate_copy:
        # an elementwise kernel over many workgroups (reads X once, writes Y once)
        for _ in range(a.steps):
            torch.mul(X, 1.0, out=Y)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": X.numel() * 8,
                          "calibrate_copy_bytes_written": Y.numel() * 8, "steps": a.steps}))
        return 0

    def step():
        op.apply_ptr(X.data_ptr(), Y.data_ptr(), nvec, nvec, nvec, prec, sptr)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # untimed pass with the library's per-launch events: zero-fill and fused-kernel times
    op.timing(a.steps)
    for _ in range(a.steps):
        step()
    n_ev, zero_sum, kern_sum = op.timing_read()
    op.timing(0)
    kern_ms, zero_ms = kern_sum / n_ev, zero_sum / n_ev
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(a.steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    ms_per_step = total_ms / a.steps
    value = free * nvec / (ms_per_step * 1e-3) / 1e9

    flops = flops_per_cell_vector(w.p, w.q) * op.ncells * nvec
    achieved = flops / (kern_ms * 1e-3) / 1e12
    executed = executed_flops_per_cell_vector(w.p, w.q, box=True) * op.ncells * nvec
    traffic = traffic_for(w.name, nvec, a.precision)
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[a.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "cells": int(op.ncells), "p": w.p, "q": w.q,
                   "ndofs": int(op.ndofs), "free_dofs": free, "nvec": nvec,
                   "precision": a.precision, "layout": "dof-major, columns contiguous"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "apply_box_kernel", "kernel_ms": kern_ms,
                     "flops_per_launch": flops, "executed_flops_per_launch": executed,
                     "executed_frac": executed / (kern_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
        "zero_fill_ms": zero_ms,
    }
    if not a.no_cpu_baseline:
        def rows_fn(rows):
            idx = torch.from_numpy(np.asarray(rows)).to(dev)
            return Y[idx].cpu().numpy()
        cb, rel = cpu_baseline_leg(w, rows_fn, a.cpu_sample_cells)
        out["cpu_baseline"] = cb
        out["rel_err_vs_oracle_sampled"] = rel
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
