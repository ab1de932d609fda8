"""Benchmark of the matrix-free product Y = A X on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
                    [--workload c2|c3|c5] [--nvec N] [--legs all|headline|...]

A step is one full product Y := A X (zero fill of Y's cell-face rows, then the
fused extraction / sum-factorised cell operator / assembly kernel) over nvec
synthetic columns already resident in HBM.  The headline workload is the
periodic [0,10]^3 box with 16^3 cells, p = 6, q = 7 (884,736 dofs), eight
seeded Gaussian wells, nvec = 64, FP64.  The library records HIP events on the
launch stream around the zero fill and the fused kernel of every timed step;
the kernel's mean and median durations come from those events inside the timed
region.  Prints one JSON line; besides the headline it carries (default
--legs all) the FP32 / BF16 applies of the same workload, the p = 8 sweep over
16 / 64 / 256 columns in the three precisions, the 32-mesh batch (loop of
single applies, one batched call, graph replay), the block-CG solves of the
20^3 workload (Jacobi against the learned preconditioner) and the CPU oracle
timed with one thread and with all threads.  Every precision's error is
measured against the oracle on sampled rows.
"""
from __future__ import annotations

import argparse
import contextlib
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
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_f64_traffic.json")
KERNEL_SOURCES = ["paper_2208_07129_amd/csrc/apply_box.hip", "paper_2208_07129_amd/csrc/box_body.h",
                  "paper_2208_07129_amd/csrc/sf_common.h",
                  "paper_2208_07129_amd/csrc/sf_tables.h"]


def flops_per_cell_vector(p: int, q: int) -> int:
    """Algorithmic FP64 flops of the sum-factorised cell operator, per cell and column:
    N and N^T stages 4(np^3 nq + np^2 nq^2 + np nq^3), Dt and Dt^T stages 12 nq^4,
    3x3 scaling and mass term 18 nq^3."""
    n, m = p + 1, q
    return 4 * (n ** 3 * m + n ** 2 * m ** 2 + n * m ** 3) + 12 * m ** 4 + 18 * m ** 3


def _eo_flops(m: int, n: int) -> int:
    """Flops of one even-odd matvec (m outputs, n inputs): fold 2 floor(n/2), per
    output pair 2(h + mid) - 1 + 2h - 1 + 2, the middle row 2(h + mid) - 1."""
    h, mi, ho, mo = n // 2, n % 2, m // 2, m % 2
    return 2 * h + ho * (4 * h + 2 * mi) + mo * (2 * h + 2 * mi - 1)


def executed_flops_per_cell_vector(p: int, q: int, box: bool) -> int:
    """FP64 flops the axis-aligned-cell kernel executes per cell and column: every 1D
    contraction in even-odd form, the collapsed symmetric derivative contraction
    per direction, and the per-point scaling and sums (zero coefficients counted)."""
    n, m = p + 1, q
    if not box:
        return flops_per_cell_vector(p, q)
    interp = _eo_flops(m, n)      # N, nq x np
    back = _eo_flops(n, m)        # N^T, np x nq
    lap = _eo_flops(m, m)         # Lf, nq x nq
    return (n * n * interp + m * n * interp + m * m * interp            # P1 - P3
            + m * m * (lap + m) + m * m * (lap + 2 * m)                   # P4, P5
            + m * m * (2 * m + lap + 2 * m + back)                        # P6
            + m * n * back + n * n * back)                                # P7, P8


def algorithmic_bytes(ndofs: int, ncells: int, p: int, q: int, nvec: int) -> int:
    """HBM bytes the method must move per apply: X read and Y written once (FP64, for
    every precision), plus per cell the potential table (8 nq^3), the node map or its
    equivalent (4 np^3) and the 3x3 factor (48)."""
    n, m = p + 1, q
    return 16 * ndofs * nvec + ncells * (4 * n ** 3 + 8 * m ** 3 + 48)


def apply_kernel_name(p: int, q: int, precision: str) -> str:
    """The kernel the default launch shape runs (FP64: one-shot while two 8-column FP64
    cell buffers fit 80 KiB of LDS, else persistent)."""
    if precision == "fp32":
        return "apply_vec32_kernel"
    if precision == "bf16":
        return "apply_mixed_kernel"
    return "apply_box_kernel" if (2 * q ** 3 * 8 + q ** 3) * 8 <= 80 * 1024 else "apply_box_pers_kernel"


MAP_KERNEL_SOURCES = ["paper_2208_07129_amd/csrc/apply_box_map.hip"] + KERNEL_SOURCES[1:]


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
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


def traffic_for(wname: str, nvec: int, precision: str, sources=None):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or
    None if they were taken on a different kernel source or workload."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    key = f"{wname}/nvec{nvec}/{precision}"
    rec = t.get(key)
    if not rec or rec.get("kernel_hash") != kernel_hash(sources):
        return None
    return rec.get("bytes_per_launch")


def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline_leg(w, sample_cells: int, sample_cells_1t: int):
    """Time the CPU oracle (as it stands) on a bounded sample of the same workload with all
    BLAS threads and with one thread.  The only place this script times the oracle."""
    from oracle import fe_oracle as fo
    t0 = time.perf_counter()
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    t_setup = time.perf_counter() - t0
    X = w.X()
    out = {}
    for label, ncell, threads in (("all", sample_cells, None), ("one", sample_cells_1t, 1)):
        cells = np.arange(min(ncell, orc.E))
        if threads is None:
            ctx = contextlib.nullcontext()
        else:
            from threadpoolctl import threadpool_limits
            ctx = threadpool_limits(limits=threads)
        with ctx:
            used = _blas_threads()
            t1 = time.perf_counter()
            Ae = orc.element_matrices(cells)
            t_elem = time.perf_counter() - t1
            times = []
            for _ in range(3):
                ta = time.perf_counter()
                orc.apply(X, cells=cells, Ae=Ae)
                times.append(time.perf_counter() - ta)
        t_apply = float(np.median(times))
        owned = cells.size * w.p ** 3 if w.mesh.bc == W.BC_PERIODIC else cells.size * (w.p + 1) ** 3
        out[label] = {"value": owned * w.nvec / t_apply / 1e9, "cores": int(used),
                      "cells": int(cells.size), "apply_s": t_apply, "element_matrices_s": t_elem}
    a = out["all"]
    return {
        "value": a["value"], "unit": UNIT, "cores": a["cores"], "kind": "oracle",
        "sample": (f"cell-matrix apply (numpy/OpenBLAS FP64, element matrices precomputed) of "
                   f"{a['cells']} of {orc.E} cells, all {w.nvec} columns, median of 3; rate counts "
                   f"the dofs the sampled cells own; oracle setup {t_setup:.1f} s"),
        "one_thread": out["one"], "all_threads": a,
        "cpu": _cpu_model(),
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class OracleRows:
    """Sampled output rows of the oracle for one workload (element matrices of the cells
    touching the rows built once), to measure every GPU result's error."""

    def __init__(self, w, nrows: int, seed: int):
        from oracle import fe_oracle as fo
        self.orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
        self.rows = np.sort(np.random.default_rng(seed).choice(self.orc.ndofs, nrows, replace=False))
        self.cells = self.orc.cells_touching(self.rows)
        self.Ae = self.orc.element_matrices(self.cells)

    def ref(self, X):
        return self.orc.apply(X, cells=self.cells, Ae=self.Ae)[self.rows]

    def error(self, Yd, X) -> float:
        """max over columns of the relative 2-norm error on the sampled rows."""
        import torch
        got = Yd[torch.from_numpy(self.rows).to(Yd.device)].cpu().numpy()
        ref = self.ref(X)
        return float((np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())


def timed_applies(op, X, Y, nvec, prec, steps, warmup, stream):
    """`steps` applies bracketed by events on the launch stream, the library's per-apply
    events (zero fill, fused kernel) recorded inside the same timed region.  Returns
    (ms per step, kernel ms samples, zero-fill ms samples)."""
    import torch
    sptr = stream.cuda_stream
    for _ in range(warmup):
        op.apply_ptr(X.data_ptr(), Y.data_ptr(), nvec, nvec, nvec, prec, sptr)
    torch.cuda.synchronize()
    op.timing(steps)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        op.apply_ptr(X.data_ptr(), Y.data_ptr(), nvec, nvec, nvec, prec, sptr)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    z, k = op.timing_samples()
    op.timing(0)
    return ms, k, z


def stats(v) -> dict:
    v = np.asarray(v, dtype=np.float64)
    return {"mean": float(v.mean()), "median": float(np.median(v)), "min": float(v.min()),
            "max": float(v.max()), "n": int(v.size)}


def mixed_leg(op, X, Xh, nvec, steps, warmup, stream, free, rows: OracleRows, base_ms):
    """FP32 / BF16 applies of the headline workload: step and kernel times, speedup over
    the FP64 step, and the error against the oracle on sampled rows."""
    import torch
    from paper_2208_07129_amd import mfmv
    res = {}
    for name in ("fp32", "bf16"):
        prec = mfmv.PRECISIONS[name]
        Yp = torch.empty_like(X)
        ms, k, _z = timed_applies(op, X, Yp, nvec, prec, steps, warmup, stream)
        res[name] = {"ms_per_step": ms, "kernel_ms": stats(k),
                     "value": free * nvec / (ms * 1e-3) / 1e9, "unit": UNIT,
                     "speedup_vs_fp64": base_ms / ms, "rel_err_vs_oracle": rows.error(Yp, Xh)}
        del Yp
    return res


def config3_leg(a) -> dict:
    """The p = 8 workload (periodic unit cube, 12^3 cells, 884,736 dofs) at 16, 64 and 256
    columns in FP64, FP32 and BF16: step time, GDoF·vec/s, speedup over FP64, error
    against the oracle on sampled rows, and the roofline fraction of each."""
    import torch
    from paper_2208_07129_amd import mfmv
    stream = torch.cuda.current_stream()
    out = {}
    rows = None
    for nvec in (16, 64, 256):
        w = W.config3(nvec)
        op = mfmv.Operator.from_workload(w)
        if rows is None:
            rows = OracleRows(w, 12, 303)
        Xh = w.X()
        X = torch.from_numpy(Xh).cuda()
        Y = torch.empty_like(X)
        flops = flops_per_cell_vector(w.p, w.q) * op.ncells * nvec
        nbytes = algorithmic_bytes(op.ndofs, op.ncells, w.p, w.q, nvec)
        res = {}
        for name in ("fp64", "fp32", "bf16"):
            prec = mfmv.PRECISIONS[name]
            ms, k, _z = timed_applies(op, X, Y, nvec, prec, max(10, min(a.steps, 50)), 3, stream)
            km = float(np.mean(k))
            r = {"ms_per_step": ms, "kernel_ms": stats(k),
                 "value": op.ndofs * nvec / (ms * 1e-3) / 1e9,
                 "rel_err_vs_oracle": rows.error(Y, Xh)}
            if name == "fp64":
                r["roofline"] = {"bound": "alu", "achieved": flops / (km * 1e-3) / 1e12,
                                 "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                 "frac": flops / (km * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
            else:
                gbs = nbytes / (km * 1e-3) / 1e9
                r["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}
                r["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / ms
            res[name] = r
        out[f"nvec{nvec}"] = res
        print(json.dumps({f"config3 nvec{nvec}": {k2: (v["ms_per_step"], v["rel_err_vs_oracle"])
                                                  for k2, v in res.items()}}),
              file=sys.stderr, flush=True)
        del X, Y, op
        torch.cuda.empty_cache()
    return {"workload": "periodic-unitcube-12^3-p8q9 (884,736 dofs)", "unit": UNIT, **out}


def solve_leg(a) -> dict:
    """Block-CG solve of (A + sigma M) X = B on the 20^3 periodic p = 6 mesh with 128
    right-hand sides to a true FP64 relative residual of 1e-10 in every column:
    Jacobi with the FP64 apply, Jacobi with the FP32 matrix-core apply inside FP64
    iterative refinement, and the learned cell-local preconditioner (Jacobi fallback)
    with the same mixed apply; network training time reported separately."""
    import torch
    from paper_2208_07129_amd import blockcg, mfmv, mlp
    w = W.config5()
    if a.nvec:
        w.nvec = a.nvec
    op = mfmv.Operator.from_workload(w)
    B = torch.from_numpy(w.X()).cuda()
    diag = mfmv.diagonal(op)
    lam = blockcg.lanczos_extremes(op, steps=a.lanczos_steps)
    out = {"metric": "time to 1e-10 relative residual (block CG, 128 RHS)", "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": w.name, "cells": int(op.ncells), "p": w.p, "q": w.q,
                      "ndofs": int(op.ndofs), "nvec": w.nvec, "sigma": w.sigma},
           "lanczos": lam, "solves": {}}
    jac = blockcg.jacobi_preconditioner(diag)
    runs = [("jacobi_fp64", jac, "fp64", None), ("jacobi_mixed_fp32", jac, "fp32", None)]
    for name, M, prec, fb in runs:
        print(f"solve {name} ...", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        X, st = blockcg.solve(op, B, M, tol=1e-10, maxit=a.solve_maxit, inner_precision=prec,
                              fallback=fb)
        out["solves"][name] = {"seconds": st.seconds, "iterations": st.iterations,
                               "refinements": st.refinements, "converged": bool(st.converged),
                               "rel_residual": st.rel_residual, "breakdown": bool(st.breakdown)}
        print(json.dumps({name: out["solves"][name]}), file=sys.stderr, flush=True)
        del X
    # learned preconditioner: train on operator-generated pairs, judge, solve
    print("training the cell network ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    net = mlp.CellMLP(op, hidden=256, seed=0, dscale=diag)
    losses = mlp.train(net, diag, steps=a.train_steps, k=16, refresh=a.train_refresh)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    floor_status = net.floor_skip()   # the deployed linear preconditioner is SPD
    verdict = mlp.judge(net, diag, k=16)
    fit = mlp.local_fit(net, diag, k=16)
    out["training"] = {"seconds": t_train, "steps": a.train_steps, "loss_first": losses[0],
                       "loss_last": float(np.mean(losses[-10:])), "judge": verdict,
                       "skip_floor_status": floor_status,
                       "local_fit": fit}
    print(json.dumps({"training": out["training"]}), file=sys.stderr, flush=True)
    use_net = bool(verdict["ratio"] < 1.0)
    # the learned preconditioner (measured whatever the judge says), both applies
    for name, prec in (("learned_fp64", "fp64"), ("learned_mixed_fp32", "fp32")):
        print(f"solve {name} ...", file=sys.stderr, flush=True)
        X, st = blockcg.solve(op, B, net.preconditioner(diag), tol=1e-10, maxit=a.solve_maxit,
                              inner_precision=prec, fallback=jac)
        out["solves"][name] = {
            "seconds": st.seconds, "iterations": st.iterations, "refinements": st.refinements,
            "converged": bool(st.converged), "rel_residual": st.rel_residual,
            "breakdown": bool(st.breakdown), "fallback_switches": st.precond_switches}
        print(json.dumps({name: out["solves"][name]}), file=sys.stderr, flush=True)
        del X
    out["judge_deploys_network"] = use_net
    out["deployed_map"] = ("the trained network's symmetric linear part S with its eigenvalue floor "
                           "(ReLU branch and biases not used in the solve)")
    best = min(out["solves"].values(), key=lambda r: r["seconds"] if r["converged"] else 1e30)
    out["value"] = best["seconds"]
    for prec in ("fp64", "mixed_fp32"):
        j, l = out["solves"][f"jacobi_{prec}"], out["solves"][f"learned_{prec}"]
        out[f"learned_vs_jacobi_{prec}"] = {"time_ratio": l["seconds"] / j["seconds"],
                                            "iteration_ratio": l["iterations"] / max(j["iterations"], 1)}
    # FP64 work of one Jacobi block-CG iteration: the apply's algorithmic flops and the
    # six n x k x k block GEMMs (three Gram blocks, three block updates)
    n, k = int(op.ndofs), w.nvec
    it_flops = flops_per_cell_vector(w.p, w.q) * op.ncells * k + 6 * 2 * n * k * k
    j = out["solves"]["jacobi_fp64"]
    achieved = it_flops * j["iterations"] / j["seconds"] / 1e12
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                       "kernel": "Jacobi block-CG iteration (FP64 apply + 6 block GEMMs)",
                       "flops_per_iteration": it_flops,
                       "floor_ms_per_iteration": it_flops / (PEAK_FP64_TFLOPS * 1e12) * 1e3,
                       "ms_per_iteration": j["seconds"] / max(j["iterations"], 1) * 1e3}
    return out


def measured_peaks() -> dict:
    """The machine's rates as measured here, for a second roofline fraction next to
    the spec peaks: FP64 FMA issue rate (mf_fma_probe: independent FMA chains, no
    memory traffic, 32 workgroups of 256 threads per CU) and HBM bandwidth (a 1 GiB
    device-to-device copy, read + write bytes)."""
    import torch
    from paper_2208_07129_amd import mfmv
    out = {}
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks, iters = cus * 32, 4096
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    probe = lambda: mfmv._check(mfmv.lib().mf_fma_probe(blocks, iters, sink.data_ptr(), None))
    probe()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        probe()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    out["fp64_tflops"] = blocks * 256 * iters * 16 / (ms * 1e-3) / 1e12
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    out["hbm_gbs"] = 2 * src.numel() * 8 / (ms * 1e-3) / 1e9
    del src, dst, sink
    return out


def deterministic_leg(op, X, Y, steps: int) -> dict:
    """The colour-ordered assembly (mf_set_deterministic) on the headline workload:
    ms per apply (kernel launches per colour plus the zero fill) and whether
    repeated applies are bitwise equal; the atomic assembly is restored after."""
    import torch
    op.set_deterministic(True)
    try:
        Y2 = torch.empty_like(Y)
        for _ in range(3):
            op.apply(X, Y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(5, min(steps, 50))
        e0.record()
        for _ in range(reps):
            op.apply(X, Y)
        e1.record()
        op.apply(X, Y2)
        torch.cuda.synchronize()
        return {"ms_per_step": e0.elapsed_time(e1) / reps, "bitwise_repeat": bool(torch.equal(Y, Y2))}
    finally:
        op.set_deterministic(False)


def chfsi_leg(a) -> dict:
    """Chebyshev-filtered subspace iteration (Alg. ChFSi) at block scale on the
    config-2 mesh (16^3 cells, p = 6, periodic, 884,736 dofs): a block of
    --chfsi-block vectors (256), the lowest three quarters wanted (a 25% buffer as in
    the paper's runs), degree --chfsi-degree filters, residual tolerance 5e-5.  Every
    step is a library call: fused filter steps, block Gram, the k x k eigen-solver
    (block Jacobi beyond 64), block updates."""
    import torch
    from paper_2208_07129_amd import chebyshev, mfmv
    w = workload("c2", None)
    op = mfmv.Operator.from_workload(w)
    k = a.chfsi_block
    nev = k * 3 // 4
    D = mfmv.gll_mass(op, inv_sqrt=True)
    t_b = time.perf_counter()
    bounds = chebyshev.standard_form_bounds(op, D, steps=a.lanczos_steps)
    t_b = time.perf_counter() - t_b
    si = chebyshev.SubspaceIteration(op, k)
    U0 = torch.from_numpy(np.random.default_rng(78).uniform(-1, 1, (op.ndofs, k))).cuda()
    print(f"chfsi k={k} ...", file=sys.stderr, flush=True)
    res = si.solve(U0, nev=nev, degree=a.chfsi_degree, tol=5e-5, maxit=a.chfsi_maxit,
                   bounds=bounds)
    res["bounds_seconds"] = t_b
    out = {"metric": "ChFSI time to residual 5e-5 (lowest eigenpairs of M^-1/2 A M^-1/2)",
           "unit": "s", "value": res["seconds"], "higher_is_better": False, "n_gpus": 1,
           "data": "synthetic", "dtype": "f64",
           "config": {"workload": w.name, "ndofs": int(op.ndofs), "block": k, "wanted": nev,
                      "degree": a.chfsi_degree},
           **{key: v for key, v in res.items() if key not in ("history", "eigenvalues")},
           "lowest_eigenvalues": res["eigenvalues"][:8], "highest_wanted": res["eigenvalues"][-1],
           "history": [float(h) for h in res["history"]]}
    print(json.dumps({"chfsi": {key: v for key, v in out.items() if key != "history"}}),
          file=sys.stderr, flush=True)
    return out


def chebyshev_leg(a) -> dict:
    """The Chebyshev filter of subspace iteration (Alg. ChFSi) on the standard form
    M^{-1/2} A M^{-1/2} of config 2 (16^3, p = 6, 64 columns): degree-m filters of fused
    steps (mf_cheb_step: a D A (D Y) + b Y + c X in one pass), timed per step."""
    import torch
    from paper_2208_07129_amd import chebyshev, mfmv
    w = workload("c2", a.nvec)
    op = mfmv.Operator.from_workload(w)
    nvec = w.nvec
    U = torch.from_numpy(w.X()).cuda()
    D = mfmv.gll_mass(op, inv_sqrt=True)
    work = (torch.empty_like(U), torch.empty_like(U))
    m = a.cheb_degree
    # spectrum bounds of the standard form: the largest from Lanczos-like growth is not
    # needed for timing; the filter coefficients only set the scalars of each step
    lam_min, lam_max, lam_u = 0.0, 400.0, 4.0
    for _ in range(2):
        chebyshev.chebyshev_filter(op, D, U, m, lam_min, lam_max, lam_u, work=work)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, min(a.steps, 20))
    s0.record()
    for _ in range(reps):
        chebyshev.chebyshev_filter(op, D, U, m, lam_min, lam_max, lam_u, work=work)
    s1.record()
    torch.cuda.synchronize()
    ms_step = s0.elapsed_time(s1) / reps / m
    free = int(op.ndofs)
    flops = flops_per_cell_vector(w.p, w.q) * op.ncells * nvec
    ach = flops / (ms_step * 1e-3) / 1e12
    # the same degree with separate applies and elementwise updates (torch), for scale
    Y = torch.empty_like(U)
    ms_apply = None
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        op.apply(U, Y)
    t1.record()
    torch.cuda.synchronize()
    ms_apply = t0.elapsed_time(t1) / reps
    # Chebyshev-filtered subspace iteration for the lowest eigenpairs of the standard
    # form (Alg. ChFSi): a block of 64 vectors, the 48 lowest wanted (a 25% buffer, as
    # in the paper's runs), to the paper's residual tolerance 5e-5
    si = chebyshev.SubspaceIteration(op, nvec)
    t_b = time.perf_counter()
    bounds = chebyshev.standard_form_bounds(op, D, steps=a.lanczos_steps)
    t_b = time.perf_counter() - t_b
    U0 = torch.from_numpy(np.random.default_rng(77).uniform(-1, 1, (op.ndofs, nvec))).cuda()
    chfsi = si.solve(U0, nev=nvec * 3 // 4, degree=a.chfsi_degree, tol=5e-5,
                     maxit=a.chfsi_maxit, bounds=bounds)
    chfsi["bounds_seconds"] = t_b
    chfsi["degree"] = a.chfsi_degree
    print(json.dumps({"chfsi": {k: v for k, v in chfsi.items() if k != "history"}}),
          file=sys.stderr, flush=True)
    return {"metric": "Chebyshev filter step (fused a D A D Y + b Y + c X) GDoF·vec/s",
            "unit": UNIT, "value": free * nvec / (ms_step * 1e-3) / 1e9, "higher_is_better": True,
            "n_gpus": 1, "data": "synthetic", "dtype": "f64",
            "config": {"workload": w.name, "nvec": nvec, "degree": m},
            "ms_per_step": ms_step, "ms_plain_apply": ms_apply, "chfsi": chfsi,
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "traffic": None,
                         "kernel": "apply_cheb_kernel"}}


def refined_surface_nodes(mesh, p: int, fine: bool) -> int:
    """Lattice nodes on the surface of the refined box (the masters of the hanging-node
    constraints on the coarse lattice, or the hanging nodes on the fine one), without the
    zero-Dirichlet nodes on the outer boundary.  Closed form for a box strictly inside."""
    k = 2 * p if fine else p
    ext = [(mesh.rhi[d] - mesh.rlo[d]) * k + 1 for d in range(3)]
    inner = [max(e - 2, 0) for e in ext]
    return int(np.prod(ext) - np.prod(inner))


def refined_leg(a) -> dict:
    """Hanging-node constraints (Sec. 3.2.2) on the once-refined stand-in mesh (12^3 coarse
    cells, central 6^3 refined, p = 6, zero Dirichlet, 64 columns): one step is
    mf_apply_constrained (C with the zero fill, A_u on the refined map, C^T); the three
    separate calls and each part alone are timed too."""
    import torch
    from paper_2208_07129_amd import mfmv
    w = W.refined_config(a.nvec or 64)
    op = mfmv.RefinedOperator.from_workload(w)
    nvec = w.nvec
    X = torch.from_numpy(w.X(op.ndofs)).cuda()
    Y = torch.empty_like(X)
    for _ in range(max(a.warmup, 2)):
        op.apply_constrained(X, Y)
    torch.cuda.synchronize()
    reps = max(5, min(a.steps, 50))

    def timed(fn):
        for _ in range(5):  # each variant warms up on its own (clocks, caches)
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_three = timed(lambda: op.apply_constrained(X, Y, steps=True))
    ms_step = timed(lambda: op.apply_constrained(X, Y))
    ms_dist = timed(lambda: op.distribute(X))
    ms_cond = timed(lambda: op.condense(Y))
    op.timing(reps)
    ms_apply = timed(lambda: op.apply(X, Y))
    n, z, k = op.timing_read()
    ms_kernel = k / n
    op.timing(reps)
    ms_apply32 = timed(lambda: op.apply(X, Y, precision="fp32"))
    n32, _z32, k32 = op.timing_read()
    flops = flops_per_cell_vector(w.p, w.q) * op.ncells * nvec
    ach = flops / (ms_kernel * 1e-3) / 1e12
    # Chebyshev filter on the constrained space (Alg. ChFSi on D C^T A_u C D): degree-10
    # filters of mf_cheb_step_constrained steps, per step
    from paper_2208_07129_amd import chebyshev
    D = mfmv.gll_mass(op, inv_sqrt=True)
    work = (torch.empty_like(X), torch.empty_like(X))
    U = X.clone()
    cheb_deg = 10
    ms_cheb = timed(lambda: chebyshev.chebyshev_filter(op, D, U, cheb_deg, 0.0, 400.0, 4.0,
                                                       work=work)) / cheb_deg
    nm = refined_surface_nodes(w.mesh, w.p, fine=False)
    ns = op.nslaves
    row = 8 * nvec
    bytes_dist = (nm + ns) * row                 # masters read, slaves written
    bytes_cond = (2 * ns + 2 * nm) * row         # slaves read and cleared, masters updated
    return {"metric": "constrained A·X on a refined mesh (C, A_u, C^T) GDoF·vec/s",
            "unit": UNIT, "value": op.ndofs * nvec / (ms_step * 1e-3) / 1e9,
            "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "f64",
            "config": {"workload": w.name, "nvec": nvec, "ndofs": op.ndofs, "cells": op.ncells,
                       "hanging": ns, "masters": nm, "sets": op.nsets},
            "ms_per_step": ms_step, "ms_three_calls": ms_three, "ms_distribute": ms_dist, "ms_apply": ms_apply,
            "ms_apply_kernel": ms_kernel, "ms_zero_fill": z / n, "ms_condense": ms_cond,
            "ms_apply_fp32": ms_apply32, "ms_apply_kernel_fp32": k32 / n32,
            "ms_cheb_step": ms_cheb,
            "constraints_gbs": {"distribute": bytes_dist / (ms_dist * 1e-3) / 1e9,
                                "condense": bytes_cond / (ms_cond * 1e-3) / 1e9,
                                "peak": PEAK_HBM_GBS},
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                         "traffic": traffic_for(w.name, nvec, "fp64", MAP_KERNEL_SOURCES),
                         "algorithmic_bytes": algorithmic_bytes(op.ndofs, op.ncells, w.p, w.q,
                                                                nvec),
                         "kernel": "apply_box_map_kernel"}}


def batched_leg(a) -> dict:
    """Config 4: 32 uneven periodic meshes (n ~ U{6..16}, p ~ U{4,6,8}, nvec ~
    U{16..128}) applied (a) one mf_apply per operator back to back, (b) as one
    batch (launch shape chosen by the tuner), (c) as a replayed hipGraph of (b);
    aggregate GDoF·vec/s over the batch, FP64 and FP32.  The same for a batch of
    64 small meshes (n ~ U{2..6}, nvec ~ U{4,8,16}), where per-operator launches
    leave most of the GPU idle."""
    import torch
    from paper_2208_07129_amd import mfmv, tune
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream

    def timed(fn, reps, st=None):
        st = st or stream
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(st)
        for _ in range(reps):
            fn()
        s1.record(st)
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / reps

    def run(ws, reps):
        ops = [mfmv.Operator.from_workload(w) for w in ws]
        nvec = [w.nvec for w in ws]
        Xs = [torch.from_numpy(w.X()).cuda() for w in ws]
        Ys = [torch.empty_like(X) for X in Xs]
        work = sum(op.ndofs * k for op, k in zip(ops, nvec))
        flops = sum(flops_per_cell_vector(w.p, w.q) * op.ncells * k
                    for w, op, k in zip(ws, ops, nvec))
        nbytes = sum(algorithmic_bytes(op.ndofs, op.ncells, w.p, w.q, k)
                     for w, op, k in zip(ws, ops, nvec))
        modes = {}
        for prec in ("fp64", "fp32"):
            ms_loop = timed(lambda: [op.apply(X, Y, precision=prec)
                                     for op, X, Y in zip(ops, Xs, Ys)], reps)
            ref = [Y.clone() for Y in Ys]
            b = mfmv.Batch(ops, nvec, prec)
            tuned = tune.tune_batch(b, Xs, Ys, cache=None)
            ms_batch = timed(lambda: b.apply(Xs, Ys), reps)
            err = max(float((torch.linalg.norm(Y - R, dim=0) / torch.linalg.norm(R, dim=0)).max())
                      for Y, R in zip(Ys, ref))
            torch.cuda.synchronize()
            b.capture(Xs, Ys, side)
            ms_graph = timed(lambda: b.replay(side), reps, side)
            modes[prec] = {
                "loop_ms": ms_loop, "batched_ms": ms_batch, "graph_ms": ms_graph,
                "loop_value": work / (ms_loop * 1e-3) / 1e9,
                "batched_value": work / (ms_batch * 1e-3) / 1e9,
                "graph_value": work / (ms_graph * 1e-3) / 1e9,
                "batched_cfg": tuned["cfg"], "rel_diff_batched_vs_loop": err}
            if prec == "fp64":
                ach = flops / (ms_graph * 1e-3) / 1e12
                modes[prec]["roofline"] = {"bound": "alu", "achieved": ach,
                                           "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                           "frac": ach / PEAK_FP64_TFLOPS, "traffic": None,
                                           "kernel": "batched apply (graph replay)"}
            else:
                gbs = nbytes / (ms_graph * 1e-3) / 1e9
                modes[prec]["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                                           "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                                           "traffic": None, "kernel": "batched apply (graph replay)"}
            print(json.dumps({prec: modes[prec]}), file=sys.stderr, flush=True)
            del b
        return work, modes

    reps = max(3, min(a.steps, 20))
    ws = W.config4_meshes(32)
    work, modes = run(ws, reps)
    out = {"metric": "batched A·X aggregate GDoF·vec/s (32 uneven meshes)", "unit": UNIT,
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "config4-32-meshes", "meshes": len(ws),
                      "dofs_x_columns": int(work),
                      "degrees": sorted(set(w.p for w in ws))}, "modes": modes}
    out["value"] = max(m["graph_value"] for m in modes.values())
    out["roofline"] = modes["fp64"]["roofline"]
    ws_small = W.small_meshes(64)
    work_s, modes_s = run(ws_small, max(reps, 20))
    out["small_meshes"] = {"workload": "64 periodic meshes n ~ U{2..6}, p ~ U{4,6,8}, "
                                       "nvec ~ U{4,8,16}", "dofs_x_columns": int(work_s),
                           "modes": modes_s}
    return out


LEGS = ("headline", "mixed", "deterministic", "cpu", "config3", "config4", "config5", "chfsi")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c5"])
    ap.add_argument("--nvec", type=int, default=None)
    ap.add_argument("--legs", default="all",
                    help="comma-separated subset of " + ",".join(LEGS) + " (headline always runs)")
    ap.add_argument("--launch-cfg", type=int, default=None,
                    help="force this launch shape of the FP64 box kernel (default: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-cells", type=int, default=512)
    ap.add_argument("--cpu-sample-cells-1t", type=int, default=64)
    ap.add_argument("--solve", action="store_true",
                    help="only the block-CG solve benchmark on the 20^3 p = 6 mesh (own JSON line)")
    ap.add_argument("--batched", action="store_true",
                    help="only the config-4 batch of 32 uneven meshes: loop vs batched vs graph")
    ap.add_argument("--chebyshev", action="store_true",
                    help="Chebyshev filter steps on the config-2 standard-form operator")
    ap.add_argument("--refined", action="store_true",
                    help="only the hanging-node constrained apply on the refined mesh")
    ap.add_argument("--cheb-degree", type=int, default=10)
    ap.add_argument("--chfsi-maxit", type=int, default=80)
    ap.add_argument("--chfsi-block", type=int, default=256,
                    help="block size of the subspace-iteration leg (wanted: three quarters)")
    ap.add_argument("--chfsi-degree", type=int, default=40)
    ap.add_argument("--solve-maxit", type=int, default=4000)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--train-refresh", type=int, default=25,
                    help="new operator-generated pairs every this many training steps")
    ap.add_argument("--lanczos-steps", type=int, default=120)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of X into Y (known bytes), for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU's partition only; --gpus {a.gpus} is not supported "
              f"(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        return 2
    legs = set(LEGS) if a.legs == "all" else {x.strip() for x in a.legs.split(",") if x.strip()}
    unknown = legs - set(LEGS)
    if unknown:
        raise SystemExit(f"unknown legs {sorted(unknown)}")
    if a.no_cpu_baseline:
        legs.discard("cpu")

    import torch
    from paper_2208_07129_amd import mfmv

    if not torch.cuda.is_available():
        raise SystemExit("no HIP device")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.solve:
        print(json.dumps(solve_leg(a)), flush=True)
        return 0
    if a.batched:
        print(json.dumps(batched_leg(a)), flush=True)
        return 0
    if a.chebyshev:
        print(json.dumps(chebyshev_leg(a)), flush=True)
        return 0
    if a.refined:
        print(json.dumps(refined_leg(a)), flush=True)
        return 0
    w = workload(a.workload, a.nvec)
    prec = mfmv.PRECISIONS[a.precision]
    op = mfmv.Operator.from_workload(w)
    if a.launch_cfg is not None:
        op.set_launch(False, a.launch_cfg)
    nvec = w.nvec
    Xh = w.X()
    X = torch.from_numpy(Xh).to(dev)
    Y = torch.empty_like(X)
    free = int(op.ndofs - mfmv.constrained_mask(w.mesh, w.p).sum())
    stream = torch.cuda.current_stream()
    if a.calibrate_copy:
        # an elementwise kernel over many workgroups (reads X once, writes Y once)
        for _ in range(a.steps):
            torch.mul(X, 1.0, out=Y)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": X.numel() * 8,
                          "calibrate_copy_bytes_written": Y.numel() * 8, "steps": a.steps}))
        return 0

    ms_per_step, ksamp, zsamp = timed_applies(op, X, Y, nvec, prec, a.steps, a.warmup, stream)
    value = free * nvec / (ms_per_step * 1e-3) / 1e9
    kern_ms = float(np.mean(ksamp))
    print(f"headline: {ms_per_step:.4f} ms per step, kernel mean {kern_ms:.4f} ms",
          file=sys.stderr, flush=True)

    flops = flops_per_cell_vector(w.p, w.q) * op.ncells * nvec
    achieved = flops / (kern_ms * 1e-3) / 1e12
    executed = executed_flops_per_cell_vector(w.p, w.q, box=True) * op.ncells * nvec
    traffic = traffic_for(w.name, nvec, a.precision)
    kname = apply_kernel_name(w.p, w.q, a.precision)
    nbytes = algorithmic_bytes(op.ndofs, op.ncells, w.p, w.q, nvec)
    peaks = measured_peaks()
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    if a.precision == "fp64" and flops / nbytes >= ridge:
        # FP64 at nvec >= 8: 18 algorithmic flop/B > the 9.8 flop/B ridge, bound by the FP64 units
        roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                    "peak_measured": peaks["fp64_tflops"],
                    "frac_measured": achieved / peaks["fp64_tflops"],
                    "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                    "kernel": kname, "kernel_ms": kern_ms,
                    "kernel_ms_median": float(np.median(ksamp)),
                    "flops_per_launch": flops,
                    "flops_basis": "algorithmic (sum-factorised count per cell and column)",
                    "executed_flops_per_launch": executed,
                    "executed_frac": executed / (kern_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                    "algorithmic_bytes_per_launch": nbytes,
                    "hbm_frac_of_algorithmic_bytes": nbytes / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    else:
        # FP32 / BF16 arithmetic with FP64 X and Y (below the FP32 ridge), or FP64 at one or
        # two columns (below the FP64 ridge): bound by HBM
        gbs = nbytes / (kern_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": gbs / PEAK_HBM_GBS, "peak_measured": peaks["hbm_gbs"],
                    "frac_measured": gbs / peaks["hbm_gbs"], "traffic": traffic, "kernel": kname,
                    "kernel_ms": kern_ms, "kernel_ms_median": float(np.median(ksamp)),
                    "bytes_per_launch": nbytes, "flops_per_launch": flops}
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[a.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "cells": int(op.ncells), "p": w.p, "q": w.q,
                   "ndofs": int(op.ndofs), "free_dofs": free, "nvec": nvec,
                   "precision": a.precision, "layout": "dof-major, columns contiguous"},
        "roofline": roofline,
        "kernel_ms": stats(ksamp), "zero_fill_ms": stats(zsamp),
    }
    rows = OracleRows(w, 32, 12345)
    out["rel_err_vs_oracle_sampled"] = rows.error(Y, Xh)
    out["oracle_rows_sampled"] = int(rows.rows.size)
    if "deterministic" in legs and a.precision == "fp64" and w.mesh.lin is None:
        out["deterministic_assembly"] = deterministic_leg(op, X, Y, a.steps)
    if "mixed" in legs and a.precision == "fp64":
        out["mixed"] = mixed_leg(op, X, Xh, nvec, a.steps, a.warmup, stream, free, rows,
                                 ms_per_step)
        print(json.dumps({"mixed": out["mixed"]}), file=sys.stderr, flush=True)
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline_leg(w, a.cpu_sample_cells, a.cpu_sample_cells_1t)
        print(json.dumps({"cpu_baseline": out["cpu_baseline"]}), file=sys.stderr, flush=True)
    del X, Y, op
    torch.cuda.empty_cache()
    if "config3" in legs:
        out["config3"] = config3_leg(a)
    if "config4" in legs:
        out["config4"] = batched_leg(a)
        torch.cuda.empty_cache()
    if "config5" in legs:
        out["config5"] = solve_leg(a)
        torch.cuda.empty_cache()
    if "chfsi" in legs:
        out["chfsi"] = chfsi_leg(a)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
