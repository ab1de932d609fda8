"""Build libmfmv.so in-tree with hipcc for gfx950.

    python -m paper_2208_07129_amd.build [-j N]

Objects go to ``_build/`` at the repository root; the shared library is
written next to this file.  Every HIP source is compiled with the packed-FP32
VALU forms switched off, and FP64 atomics compile to the hardware add.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libmfmv.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
MAX_P = 10

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
          f"-I{os.path.join(ROOT, 'include')}"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def jobs():
    """(source, object, extra flags) for every translation unit."""
    out = [
        ("capi.cpp", "capi.o", []),
        ("capi_batch.cpp", "capi_batch.o", []),
        ("capi_tune.cpp", "capi_tune.o", []),
        ("host_setup.cpp", "host_setup.o", []),
        ("dispatch.hip", "dispatch.o", []),
        ("solver.hip", "solver.o", []),
        ("blas64.hip", "blas64.o", []),
        ("eig.hip", "eig.o", []),
        ("capi_solver.cpp", "capi_solver.o", []),
        ("mlp.hip", "mlp.o", []),
        ("capi_mlp.cpp", "capi_mlp.o", []),
        ("capi_cheb.cpp", "capi_cheb.o", []),
        ("refine.cpp", "refine.o", []),
        ("constraints.hip", "constraints.o", []),
    ]
    for p in range(1, MAX_P + 1):
        out.append(("apply_f64.hip", f"apply_f64_p{p}.o", [f"-DMF_P={p}"]))
        out.append(("apply_box.hip", f"apply_box_p{p}.o", [f"-DMF_P={p}"]))
        if p <= 7:
            out.append(("apply_mfma.hip", f"apply_mfma_p{p}.o", [f"-DMF_P={p}"]))
        out.append(("apply_mixed.hip", f"apply_mixed_p{p}.o", [f"-DMF_P={p}"]))
        out.append(("apply_cheb.hip", f"apply_cheb_p{p}.o", [f"-DMF_P={p}"]))
        out.append(("apply_box_map.hip", f"apply_box_map_p{p}.o", [f"-DMF_P={p}"]))
    for prec in range(3):
        for cfg in range(3):
            out.append(("apply_batched.hip", f"apply_batched_{prec}_{cfg}.o",
                        [f"-DMF_BPREC={prec}", f"-DMF_BCFG={cfg}"]))
    return out


def _newest_input(src):
    """Modification time of the newest of the source and every header it may include."""
    t = os.path.getmtime(os.path.join(CSRC, src))
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in os.listdir(d):
            if f.endswith(".h"):
                t = max(t, os.path.getmtime(os.path.join(d, f)))
    return t


def _compile(cc, src, obj, extra, incremental=False):
    out = os.path.join(BUILD, obj)
    if incremental and os.path.exists(out) and os.path.getmtime(out) >= _newest_input(src):
        return obj
    cmd = [cc, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(nproc: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit and link.  incremental=True (a developer
    option) skips objects newer than their source and every header."""
    cc = hipcc()
    os.makedirs(BUILD, exist_ok=True)
    nproc = nproc or min(8, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=nproc) as ex:
        futs = [ex.submit(_compile, cc, s, o, e, incremental) for s, o, e in jobs()]
        for f in futs:
            objs.append(f.result())
            if verbose:
                print("compiled", objs[-1], flush=True)
    tmp = OUT + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[os.path.join(BUILD, o) for o in objs]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only objects older than their source or a header")
    a = ap.parse_args(argv)
    print(build(a.j, a.v, a.incremental))


if __name__ == "__main__":
    sys.exit(main())
