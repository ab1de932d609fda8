"""ctypes binding of libmfmv.so (argument marshalling only).

Every step of the product runs in the library's HIP kernels.  PyTorch is used
for device memory and streams: tensors are passed by ``data_ptr()`` and the
stream by ``torch.cuda.current_stream().cuda_stream``.  There is no fallback:
if the library is missing, or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfmv.so")

MF_OK, MF_ERR_ARG, MF_ERR_UNSUPPORTED, MF_ERR_OOM, MF_ERR_HIP = 0, -1, -2, -3, -4
MF_BC_NONE, MF_BC_DIRICHLET0, MF_BC_PERIODIC = 0, 1, 2
MF_FP64, MF_FP32, MF_BF16 = 0, 1, 2
MF_FP32_MFMA, MF_BF16_MFMA = MF_FP32, MF_BF16  # names of the original interface description
PRECISIONS = {"fp64": MF_FP64, "fp32": MF_FP32, "bf16": MF_BF16}
BOX_CFGS, MIXED_CFGS, BATCH_CFGS = 13, 7, 6
BOX_MFMA_CFGS = (10,)  # FP64 matrix-core shape (q = p + 1 <= 8)
MIXED_MFMA_CFGS = 4  # mixed shapes 0..3 are matrix-core kernels; 4..6 are FP32 vector kernels

# Every symbol declared in include/mfmv.h.
EXPORTS = ("mf_num_dofs", "mf_num_cells", "mf_quad_points", "mf_constrained_mask", "mf_basis_1d",
           "mf_create_operator", "mf_destroy_operator", "mf_operator_info", "mf_cell_order",
           "mf_apply",
           "mf_apply_add", "mf_zero", "mf_set_launch", "mf_set_launch_mixed", "mf_timing",
           "mf_timing_read", "mf_timing_samples", "mf_batch_create", "mf_batch_destroy", "mf_batch_set_launch",
           "mf_batch_apply", "mf_batch_capture", "mf_batch_replay", "mf_batch_info",
           "mf_tune", "mf_tune_info", "mf_set_deterministic", "mf_fma_probe", "mf_batch_tune", "mf_apply_batched",
           "mf_last_error",
           # include/mfsolve.h
           "mf_diagonal", "mf_block_gram", "mf_block_gram_noalloc", "mf_block_gram_work",
           "mf_block_gram2", "mf_block_gram2_work", "mf_block_update", "mf_block_update_norms",
           "mf_block_update_norms_work", "mf_col_dots",
           "mf_axpby",
           "mf_jacobi", "mf_spd_solve",
           # include/mfmlp.h
           "mf_mlp_gemm", "mf_cell_gather", "mf_cell_scatter", "mf_mse_grad", "mf_row_sums",
           "mf_adam", "mf_symmetrize", "mf_to_bf16", "mf_fill_f32", "mf_skip_floor",
           "mf_skip_floor_work",
           # include/mfcheb.h
           "mf_gll_mass", "mf_cheb_step", "mf_sym_eig", "mf_sym_eig_work",
           # include/mfrefine.h
           "mf_refined_sizes", "mf_refined_layout", "mf_refined_quad_points",
           "mf_create_refined_operator", "mf_apply_constrained", "mf_cheb_step_constrained",
           "mf_constraints_distribute", "mf_constraints_condense")


class MfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libmfmv status {status}: {msg}")
        self.status = status


class MeshC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", ctypes.c_int32), ("lin", ctypes.c_double * 9)]


class RefinedMeshC(ctypes.Structure):
    _fields_ = [("coarse", MeshC), ("rlo", ctypes.c_int32 * 3), ("rhi", ctypes.c_int32 * 3)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_07129_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        F32 = ctypes.c_float
        MP = ctypes.POINTER(MeshC)
        RP = ctypes.POINTER(RefinedMeshC)
        sig = {
            "mf_num_dofs": (I, [MP, I, ctypes.POINTER(I64)]),
            "mf_num_cells": (I, [MP, ctypes.POINTER(I64)]),
            "mf_quad_points": (I, [MP, I, P]),
            "mf_constrained_mask": (I, [MP, I, P]),
            "mf_basis_1d": (I, [I, I, P, P, P, P, P, P]),
            "mf_create_operator": (I, [MP, I, I, D, P, D, ctypes.POINTER(P)]),
            "mf_destroy_operator": (None, [P]),
            "mf_operator_info": (I, [P, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                     ctypes.POINTER(I), ctypes.POINTER(I)]),
            "mf_cell_order": (I, [P, P]),
            "mf_set_deterministic": (I, [P, I]),
            "mf_fma_probe": (I, [I, I64, P, P]),
            "mf_apply": (I, [P, P, P, I, I64, I64, I, P]),
            "mf_apply_add": (I, [P, P, P, I, I64, I64, I, P]),
            "mf_zero": (I, [P, I64, I, I64, P]),
            "mf_set_launch": (I, [P, I, I]),
            "mf_set_launch_mixed": (I, [P, I]),
            "mf_timing": (I, [P, I]),
            "mf_timing_read": (I, [P, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D)]),
            "mf_timing_samples": (I, [P, I, P, P, ctypes.POINTER(I)]),
            "mf_last_error": (ctypes.c_char_p, []),
            "mf_batch_create": (I, [I, P, P, I, ctypes.POINTER(P)]),
            "mf_batch_destroy": (None, [P]),
            "mf_batch_set_launch": (I, [P, I]),
            "mf_batch_apply": (I, [P, P, P, P, P, P]),
            "mf_batch_capture": (I, [P, P, P, P, P, P]),
            "mf_batch_replay": (I, [P, P]),
            "mf_batch_info": (I, [P, ctypes.POINTER(I64), ctypes.POINTER(I), ctypes.POINTER(I)]),
            "mf_tune": (I, [P, I, I, ctypes.c_char_p]),
            "mf_tune_info": (I, [P, I, I, ctypes.POINTER(I), P, I]),
            "mf_batch_tune": (I, [P, P, P, P, P, ctypes.c_char_p, P]),
            "mf_apply_batched": (I, [I, P, P, P, P, I, P]),
            "mf_diagonal": (I, [P, P, P]),
            "mf_block_gram": (I, [I64, I, P, I64, P, I64, D, D, P, I, P, I64, P]),
            "mf_block_gram_work": (I64, [I64, I]),
            "mf_block_gram_noalloc": (I, [I64, I, P, I64, P, I64, D, D, P, I, P]),
            "mf_block_update": (I, [I64, I, I, D, P, I64, P, I, D, P, I64, P]),
            "mf_block_gram2": (I, [I64, I, P, I64, P, I64, P, I64, D, D, P, I, P, I, P, I64, P]),
            "mf_block_gram2_work": (I64, [I64, I]),
            "mf_block_update_norms": (I, [I64, I, I, D, P, I64, P, I, D, P, I64, P, P, I64, P]),
            "mf_block_update_norms_work": (I64, [I64, I]),
            "mf_col_dots": (I, [I64, I, P, I64, P, I64, P, P]),
            "mf_axpby": (I, [I64, I, D, P, I64, D, P, I64, P]),
            "mf_jacobi": (I, [I64, I, P, P, I64, P, I64, P]),
            "mf_spd_solve": (I, [I, I, P, P, P, P, P]),
            "mf_mlp_gemm": (I, [I, I, I, I, I, P, I64, P, I64, I, P, I, P, I64, P, I64, I, P, I64,
                                I, P]),
            "mf_cell_gather": (I, [P, I, P, I64, P, I64, I, P, P, I64, P, I, P, I, P]),
            "mf_cell_scatter": (I, [P, I, P, I64, P, P, P, I64, P, I64, I, P, I, P]),
            "mf_symmetrize": (I, [I, P, I64, P, P]),
            "mf_skip_floor": (I, [I, P, I64, P, I64, D, P, I64, P, P]),
            "mf_skip_floor_work": (I64, [I]),
            "mf_mse_grad": (I, [I, I, I64, P, P, I64, P, F32, P, P, P]),
            "mf_row_sums": (I, [I, I64, P, I64, P, I, P]),
            "mf_adam": (I, [I64, P, P, P, P, P, F32, F32, F32, F32, I, P]),
            "mf_to_bf16": (I, [I64, P, P, P]),
            "mf_fill_f32": (I, [I64, P, F32, P]),
            "mf_gll_mass": (I, [P, I, P, P]),
            "mf_cheb_step": (I, [P, P, P, P, P, I, I64, D, D, D, P]),
            "mf_sym_eig": (I, [I, P, I64, P, P, I64, D, P, P, I64, P]),
            "mf_sym_eig_work": (I64, [I]),
            "mf_refined_sizes": (I, [RP, I, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                     ctypes.POINTER(I64), ctypes.POINTER(I64)]),
            "mf_refined_layout": (I, [RP, I, P, P]),
            "mf_refined_quad_points": (I, [RP, I, P]),
            "mf_create_refined_operator": (I, [RP, I, I, D, P, D, ctypes.POINTER(P)]),
            "mf_apply_constrained": (I, [P, P, P, I, I64, I64, P]),
            "mf_cheb_step_constrained": (I, [P, P, P, P, P, I, I64, D, D, D, P, P]),
            "mf_constraints_distribute": (I, [P, P, I, I64, P]),
            "mf_constraints_condense": (I, [P, P, I, I64, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != MF_OK:
        raise MfError(status, lib().mf_last_error().decode())


def mesh_c(mesh) -> MeshC:
    """Convert a workloads.BoxMesh (or any object with n, lo, hi, bc, lin) to the C struct."""
    m = MeshC()
    for d in range(3):
        m.n[d] = int(mesh.n[d])
        m.lo[d] = float(mesh.lo[d])
        m.hi[d] = float(mesh.hi[d])
    m.bc = int(mesh.bc)
    lin = getattr(mesh, "lin", None)
    if lin is not None:
        flat = np.asarray(lin, dtype=np.float64).reshape(9)
        for k in range(9):
            m.lin[k] = float(flat[k])
    return m


def num_dofs(mesh, p: int) -> int:
    out = ctypes.c_int64()
    _check(lib().mf_num_dofs(ctypes.byref(mesh_c(mesh)), p, ctypes.byref(out)))
    return out.value


def num_cells(mesh) -> int:
    out = ctypes.c_int64()
    _check(lib().mf_num_cells(ctypes.byref(mesh_c(mesh)), ctypes.byref(out)))
    return out.value


def quad_points(mesh, q: int) -> np.ndarray:
    E = num_cells(mesh)
    xq = np.empty((E, q ** 3, 3), dtype=np.float64)
    _check(lib().mf_quad_points(ctypes.byref(mesh_c(mesh)), q, xq.ctypes.data))
    return xq


def constrained_mask(mesh, p: int) -> np.ndarray:
    m = np.empty(num_dofs(mesh, p), dtype=np.uint8)
    _check(lib().mf_constrained_mask(ctypes.byref(mesh_c(mesh)), p, m.ctypes.data))
    return m.astype(bool)


def basis_1d(p: int, q: int) -> dict:
    np1 = p + 1
    out = {"xq": np.empty(q), "wq": np.empty(q), "xn": np.empty(np1), "N": np.empty((q, np1)),
           "D": np.empty((q, np1)), "Dt": np.empty((q, q))}
    _check(lib().mf_basis_1d(p, q, *(out[k].ctypes.data for k in ("xq", "wq", "xn", "N", "D", "Dt"))))
    return out


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Operator:
    """A = mu K + M_{V+sigma} on the current HIP device (owns its device data)."""

    def __init__(self, mesh, p: int, q: int, mu: float = 0.5, Vq: Optional[np.ndarray] = None,
                 sigma: float = 0.0):
        self._h = ctypes.c_void_p()
        self.mesh, self.p, self.q, self.mu, self.sigma = mesh, p, q, mu, sigma
        vptr = None
        if Vq is not None:
            self._vq = np.ascontiguousarray(Vq, dtype=np.float64).reshape(-1)
            if self._vq.size != num_cells(mesh) * q ** 3:
                raise ValueError("Vq must hold E*q^3 values")
            vptr = self._vq.ctypes.data
        _check(lib().mf_create_operator(ctypes.byref(mesh_c(mesh)), p, q, float(mu), vptr,
                                        float(sigma), ctypes.byref(self._h)))
        nd, nc = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().mf_operator_info(self._h, ctypes.byref(nd), ctypes.byref(nc), None, None))
        self.ndofs, self.ncells = nd.value, nc.value

    def constrained_rows(self) -> np.ndarray:
        """Rows that carry no unknown (zero-Dirichlet), as a boolean host array."""
        return constrained_mask(self.mesh, self.p).astype(bool)

    @classmethod
    def from_workload(cls, w):
        """Build the operator of a workloads.Workload, tabulating V at the library's points."""
        Vq = w.V(quad_points(w.mesh, w.q)) if w.V is not None else None
        return cls(w.mesh, w.p, w.q, w.mu, Vq, w.sigma)

    def close(self):
        if self._h:
            lib().mf_destroy_operator(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_ptr(self, X_ptr: int, Y_ptr: int, nvec: int, ldx: int, ldy: int,
                  prec: int = MF_FP64, stream=None):
        _check(lib().mf_apply(self._h, X_ptr, Y_ptr, nvec, ldx, ldy, prec, _stream_ptr(stream)))

    def cell_order(self) -> np.ndarray:
        """The order in which the fused apply takes the cells (see mf_cell_order)."""
        out = np.empty(self.ncells, dtype=np.int32)
        _check(lib().mf_cell_order(self._h, out.ctypes.data))
        return out

    def set_deterministic(self, on: bool = True):
        """Colour-ordered assembly: bitwise reproducible applies (mf_set_deterministic)."""
        _check(lib().mf_set_deterministic(self._h, int(bool(on))))

    def set_launch(self, general: bool = False, cfg: int = -1):
        _check(lib().mf_set_launch(self._h, int(general), int(cfg)))

    def tune(self, nvec: int, precision: str = "fp64", cache_path: Optional[str] = None) -> dict:
        """Time the launch shapes for nvec columns and keep the fastest (mf_tune); returns
        {"cfg": chosen shape, "ms": {shape: median ms}} (empty when taken from the cache)."""
        prec = PRECISIONS[precision]
        _check(lib().mf_tune(self._h, int(nvec), prec, cache_path.encode() if cache_path else None))
        cfg = ctypes.c_int()
        ms = (ctypes.c_double * 16)()
        _check(lib().mf_tune_info(self._h, int(nvec), prec, ctypes.byref(cfg), ms, 16))
        return {"cfg": cfg.value, "ms": {str(i): ms[i] for i in range(16) if ms[i] >= 0}}

    def set_launch_mixed(self, cfg: int = -1):
        _check(lib().mf_set_launch_mixed(self._h, int(cfg)))

    def timing(self, slots: int):
        _check(lib().mf_timing(self._h, int(slots)))

    def timing_read(self):
        """(count, zero-fill ms summed, fused-kernel ms summed) since the last read."""
        n, z, k = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(lib().mf_timing_read(self._h, ctypes.byref(n), ctypes.byref(z), ctypes.byref(k)))
        return n.value, z.value, k.value

    def timing_samples(self, cap: int = 100000):
        """Per-apply (zero-fill ms, fused-kernel ms) arrays since the last read, oldest first."""
        z, k = np.empty(cap), np.empty(cap)
        n = ctypes.c_int()
        _check(lib().mf_timing_samples(self._h, cap, z.ctypes.data, k.ctypes.data, ctypes.byref(n)))
        return z[:n.value].copy(), k[:n.value].copy()

    def apply_add_ptr(self, X_ptr: int, Y_ptr: int, nvec: int, ldx: int, ldy: int,
                      prec: int = MF_FP64, stream=None):
        _check(lib().mf_apply_add(self._h, X_ptr, Y_ptr, nvec, ldx, ldy, prec, _stream_ptr(stream)))

    def apply(self, X, Y=None, precision: str = "fp64", stream=None, accumulate: bool = False):
        """Y := A X for torch float64 device tensors of shape (ndofs, nvec) (row stride >= nvec)."""
        import torch
        if X.dtype != torch.float64 or not X.is_cuda:
            raise TypeError("X must be a float64 device tensor")
        # the column stride of a single column is immaterial
        if X.dim() != 2 or X.shape[0] != self.ndofs or (X.shape[1] > 1 and X.stride(1) != 1):
            raise ValueError("X must be (ndofs, nvec) with unit column stride")
        nvec = X.shape[1]
        if Y is None:
            Y = torch.empty(X.shape, dtype=X.dtype, device=X.device)
        if Y.dtype != torch.float64 or Y.shape != X.shape or (nvec > 1 and Y.stride(1) != 1):
            raise ValueError("Y must match X")
        ldx = X.stride(0) if nvec > 1 or X.shape[0] <= 1 else max(X.stride(0), 1)
        ldy = Y.stride(0) if nvec > 1 or Y.shape[0] <= 1 else max(Y.stride(0), 1)
        fn = self.apply_add_ptr if accumulate else self.apply_ptr
        fn(X.data_ptr(), Y.data_ptr(), nvec, max(ldx, nvec), max(ldy, nvec), PRECISIONS[precision],
           stream)
        return Y


# ----------------------------------------------------------- include/mfrefine.h
def refined_mesh_c(rmesh) -> RefinedMeshC:
    """Convert a workloads.RefinedMesh (n, lo, hi, bc, lin, rlo, rhi) to the C struct."""
    m = RefinedMeshC()
    m.coarse = mesh_c(rmesh)
    for d in range(3):
        m.rlo[d] = int(rmesh.rlo[d])
        m.rhi[d] = int(rmesh.rhi[d])
    return m


def refined_sizes(rmesh, p: int) -> dict:
    """Nodes, cells, hanging nodes and constraint sets of a refined mesh of degree p."""
    v = [ctypes.c_int64() for _ in range(4)]
    _check(lib().mf_refined_sizes(ctypes.byref(refined_mesh_c(rmesh)), p, *map(ctypes.byref, v)))
    return dict(zip(("ndofs", "ncells", "nslaves", "nsets"), (x.value for x in v)))


def refined_layout(rmesh, p: int):
    """(cell-to-node map E x (p+1)^3, node kinds: 0 free, 1 zero-Dirichlet, 2 hanging)."""
    sz = refined_sizes(rmesh, p)
    cmap = np.empty((sz["ncells"], (p + 1) ** 3), dtype=np.int32)
    kind = np.empty(sz["ndofs"], dtype=np.uint8)
    _check(lib().mf_refined_layout(ctypes.byref(refined_mesh_c(rmesh)), p, cmap.ctypes.data,
                                   kind.ctypes.data))
    return cmap, kind


def refined_quad_points(rmesh, q: int) -> np.ndarray:
    ncells = refined_sizes(rmesh, 1)["ncells"]
    out = np.empty((ncells, q ** 3, 3))
    _check(lib().mf_refined_quad_points(ctypes.byref(refined_mesh_c(rmesh)), q, out.ctypes.data))
    return out


class RefinedOperator(Operator):
    """A = mu K + M_{V+sigma} on a once-refined box with hanging-node constraints: ``apply``
    is A_u (hanging rows as ordinary rows); ``distribute`` / ``condense`` are C and C^T;
    ``apply_constrained`` runs the three in order."""

    def __init__(self, rmesh, p: int, q: int, mu: float = 0.5, Vq: Optional[np.ndarray] = None,
                 sigma: float = 0.0):
        self._h = ctypes.c_void_p()
        self.mesh, self.p, self.q, self.mu, self.sigma = rmesh, p, q, mu, sigma
        sz = refined_sizes(rmesh, p)
        self.nslaves, self.nsets = sz["nslaves"], sz["nsets"]
        vptr = None
        if Vq is not None:
            self._vq = np.ascontiguousarray(Vq, dtype=np.float64).reshape(-1)
            if self._vq.size != sz["ncells"] * q ** 3:
                raise ValueError("Vq must hold E*q^3 values")
            vptr = self._vq.ctypes.data
        _check(lib().mf_create_refined_operator(ctypes.byref(refined_mesh_c(rmesh)), p, q,
                                                float(mu), vptr, float(sigma),
                                                ctypes.byref(self._h)))
        self.ndofs, self.ncells = sz["ndofs"], sz["ncells"]

    def constrained_rows(self) -> np.ndarray:
        """Rows that carry no unknown (zero-Dirichlet and hanging), as a boolean host array."""
        return refined_layout(self.mesh, self.p)[1] != 0

    @classmethod
    def from_workload(cls, w):
        Vq = w.V(refined_quad_points(w.mesh, w.q)) if w.V is not None else None
        return cls(w.mesh, w.p, w.q, w.mu, Vq, w.sigma)

    def _ptr(self, V, name):
        ptr, n, k, ld = _mv(V, name)
        if n != self.ndofs:
            raise ValueError(f"{name} must have ndofs rows")
        return ptr, k, ld

    def distribute(self, X, stream=None):
        """C: hanging rows of X := W_I X_M, in place."""
        ptr, k, ld = self._ptr(X, "X")
        _check(lib().mf_constraints_distribute(self._h, ptr, k, ld, _stream_ptr(stream)))
        return X

    def condense(self, Y, stream=None):
        """C^T: Y_M += W_I^T Y_S, Y_S := 0, in place."""
        ptr, k, ld = self._ptr(Y, "Y")
        _check(lib().mf_constraints_condense(self._h, ptr, k, ld, _stream_ptr(stream)))
        return Y

    def apply_constrained(self, X, Y=None, stream=None, steps: bool = False):
        """Y := C^T A_u C X (mf_apply_constrained); the hanging rows of X are overwritten by
        C X.  steps=True issues the three calls (C, A_u, C^T) separately instead."""
        import torch
        if steps:
            self.distribute(X, stream)
            Y = self.apply(X, Y, stream=stream)
            return self.condense(Y, stream)
        xp, k, ldx = self._ptr(X, "X")
        if Y is None:
            Y = torch.empty((self.ndofs, k), dtype=torch.float64, device=X.device)
        yp, ky, ldy = self._ptr(Y, "Y")
        if ky != k:
            raise ValueError("Y must have as many columns as X")
        _check(lib().mf_apply_constrained(self._h, xp, yp, k, ldx, ldy, _stream_ptr(stream)))
        return Y


def zero_ptr(Y_ptr: int, nrows: int, ncols: int, ld: int, stream=None):
    _check(lib().mf_zero(Y_ptr, nrows, ncols, ld, _stream_ptr(stream)))


# ------------------------------------------------------------ include/mfsolve.h
def _mv(V, name):
    """(pointer, rows, cols, ld) of a float64 device matrix with unit column stride."""
    import torch
    if V.dtype != torch.float64 or not V.is_cuda or V.dim() != 2:
        raise ValueError(f"{name} must be a 2-D float64 device tensor")
    n, k = V.shape
    if n > 0 and k > 1 and V.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    ld = V.stride(0) if n > 1 else k
    return V.data_ptr(), n, k, max(ld, k)


def diagonal(op: Operator, out=None, stream=None):
    """Operator diagonal (constrained rows 1) as a float64 device vector."""
    import torch
    if out is None:
        out = torch.empty(op.ndofs, dtype=torch.float64, device="cuda")
    _check(lib().mf_diagonal(op._h, out.data_ptr(), _stream_ptr(stream)))
    return out


def gll_mass(op: Operator, inv_sqrt: bool = False, out=None, stream=None):
    """GLL-lumped mass diagonal (or its inverse square root; 0 on constrained rows) as a
    float64 device vector."""
    import torch
    if out is None:
        out = torch.empty(op.ndofs, dtype=torch.float64, device="cuda")
    _check(lib().mf_gll_mass(op._h, int(bool(inv_sqrt)), out.data_ptr(), _stream_ptr(stream)))
    return out


def cheb_step(op: Operator, D, Y, Xp, Out, a: float, b: float, c: float, stream=None):
    """Out := a D A (D Y) + b Y + c Xp (Xp may be None or Out itself); returns Out."""
    py, n, k, ld = _mv(Y, "Y")
    po, no, ko, ldo = _mv(Out, "Out")
    if (no, ko, ldo) != (n, k, ld):
        raise ValueError("Y and Out must have the same shape and row stride")
    px = 0
    if Xp is not None:
        px, nx, kx, ldx = _mv(Xp, "Xp")
        if (nx, kx, ldx) != (n, k, ld):
            raise ValueError("Xp must have the shape and row stride of Y")
    if isinstance(op, RefinedOperator):
        # the constrained space: row scaling, mf_apply_constrained, combine (workspace cached)
        import torch
        work = getattr(op, "_cheb_work", None)
        if work is None or work.numel() < 2 * n * k:
            work = op._cheb_work = torch.empty(2 * n * k, dtype=torch.float64, device=Y.device)
        _check(lib().mf_cheb_step_constrained(op._h, D.data_ptr(), py, px or None, po, k, ld,
                                              float(a), float(b), float(c), work.data_ptr(),
                                              _stream_ptr(stream)))
        return Out
    _check(lib().mf_cheb_step(op._h, D.data_ptr(), py, px or None, po, k, ld, float(a), float(b),
                              float(c), _stream_ptr(stream)))
    return Out


def sym_eig_work(k: int, device="cuda"):
    """A work array for sym_eig on k x k blocks (None when k <= 64 needs none)."""
    import torch
    n = int(lib().mf_sym_eig_work(k))
    if n < 0:
        raise ValueError(f"sym_eig takes 1 <= k <= 2048, got {k}")
    return None if n == 0 else torch.empty(n, dtype=torch.float64, device=device)


def sym_eig(A, w=None, V=None, status=None, vpow: float = 0.0, work=None, stream=None):
    """(w ascending, V columns scaled by w^vpow, status) of a symmetric k x k float64
    device block (k <= 2048; k > 64 takes a work array, allocated here if not given)."""
    import torch
    pa, k, k2, lda = _mv(A, "A")
    if k != k2:
        raise ValueError("A must be square")
    if w is None:
        w = torch.empty(k, dtype=torch.float64, device=A.device)
    if V is None:
        V = torch.empty(k, k, dtype=torch.float64, device=A.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
    if work is None and k > 64 and 0 < k <= 2048:
        work = sym_eig_work(k, A.device)
    _check(lib().mf_sym_eig(k, pa, lda, w.data_ptr(), V.data_ptr(), V.stride(0), float(vpow),
                            status.data_ptr(), None if work is None else work.data_ptr(),
                            0 if work is None else work.numel(), _stream_ptr(stream)))
    return w, V, status


def block_gram_work(n: int, k: int, device="cuda"):
    """A work array for block_gram on n x k multivectors."""
    import torch
    return torch.empty(max(1, lib().mf_block_gram_work(n, k)), dtype=torch.float64, device=device)


def block_gram(A, B, C=None, alpha: float = 1.0, beta: float = 0.0, work=None, stream=None):
    """C := alpha A^T B + beta C (k x k); `work` from block_gram_work (allocated
    here when not given)."""
    import torch
    pa, n, k, lda = _mv(A, "A")
    pb, nb, kb, ldb = _mv(B, "B")
    if (nb, kb) != (n, k):
        raise ValueError("A and B must have the same shape")
    if C is None:
        C = torch.empty(k, k, dtype=torch.float64, device=A.device)
    pc, kc, kc2, ldc = _mv(C, "C")
    if (kc, kc2) != (k, k):
        raise ValueError("C must be k x k")
    if work is None:
        work = block_gram_work(n, k, A.device)
    _check(lib().mf_block_gram(n, k, pa, lda, pb, ldb, float(alpha), float(beta), pc, ldc,
                               work.data_ptr(), work.numel(), _stream_ptr(stream)))
    return C


def block_update(P, M, Y, alpha: float = 1.0, beta: float = 1.0, stream=None):
    """Y := beta Y + alpha P M."""
    pp, n, kp, ldp = _mv(P, "P")
    pm, km, k, ldm = _mv(M, "M")
    py, ny, ky, ldy = _mv(Y, "Y")
    if km != kp or ny != n or ky != k:
        raise ValueError("shape mismatch in block_update")
    _check(lib().mf_block_update(n, k, kp, float(alpha), pp, ldp, pm, ldm, float(beta), py, ldy,
                                 _stream_ptr(stream)))
    return Y


def block_gram2_work(n: int, k: int, device="cuda"):
    """A work array for block_gram2 on n x k multivectors."""
    import torch
    return torch.empty(max(1, lib().mf_block_gram2_work(n, k)), dtype=torch.float64, device=device)


def block_gram2(A, B1, B2, C1=None, C2=None, alpha: float = 1.0, beta: float = 0.0, work=None,
                stream=None):
    """(C1, C2) := (alpha A^T B1 + beta C1, alpha A^T B2 + beta C2) in one pass over A;
    `work` from block_gram2_work (allocated here when not given)."""
    import torch
    pa, n, k, lda = _mv(A, "A")
    pb1, n1, k1, ldb1 = _mv(B1, "B1")
    pb2, n2, k2, ldb2 = _mv(B2, "B2")
    if (n1, k1) != (n, k) or (n2, k2) != (n, k):
        raise ValueError("A, B1 and B2 must have the same shape")
    if C1 is None:
        C1 = torch.empty(k, k, dtype=torch.float64, device=A.device)
    if C2 is None:
        C2 = torch.empty(k, k, dtype=torch.float64, device=A.device)
    pc1, r1, c1, ldc1 = _mv(C1, "C1")
    pc2, r2, c2, ldc2 = _mv(C2, "C2")
    if (r1, c1) != (k, k) or (r2, c2) != (k, k):
        raise ValueError("C1 and C2 must be k x k")
    if work is None:
        work = block_gram2_work(n, k, A.device)
    _check(lib().mf_block_gram2(n, k, pa, lda, pb1, ldb1, pb2, ldb2, float(alpha), float(beta),
                                pc1, ldc1, pc2, ldc2, work.data_ptr(), work.numel(),
                                _stream_ptr(stream)))
    return C1, C2


def block_update_norms_work(n: int, k: int, device="cuda"):
    """A work array for block_update_norms on n x k multivectors."""
    import torch
    return torch.empty(max(1, lib().mf_block_update_norms_work(n, k)), dtype=torch.float64,
                       device=device)


def block_update_norms(P, M, Y, norms2=None, alpha: float = 1.0, beta: float = 1.0, work=None,
                       stream=None):
    """Y := beta Y + alpha P M and norms2[j] := ||Y[:, j]||^2 of the new Y (k, kp <= 128)."""
    import torch
    pp, n, kp, ldp = _mv(P, "P")
    pm, km, k, ldm = _mv(M, "M")
    py, ny, ky, ldy = _mv(Y, "Y")
    if km != kp or ny != n or ky != k:
        raise ValueError("shape mismatch in block_update_norms")
    if norms2 is None:
        norms2 = torch.empty(k, dtype=torch.float64, device=Y.device)
    if norms2.numel() != k or norms2.dtype != torch.float64:
        raise ValueError("norms2 must hold k float64 values")
    if work is None:
        work = block_update_norms_work(n, k, Y.device)
    _check(lib().mf_block_update_norms(n, k, kp, float(alpha), pp, ldp, pm, ldm, float(beta), py,
                                       ldy, norms2.data_ptr(), work.data_ptr(), work.numel(),
                                       _stream_ptr(stream)))
    return Y, norms2


def col_dots(A, B, out=None, stream=None):
    """out[j] = sum_i A[i, j] B[i, j]."""
    import torch
    pa, n, k, lda = _mv(A, "A")
    pb, nb, kb, ldb = _mv(B, "B")
    if (nb, kb) != (n, k):
        raise ValueError("A and B must have the same shape")
    if out is None:
        out = torch.empty(k, dtype=torch.float64, device=A.device)
    _check(lib().mf_col_dots(n, k, pa, lda, pb, ldb, out.data_ptr(), _stream_ptr(stream)))
    return out


def col_norms2(V, out=None, stream=None):
    return col_dots(V, V, out, stream)


def axpby(a: float, X, b: float, Y, stream=None):
    """Y := a X + b Y (b = 0: Y only written)."""
    px, n, k, ldx = _mv(X, "X")
    py, ny, ky, ldy = _mv(Y, "Y")
    if (ny, ky) != (n, k):
        raise ValueError("X and Y must have the same shape")
    _check(lib().mf_axpby(n, k, float(a), px, ldx, float(b), py, ldy, _stream_ptr(stream)))
    return Y


def jacobi(diag, R, Z=None, stream=None):
    """Z := R / diag row-wise."""
    import torch
    pr, n, k, ldr = _mv(R, "R")
    if Z is None:
        Z = torch.empty_like(R)
    pz, nz, kz, ldz = _mv(Z, "Z")
    if (nz, kz) != (n, k) or diag.numel() != n:
        raise ValueError("shape mismatch in jacobi")
    _check(lib().mf_jacobi(n, k, diag.data_ptr(), pr, ldr, pz, ldz, _stream_ptr(stream)))
    return Z


def spd_solve(G, S, X=None, status=None, stream=None):
    """X := G^{-1} S (Cholesky); returns (X, status) with status a device int32 (0 = ok)."""
    import torch
    pg, k, k2, ldg = _mv(G, "G")
    ps, ks, m, lds = _mv(S, "S")
    if k2 != k or ks != k or ldg != k or lds != m:
        raise ValueError("G must be k x k and S k x m, both contiguous")
    if X is None:
        X = torch.empty_like(S)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=G.device)
    _check(lib().mf_spd_solve(k, m, pg, ps, X.data_ptr(), status.data_ptr(), _stream_ptr(stream)))
    return X, status


class Batch:
    """Y_i := A_i X_i for a list of operators in one persistent launch (see mf_batch_*)."""

    def __init__(self, ops: Sequence[Operator], nvec: Sequence[int], precision: str = "fp64"):
        self._h = ctypes.c_void_p()
        self.ops = list(ops)
        self.nvec = [int(v) for v in nvec]
        n = len(self.ops)
        handles = (ctypes.c_void_p * n)(*[o._h.value for o in self.ops])
        nv = (ctypes.c_int * n)(*self.nvec)
        _check(lib().mf_batch_create(n, handles, nv, PRECISIONS[precision], ctypes.byref(self._h)))
        self._keep = (handles, nv)

    def close(self):
        if self._h:
            lib().mf_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, cfg: int):
        _check(lib().mf_batch_set_launch(self._h, int(cfg)))

    def info(self):
        items, cfg, grid = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        _check(lib().mf_batch_info(self._h, ctypes.byref(items), ctypes.byref(cfg), ctypes.byref(grid)))
        return {"items": items.value, "cfg": cfg.value, "grid": grid.value}

    def _arrays(self, Xs, Ys):
        n = len(self.ops)
        if len(Xs) != n or len(Ys) != n:
            raise ValueError("one X and one Y per operator")
        for X, Y, op, nv in zip(Xs, Ys, self.ops, self.nvec):
            if X.shape != (op.ndofs, nv) or Y.shape != (op.ndofs, nv) or X.stride(1) != 1 or Y.stride(1) != 1:
                raise ValueError("X_i, Y_i must be (ndofs_i, nvec_i) with unit column stride")
        xp = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
        yp = (ctypes.c_void_p * n)(*[Y.data_ptr() for Y in Ys])
        lx = (ctypes.c_int64 * n)(*[X.stride(0) for X in Xs])
        ly = (ctypes.c_int64 * n)(*[Y.stride(0) for Y in Ys])
        return xp, yp, lx, ly

    def apply(self, Xs, Ys, stream=None):
        xp, yp, lx, ly = self._arrays(Xs, Ys)
        _check(lib().mf_batch_apply(self._h, xp, yp, lx, ly, _stream_ptr(stream)))

    def capture(self, Xs, Ys, stream):
        xp, yp, lx, ly = self._arrays(Xs, Ys)
        _check(lib().mf_batch_capture(self._h, xp, yp, lx, ly, _stream_ptr(stream)))

    def replay(self, stream=None):
        _check(lib().mf_batch_replay(self._h, _stream_ptr(stream)))

    def tune(self, Xs, Ys, cache_path: Optional[str] = None, stream=None):
        """Time every launch shape on these buffers and keep the fastest (mf_batch_tune)."""
        xp, yp, lx, ly = self._arrays(Xs, Ys)
        _check(lib().mf_batch_tune(self._h, xp, yp, lx, ly,
                                   cache_path.encode() if cache_path else None, _stream_ptr(stream)))
        return self.info()["cfg"]


def apply_batched(ops: Sequence[Operator], Xs, Ys, precision: str = "fp64", stream=None):
    """Y_i := A_i X_i in one call (mf_apply_batched; ld = nvec_i, contiguous tensors)."""
    n = len(ops)
    if len(Xs) != n or len(Ys) != n:
        raise ValueError("one X and one Y per operator")
    for X, Y, op in zip(Xs, Ys, ops):
        if X.dim() != 2 or X.shape != Y.shape or X.shape[0] != op.ndofs or not X.is_contiguous() \
                or not Y.is_contiguous():
            raise ValueError("X_i, Y_i must be contiguous (ndofs_i, nvec_i)")
    handles = (ctypes.c_void_p * n)(*[o._h.value for o in ops])
    xp = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
    yp = (ctypes.c_void_p * n)(*[Y.data_ptr() for Y in Ys])
    nv = (ctypes.c_int * n)(*[int(X.shape[1]) for X in Xs])
    _check(lib().mf_apply_batched(n, handles, xp, yp, nv, PRECISIONS[precision], _stream_ptr(stream)))
