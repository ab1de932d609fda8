"""Learned cell-local preconditioner for block CG (state, training and
inference; every step runs in the library's kernels, include/mfmlp.h).

    z = D^{-1} r + sum_e Q_e^T W_e rho_e f_theta(Q_e r / rho_e)

f_theta: F = np^3 -> 256 -> 256 -> F, ReLU, BF16 weights on the matrix cores
with FP32 master weights and Adam.  The network learns the correction to the
Jacobi step: from pairs (R = A E, E) that the operator generates, the target
of cell e and column j is (E - D^{-1} R) restricted to the cell and scaled by
the same 1 / rho as the input, so a network that has learnt nothing (f = 0)
leaves plain Jacobi.  Rows of a batch are (cell, column) pairs; activations
are stored feature-major (features x rows).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import mfmv
from .mfmv import _check, _stream_ptr, lib


def _ceil8(n: int) -> int:
    return (n + 7) // 8 * 8


def _host_bf16(a: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (int16) of FP32 values, round to nearest even."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return u.view(np.int16)


@dataclass
class TrainLog:
    steps: int = 0
    loss: List[float] = None
    seconds: float = 0.0


class CellMLP:
    """The network and its optimizer state for one operator (cell size np^3)."""

    def __init__(self, op: mfmv.Operator, hidden: int = 256, seed: int = 0, out_scale: float = 0.0):
        import torch
        self.op = op
        self.F = (op.p + 1) ** 3
        self.Fp = _ceil8(self.F)
        self.H = hidden
        if hidden % 8:
            raise ValueError("hidden width must be a multiple of 8")
        rng = np.random.default_rng(seed)
        F, Fp, H = self.F, self.Fp, self.H
        W1 = np.zeros((H, Fp), np.float32)
        W1[:, :F] = rng.standard_normal((H, F)) * math.sqrt(2.0 / F)
        W2 = (rng.standard_normal((H, H)) * math.sqrt(2.0 / H)).astype(np.float32)
        W3 = np.zeros((Fp, H), np.float32)
        W3[:F] = rng.standard_normal((F, H)) * out_scale * math.sqrt(1.0 / H)
        host = [W1, np.zeros(H, np.float32), W2, np.zeros(H, np.float32), W3,
                np.zeros(Fp, np.float32)]
        dev = torch.device("cuda")
        self.params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in host]
        self.grads = [torch.empty_like(p) for p in self.params]
        self.m1 = [torch.zeros_like(p) for p in self.params]
        self.m2 = [torch.zeros_like(p) for p in self.params]
        self.wbf = {i: torch.from_numpy(_host_bf16(host[i])).to(dev) for i in (0, 2, 4)}
        self.step = 0
        self._buf: Dict[str, object] = {}
        self._loss = torch.zeros(1, dtype=torch.float64, device=dev)

    # ------------------------------------------------------------ buffers
    def _buffers(self, k: int):
        """Activation blocks for ncells * k rows, stored with the row count padded
        to a multiple of 8 (padding columns stay zero in inputs, targets and
        output gradients, so they add nothing to the gradients)."""
        import torch
        rows = self.op.ncells * k
        if self._buf.get("rows") != rows:
            dev = torch.device("cuda")
            Fp, H, ld = self.Fp, self.H, _ceil8(rows)
            i16, f32 = torch.int16, torch.float32
            self._buf = dict(
                rows=rows, ld=ld,
                X0=torch.zeros(Fp, ld, dtype=i16, device=dev),
                H1=torch.zeros(H, ld, dtype=i16, device=dev),
                H2=torch.zeros(H, ld, dtype=i16, device=dev),
                Y=torch.zeros(Fp, ld, dtype=f32, device=dev),
                T=torch.zeros(Fp, ld, dtype=f32, device=dev),
                dY=torch.zeros(Fp, ld, dtype=i16, device=dev),
                dH2=torch.zeros(H, ld, dtype=i16, device=dev),
                dH1=torch.zeros(H, ld, dtype=i16, device=dev),
                rho=torch.zeros(ld, dtype=f32, device=dev),
            )
        return self._buf

    # ------------------------------------------------------------ kernels
    @staticmethod
    def _gemm(M, N, K, ta, tb, A, lda, B, ldb, kchunk=0, bias=None, relu=False, mask=None,
              ldmask=0, out_f32=None, ld_f32=0, atomic=False, out_bf16=None, ld_bf16=0):
        ptr = (lambda t: None if t is None else t.data_ptr())
        _check(lib().mf_mlp_gemm(M, N, K, int(ta), int(tb), A.data_ptr(), lda, B.data_ptr(), ldb,
                                 kchunk, ptr(bias), int(relu), ptr(mask), ldmask, ptr(out_f32),
                                 ld_f32, int(atomic), ptr(out_bf16), ld_bf16, _stream_ptr(None)))

    def gather(self, R, E=None):
        """Network inputs (and targets) of every (cell, column) of R (and E)."""
        b = self._buffers(R.shape[1])
        k = R.shape[1]
        _check(lib().mf_cell_gather(self.op._h, k, R.data_ptr(), R.stride(0),
                                    None if E is None else E.data_ptr(),
                                    0 if E is None else E.stride(0), self.Fp, b["X0"].data_ptr(),
                                    None if E is None else b["T"].data_ptr(), b["ld"],
                                    b["rho"].data_ptr(), _stream_ptr(None)))
        return b

    def forward(self, b):
        n, Fp, H = b["ld"], self.Fp, self.H
        W1, b1, W2, b2, W3, b3 = self.params
        self._gemm(H, n, Fp, False, False, self.wbf[0], Fp, b["X0"], n, bias=b1, relu=True,
                   out_bf16=b["H1"], ld_bf16=n)
        self._gemm(H, n, H, False, False, self.wbf[2], H, b["H1"], n, bias=b2, relu=True,
                   out_bf16=b["H2"], ld_bf16=n)
        self._gemm(Fp, n, H, False, False, self.wbf[4], H, b["H2"], n, bias=b3,
                   out_f32=b["Y"], ld_f32=n)
        return b["Y"]

    def backward(self, b, kchunk: int = 8192):
        """Gradients of the last loss_grad (dY in b['dY']) into self.grads."""
        n, Fp, H = b["ld"], self.Fp, self.H
        gW1, gb1, gW2, gb2, gW3, gb3 = self.grads
        s = _stream_ptr(None)
        for g in (gW1, gW2, gW3):
            _check(lib().mf_fill_f32(g.numel(), g.data_ptr(), 0.0, s))
        # layer 3
        self._gemm(Fp, H, n, False, True, b["dY"], n, b["H2"], n, kchunk=kchunk,
                   out_f32=gW3, ld_f32=H, atomic=True)
        _check(lib().mf_row_sums(Fp, n, b["dY"].data_ptr(), n, gb3.data_ptr(), 0, s))
        self._gemm(H, n, Fp, True, False, self.wbf[4], H, b["dY"], n, mask=b["H2"],
                   ldmask=n, out_bf16=b["dH2"], ld_bf16=n)
        # layer 2
        self._gemm(H, H, n, False, True, b["dH2"], n, b["H1"], n, kchunk=kchunk,
                   out_f32=gW2, ld_f32=H, atomic=True)
        _check(lib().mf_row_sums(H, n, b["dH2"].data_ptr(), n, gb2.data_ptr(), 0, s))
        self._gemm(H, n, H, True, False, self.wbf[2], H, b["dH2"], n, mask=b["H1"],
                   ldmask=n, out_bf16=b["dH1"], ld_bf16=n)
        # layer 1
        self._gemm(H, Fp, n, False, True, b["dH1"], n, b["X0"], n, kchunk=kchunk,
                   out_f32=gW1, ld_f32=Fp, atomic=True)
        _check(lib().mf_row_sums(H, n, b["dH1"].data_ptr(), n, gb1.data_ptr(), 0, s))

    def loss_grad(self, b) -> None:
        _check(lib().mf_mse_grad(self.F, self.Fp, b["rows"], b["Y"].data_ptr(), b["T"].data_ptr(),
                                 b["ld"], b["dY"].data_ptr(), self._loss.data_ptr(),
                                 _stream_ptr(None)))

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        for i, (w, g, m1, m2) in enumerate(zip(self.params, self.grads, self.m1, self.m2)):
            wbf = self.wbf.get(i)
            _check(lib().mf_adam(w.numel(), w.data_ptr(), g.data_ptr(), m1.data_ptr(),
                                 m2.data_ptr(), None if wbf is None else wbf.data_ptr(),
                                 ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2),
                                 ctypes.c_float(eps), self.step, _stream_ptr(None)))

    def train_step(self, R, T_err, lr: float) -> float:
        """One Adam step on the pairs (R, T_err) (T_err: the error to predict, in
        the Jacobi-correction form E - D^{-1} R); returns the loss before the step."""
        b = self.gather(R, T_err)
        self.forward(b)
        self._loss.zero_()
        self.loss_grad(b)
        self.backward(b)
        self.adam(lr)
        return float(self._loss.item())

    def precondition(self, R, Z, diag) -> None:
        """Z := D^{-1} R + sum_e Q_e^T W_e rho f(Q_e R / rho)."""
        b = self.gather(R)
        self.forward(b)
        _check(lib().mf_cell_scatter(self.op._h, R.shape[1], b["Y"].data_ptr(), b["ld"],
                                     b["rho"].data_ptr(), diag.data_ptr(), R.data_ptr(),
                                     R.stride(0), Z.data_ptr(), Z.stride(0), _stream_ptr(None)))

    def preconditioner(self, diag):
        def M(R, Z):
            self.precondition(R, Z, diag)
            return Z
        return M


# ---------------------------------------------------------------- training data
def make_pairs(op: mfmv.Operator, diag, k: int, seed: int, smooth_steps: int, omega: float = 0.6):
    """(R, T) with E random U[-1, 1] columns smoothed by `smooth_steps` damped
    Jacobi sweeps on the error (e <- e - omega D^{-1} A e), R = A E and the
    Jacobi-correction target T = E - D^{-1} R.  All steps are library calls."""
    import torch
    rng = np.random.default_rng(seed)
    E = torch.from_numpy(rng.uniform(-1.0, 1.0, (op.ndofs, k))).cuda()
    AE = torch.empty_like(E)
    for _ in range(smooth_steps):
        op.apply(E, AE)
        mfmv.jacobi(diag, AE, AE)
        mfmv.axpby(-omega, AE, 1.0, E)
    R = torch.empty_like(E)
    op.apply(E, R)
    T = torch.empty_like(E)
    mfmv.jacobi(diag, R, T)
    mfmv.axpby(1.0, E, -1.0, T)   # T = E - D^{-1} R
    return R, T, E


def train(net: CellMLP, diag, steps: int, k: int = 16, lr: float = 1e-3, seed: int = 0,
          smooth=(0, 1, 2, 4, 8), refresh: int = 10, log: Optional[list] = None) -> list:
    """Adam on fresh operator-generated pairs (a new pair block every `refresh`
    steps, cycling through the smoothing depths)."""
    losses = [] if log is None else log
    pairs = None
    for s in range(steps):
        if s % refresh == 0:
            depth = smooth[(s // refresh) % len(smooth)]
            pairs = make_pairs(net.op, diag, k, seed * 100003 + s, depth)
        R, T, _ = pairs
        losses.append(net.train_step(R, T, lr))
    return losses


def a_norm_error(op: mfmv.Operator, E, Z):
    """Per column ||E - Z||_A^2 (FP64 apply and library dot products)."""
    import torch
    D = torch.empty_like(E)
    mfmv.axpby(1.0, E, 0.0, D)
    mfmv.axpby(-1.0, Z, 1.0, D)
    AD = torch.empty_like(D)
    op.apply(D, AD)
    return mfmv.col_dots(D, AD).cpu().numpy()


def judge(net: CellMLP, diag, k: int = 16, seed: int = 12345, depths=(0, 2, 8)) -> dict:
    """Held-out check of the learned step against the Jacobi step: the A-norm
    of the error left by one application, z = M(r) for r = A e, averaged over
    columns and smoothing depths.  ratio < 1: the network improves on Jacobi."""
    import torch
    num, den = 0.0, 0.0
    for i, d in enumerate(depths):
        R, _, E = make_pairs(net.op, diag, k, seed + i, d)
        Zl = torch.empty_like(R)
        net.precondition(R, Zl, diag)
        Zj = torch.empty_like(R)
        mfmv.jacobi(diag, R, Zj)
        # best scalar multiple of each step (CG rescales directions anyway)
        for Z, acc in ((Zl, "l"), (Zj, "j")):
            AZ = torch.empty_like(Z)
            net.op.apply(Z, AZ)
            zaz = mfmv.col_dots(Z, AZ).cpu().numpy()
            zae = mfmv.col_dots(AZ, E).cpu().numpy()
            AE = torch.empty_like(E)
            net.op.apply(E, AE)
            eae = mfmv.col_dots(E, AE).cpu().numpy()
            left = np.mean(1.0 - zae ** 2 / np.maximum(zaz * eae, 1e-300))
            if acc == "l":
                num += left
            else:
                den += left
    return {"learned": num / len(depths), "jacobi": den / len(depths),
            "ratio": num / max(den, 1e-300)}
