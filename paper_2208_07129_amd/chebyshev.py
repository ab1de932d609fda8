"""Chebyshev filter of subspace iteration (Alg. ChFSi) on the standard form
H~ = M^{-1/2} H M^{-1/2} of the eigenproblem H U = M U Lambda (eq. ghep,
eq. shep), M the GLL-lumped diagonal mass.

Every step of the filter is one fused library call (mf_cheb_step); this module
only sequences them with the scalar recurrence of the scaled Chebyshev
polynomial.  The orthogonalisation and Rayleigh-Ritz steps of subspace
iteration are not part of this module.
"""
from __future__ import annotations

from . import mfmv


def filter_coefficients(m: int, lam_min: float, lam_max: float, lam_u: float):
    """The (a, b, c) of each of the m steps of the filter, step d computing
    X_d = a H~ X_{d-1} + b X_{d-1} + c X_{d-2} (X_0 the input, c = 0 at d = 1):
    the scaled Chebyshev polynomial of degree m that damps [lam_u, lam_max] and
    is normalised to 1 at lam_min."""
    if m < 1:
        raise ValueError("m >= 1")
    e = (lam_max - lam_u) / 2.0
    c = (lam_max + lam_u) / 2.0
    sigma = e / (lam_min - c)
    gamma = 2.0 / sigma
    a1 = sigma / e
    steps = [(a1, -c * a1, 0.0)]
    for _ in range(2, m + 1):
        sigma2 = 1.0 / (gamma - sigma)
        a1 = 2.0 * sigma2 / e
        steps.append((a1, -c * a1, -sigma * sigma2))
        sigma = sigma2
    return steps


def chebyshev_filter(op: mfmv.Operator, D, U, m: int, lam_min: float, lam_max: float,
                     lam_u: float, work=None, stream=None):
    """p_m(H~) U with D = M^{-1/2} (mfmv.gll_mass(op, inv_sqrt=True)).  U is not
    modified; `work` (two tensors shaped like U) may be given to avoid allocation.
    Returns the tensor holding the result (one of the work tensors)."""
    import torch
    X, Y = work if work is not None else (torch.empty_like(U), torch.empty_like(U))
    steps = filter_coefficients(m, lam_min, lam_max, lam_u)
    a, b, _c = steps[0]
    mfmv.cheb_step(op, D, U, None, Y, a, b, 0.0, stream)     # Y = a1 H~ U + a1 a2 U
    prev, cur = U, Y
    for a, b, c in steps[1:]:
        # X <- a H~ Y + b Y + c X, written over the older iterate (in place once X is
        # a work tensor; the first time it starts from U, which is left unmodified)
        out = X if prev is U else prev
        mfmv.cheb_step(op, D, cur, prev, out, a, b, c, stream)
        prev, cur = cur, out
    return cur


# ------------------------------------------------------ subspace iteration
def standard_form_bounds(op: mfmv.Operator, D, steps: int = 60, seed: int = 0) -> tuple:
    """(lower, upper) bounds of the spectrum of H~ = D A D from Lanczos Ritz values:
    the upper one padded by the last Ritz residual scale (the filter must damp the
    whole unwanted interval up to the true largest eigenvalue)."""
    from .blockcg import lanczos_extremes
    lam = lanczos_extremes(op, steps=steps, seed=seed,
                           matvec=lambda v, w: mfmv.cheb_step(op, D, v, None, w, 1.0, 0.0, 0.0))
    span = lam["lambda_max"] - lam["lambda_min"]
    return lam["lambda_min"], lam["lambda_max"] + 0.01 * span


class SubspaceIteration:
    """Chebyshev-filtered subspace iteration (Alg. ChFSi) for the lowest
    eigenpairs of H~ = M^{-1/2} A M^{-1/2} (eq. shep) on a block of k <= 2048
    vectors: filter, orthonormalise (Gram block, its eigen-decomposition,
    X V diag(w)^{-1/2}), Rayleigh-Ritz (projected block, its eigen-decomposition,
    rotation), residual norms.  Every step is a library call; the host reads
    back only the Ritz values and residual norms that steer the iteration."""

    def __init__(self, op: mfmv.Operator, k: int):
        import torch
        self.op, self.k = op, k
        n = op.ndofs
        self.D = mfmv.gll_mass(op, inv_sqrt=True)
        mk = lambda: torch.empty((n, k), dtype=torch.float64, device="cuda")
        self.U, self.X, self.Y, self.Xo, self.HX, self.HU = (mk() for _ in range(6))
        mk2 = lambda: torch.empty((k, k), dtype=torch.float64, device="cuda")
        self.G, self.M, self.Hp, self.Q = (mk2() for _ in range(4))
        self.w = torch.empty(k, dtype=torch.float64, device="cuda")
        self.theta = torch.empty(k, dtype=torch.float64, device="cuda")
        self.st = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.rn2 = torch.empty(k, dtype=torch.float64, device="cuda")
        self.gwork = mfmv.block_gram_work(n, k)
        self.ework = mfmv.sym_eig_work(k)

    def rayleigh_ritz(self, B) -> tuple:
        """U, HU := the Ritz vectors of span(B) and H~ U; returns (Ritz values,
        residual norms ||H~ u_j - theta_j u_j||) as host arrays.  The norms come
        from ||H~ u_j||^2 - theta_j^2 (u_j orthonormal, theta_j = u_j^T H~ u_j), which
        resolves them down to about 1e-8 |theta_j|."""
        import numpy as np
        op, D = self.op, self.D
        mfmv.block_gram(B, B, self.G, work=self.gwork)                 # B^T B
        mfmv.sym_eig(self.G, self.w, self.M, self.st, vpow=-0.5,
                     work=self.ework)                                   # V diag(w)^{-1/2}
        if int(self.st.item()) != 0:
            raise RuntimeError("the filtered block lost rank (Gram block not positive definite)")
        mfmv.block_update(B, self.M, self.Xo, 1.0, 0.0)                 # orthonormal basis
        mfmv.cheb_step(op, D, self.Xo, None, self.HX, 1.0, 0.0, 0.0)   # H~ Xo
        mfmv.block_gram(self.Xo, self.HX, self.Hp, work=self.gwork)     # Xo^T H~ Xo
        mfmv.sym_eig(self.Hp, self.theta, self.Q, self.st, work=self.ework)
        mfmv.block_update(self.Xo, self.Q, self.U, 1.0, 0.0)
        mfmv.block_update(self.HX, self.Q, self.HU, 1.0, 0.0)
        th = self.theta.cpu().numpy()
        hn2 = mfmv.col_norms2(self.HU, self.rn2).cpu().numpy()
        res = np.sqrt(np.maximum(hn2 - th * th, 0.0))
        return th, res

    def solve(self, U0, nev: int, degree: int, tol: float, maxit: int, bounds=None) -> dict:
        """Iterate from the block U0 until the nev lowest residual norms are <= tol
        (or maxit filter passes).  bounds: (lower, upper) of the spectrum of H~, from
        Lanczos when None."""
        import time
        import torch
        t0 = time.perf_counter()
        lo, hi = bounds if bounds is not None else standard_form_bounds(self.op, self.D)
        th, res = self.rayleigh_ritz(U0)
        hist = [float(res[:nev].max())]
        it = 0
        t_filter = t_rr = 0.0
        while hist[-1] > tol and it < maxit:
            t1 = time.perf_counter()
            Yf = chebyshev_filter(self.op, self.D, self.U, degree, min(lo, th[0]), hi, th[-1],
                                  work=(self.X, self.Y))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            th, res = self.rayleigh_ritz(Yf)   # ends with a read-back
            t_rr += time.perf_counter() - t2
            t_filter += t2 - t1
            hist.append(float(res[:nev].max()))
            it += 1
        return {"eigenvalues": th[:nev].tolist(), "residual": hist[-1], "iterations": it,
                "converged": bool(hist[-1] <= tol), "history": hist,
                "seconds": time.perf_counter() - t0, "filter_seconds": t_filter,
                "rayleigh_ritz_seconds": t_rr, "bounds": [lo, hi]}
