"""Block conjugate gradients for A X = B with k right-hand sides (multivectors
in the library's dof-major layout), built from the C-ABI calls of
include/mfsolve.h and the operator apply; this module only sequences them.

Iteration (flexible block PCG, one previous direction block kept):
    Q = A P,  G = P^T Q,  alpha = G^{-1} P^T R
    X += P alpha,  R -= Q alpha
    Z = M(R),  beta = -G^{-1} Q^T Z,  P <- Z + P beta
With a fixed symmetric preconditioner this is block PCG (O'Leary); the
A-orthogonalisation of Z against the last block keeps it a descent method for
a preconditioner that changes between applications (the learned one).

Mixed precision: `solve` wraps the inner iteration in FP64 iterative
refinement: R = B - A X with the FP64 apply, inner solve of A D = R with the
FP32/BF16 matrix-core apply to a loose tolerance, X += D, until the true
relative residual of every column is below the target.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import mfmv


def _col_norms_host(V, floor: bool = True) -> np.ndarray:
    """Column 2-norms (library kernel), copied to the host; zero norms -> 1."""
    nrm = np.sqrt(mfmv.col_norms2(V).cpu().numpy())
    return np.where(nrm > 0, nrm, 1.0) if floor else nrm


@dataclass
class SolveStats:
    iterations: int = 0                 # inner block iterations, all refinement steps
    refinements: int = 0                # FP64 outer steps
    converged: bool = False
    rel_residual: float = math.inf      # max over columns, true FP64 residual
    history: List[float] = field(default_factory=list)  # max column residual per iteration
    seconds: float = 0.0
    breakdown: bool = False
    precond_switches: int = 0           # learned -> Jacobi fallbacks


def jacobi_preconditioner(diag) -> Callable:
    def M(R, Z):
        return mfmv.jacobi(diag, R, Z)
    return M


def block_pcg(op: mfmv.Operator, B, X, precond: Callable, tol: float, maxit: int,
              precision: str = "fp64", stats: Optional[SolveStats] = None,
              fallback: Optional[Callable] = None, check_every: int = 1):
    """Improve X in place towards A X = B until every column's recursive residual
    ||R_j|| <= tol ||B_j||; returns (X, iterations, converged, breakdown).

    `precond(R, Z)` writes M(R) into Z.  If `fallback` is given, the iteration
    switches to it (restarting the direction block) when the preconditioned
    direction is not a descent direction for some column (p_j^T r_j <= 0).
    """
    import torch
    n, k = B.shape
    dev = B.device
    R = torch.empty_like(B)
    op.apply(X, R, precision=precision)
    mfmv.axpby(1.0, B, -1.0, R)          # R = B - A X (recursive residual from here on)
    bn = _col_norms_host(B)
    Z = torch.empty_like(B)
    P = torch.empty_like(B)
    Q = torch.empty_like(B)
    G = torch.empty(k, k, dtype=torch.float64, device=dev)
    S = torch.empty(k, k, dtype=torch.float64, device=dev)
    alpha = torch.empty(k, k, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    rn2 = torch.empty(k, dtype=torch.float64, device=dev)
    # one work array serves the paired Gram blocks and the single ones (it is at
    # least as long); the residual norms come with the update of R where the
    # fused kernel takes the block width
    work = mfmv.block_gram2_work(n, k, dev)
    fused_norms = k <= 128
    nwork = mfmv.block_update_norms_work(n, k, dev) if fused_norms else None

    it, converged, breakdown = 0, False, False
    active = precond

    active(R, P)
    while it < maxit:
        op.apply(P, Q, precision=precision)
        mfmv.block_gram2(P, Q, R, G, S, work=work)    # P^T A P and P^T R, one pass over P
        if fallback is not None and active is not fallback:
            # Descent check on the direction about to be used: p_j^T r_j, the diagonal
            # of S = P^T R (= z_j^T r_j, R being orthogonal to the previous block).  If
            # it is not positive for every column (a NaN fails too), the rest of the run
            # uses the fallback, from a restarted direction block.
            if not bool(np.all(np.diagonal(S.cpu().numpy()) > 0)):   # host sync
                active = fallback
                if stats is not None:
                    stats.precond_switches += 1
                active(R, P)
                continue
        mfmv.spd_solve(G, S, alpha, st)
        mfmv.block_update(P, alpha, X, 1.0, 1.0)      # X += P alpha
        check = it + 1 == maxit or (it + 1) % check_every == 0
        if fused_norms:                               # R -= Q alpha, with ||r_j||^2
            mfmv.block_update_norms(Q, alpha, R, rn2, -1.0, 1.0, work=nwork)
        else:
            mfmv.block_update(Q, alpha, R, -1.0, 1.0)
            if check:
                mfmv.col_norms2(R, rn2)
        it += 1
        if check:
            rel = float((np.sqrt(rn2.cpu().numpy()) / bn).max())  # host sync
            if stats is not None:
                stats.history.append(rel)
            if int(st.item()) != 0 or not math.isfinite(rel):
                breakdown = True
                break
            if rel <= tol:
                converged = True
                break
        active(R, Z)
        mfmv.block_gram(Q, Z, S, work=work)           # (A P)^T Z
        mfmv.spd_solve(G, S, alpha, st)               # G^{-1} (A P)^T Z
        mfmv.block_update(P, alpha, Z, -1.0, 1.0)     # Z -= P G^{-1} (AP)^T Z
        P, Z = Z, P
    return X, it, converged, breakdown


def solve(op: mfmv.Operator, B, precond: Callable, tol: float = 1e-10, maxit: int = 2000,
          inner_precision: str = "fp64", inner_tol: float = 1e-6, max_refine: int = 20,
          fallback: Optional[Callable] = None, X0=None) -> tuple:
    """Solve A X = B to a true FP64 relative residual <= tol in every column.

    inner_precision "fp64": one block-PCG run with the FP64 apply (then a true
    residual check).  "fp32"/"bf16": FP64 iterative refinement around inner
    block-PCG runs with the matrix-core apply, each to `inner_tol`.
    Returns (X, SolveStats).
    """
    import torch
    t0 = time.perf_counter()
    stats = SolveStats()
    n, k = B.shape
    X = torch.empty_like(B)
    if X0 is None:
        mfmv.zero_ptr(X.data_ptr(), n, k, X.stride(0))
    else:
        mfmv.axpby(1.0, X0, 0.0, X)
    bn = _col_norms_host(B)
    R = torch.empty_like(B)

    def true_rel():
        op.apply(X, R)
        mfmv.axpby(1.0, B, -1.0, R)
        return float((_col_norms_host(R, floor=False) / bn).max())

    rel = true_rel()
    if inner_precision == "fp64":
        # one block-PCG run on (B, X); restarted from the current X after a
        # breakdown of the k x k step
        while rel > tol and stats.refinements < max_refine and stats.iterations < maxit:
            _, its, conv, bd = block_pcg(op, B, X, precond, tol, maxit - stats.iterations, "fp64",
                                         stats, fallback)
            stats.iterations += its
            stats.refinements += 1
            stats.breakdown |= bd
            rel = true_rel()
            if not bd and not conv:
                break
            if bd and its <= 1:
                break
    else:
        D = torch.empty_like(B)
        Rk = torch.empty_like(B)
        while rel > tol and stats.refinements < max_refine and stats.iterations < maxit:
            mfmv.zero_ptr(D.data_ptr(), n, k, D.stride(0))
            mfmv.axpby(1.0, R, 0.0, Rk)
            _, its, conv, bd = block_pcg(op, Rk, D, precond, max(inner_tol, 0.5 * tol / max(rel, tol)),
                                         maxit - stats.iterations, inner_precision, stats, fallback)
            stats.iterations += its
            stats.refinements += 1
            stats.breakdown |= bd
            mfmv.axpby(1.0, D, 1.0, X)
            rel = true_rel()
            if bd and its <= 1:
                break
    stats.rel_residual = rel
    stats.converged = stats.rel_residual <= tol
    torch.cuda.synchronize()
    stats.seconds = time.perf_counter() - t0
    return X, stats


def lanczos_extremes(op: mfmv.Operator, steps: int = 100, seed: int = 0,
                     matvec: Optional[Callable] = None) -> dict:
    """Ritz estimates of the extreme eigenvalues of A (FP64 apply, plain Lanczos
    from a seeded random vector on the free dofs): the SPD check before a solve
    (lambda_min > 0; Ritz values of the smallest end converge from above).
    `matvec(v, w)` (w := S v) replaces the apply for another symmetric S."""
    import torch
    n = op.ndofs
    rng = np.random.default_rng(seed)
    v0 = rng.uniform(-1.0, 1.0, (n, 1))
    v0[op.constrained_rows()] = 0.0
    v = torch.from_numpy(v0).cuda()
    w = torch.empty_like(v)
    vp = torch.zeros_like(v)
    nrm = float(np.sqrt(mfmv.col_norms2(v).cpu().numpy()[0]))
    mfmv.axpby(1.0 / nrm, v, 0.0, v)
    alphas, betas = [], []
    beta = 0.0
    for j in range(steps):
        if matvec is None:
            op.apply(v, w)
        else:
            matvec(v, w)
        if j > 0:
            mfmv.axpby(-beta, vp, 1.0, w)
        alpha = float(mfmv.col_dots(w, v).cpu().numpy()[0])
        mfmv.axpby(-alpha, v, 1.0, w)
        alphas.append(alpha)
        beta = float(np.sqrt(mfmv.col_norms2(w).cpu().numpy()[0]))
        if beta <= 1e-12 * abs(alpha) or j == steps - 1:
            break
        betas.append(beta)
        vp, v = v, vp
        mfmv.axpby(1.0 / beta, w, 0.0, v)
    m = len(alphas)
    Tm = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    ev = np.linalg.eigvalsh(Tm)
    return {"lambda_min": float(ev[0]), "lambda_max": float(ev[-1]), "steps": m}
