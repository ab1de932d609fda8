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
