"""Oracle (test infrastructure only) for the learned cell-local preconditioner.

Plain numpy FP64, loops over cells, written from the definitions; shares no
code with the HIP path.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may use it.

Definitions (the preconditioner of block CG, a learned component that the
paper does not have; the cell extraction Q_e is that of Sec. 3.2.3):
- cell input: x_{e,j} = (Q_e r_j) / rho_{e,j}, rho = RMS of Q_e r_j over the
  cell's np^3 nodes (constrained nodes read as 0), x = 0 when rho = 0;
- network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
  y = W3 h2 + b3 + S x (weights W_l stored as (out, in) matrices, S the
  symmetric F x F skip);
- output: z_j = d^{-1} r_j + sum_e Q_e^T (w * rho_{e,j} y_{e,j}) with w the
  partition-of-unity weight (1 / number of cell occurrences of a node), or
  with sqrt(w) on the input and on the output (symmetric form); the Jacobi
  term optional;
- training loss: mean over (cell, column) rows of ||y - t||^2, t = target
  cell vector scaled by the same 1 / rho.
Parity pin of the backward pass: central finite differences of the loss
(tests/test_mlp_oracle.py).
"""
from __future__ import annotations

import numpy as np

from .fe_oracle import cell_dof_map, constrained_mask


def bf16_round(a):
    """Round FP32 values to BF16 (nearest even) and return them as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def pou_weights(mesh, p):
    """Per (cell, local node): 1 / (number of (cell, local node) occurrences of its
    global node), 0 for constrained nodes."""
    cmap = cell_dof_map(mesh, p)
    cons = constrained_mask(mesh, p)
    count = np.zeros(cons.size)
    np.add.at(count, cmap.ravel(), 1.0)
    w = 1.0 / count[cmap]
    w[cons[cmap]] = 0.0
    return w


def cell_inputs(mesh, p, R, E=None, pou_sqrt=False, dscale=None):
    """(X, T, rho): X[e*k + j] = u / rho with u = Q_e r_j (times sqrt(w) if
    pou_sqrt, divided by sqrt(dscale) at each node if given), rho = RMS of u;
    T = Q_e E_j sqrt(dscale) / rho (no partition weight) or None; rows are
    (cell, column) pairs, features the np^3 local nodes."""
    cmap = cell_dof_map(mesh, p)
    cons = constrained_mask(mesh, p)
    wts = np.sqrt(pou_weights(mesh, p)) if pou_sqrt else None
    dh = None if dscale is None else np.sqrt(dscale)
    ncell, F = cmap.shape
    k = R.shape[1]
    X = np.zeros((ncell * k, F))
    T = None if E is None else np.zeros((ncell * k, F))
    rho = np.zeros(ncell * k)
    for e in range(ncell):
        live = ~cons[cmap[e]]
        Re = np.where(live[:, None], R[cmap[e]], 0.0)          # F x k
        if wts is not None:
            Re = Re * wts[e][:, None]
        if dh is not None:
            Re = Re / dh[cmap[e]][:, None]
        r = np.sqrt((Re * Re).sum(axis=0) / F)
        s = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
        X[e * k:(e + 1) * k] = (Re * s).T
        rho[e * k:(e + 1) * k] = r
        if E is not None:
            Ee = np.where(live[:, None], E[cmap[e]], 0.0)
            if dh is not None:
                Ee = Ee * dh[cmap[e]][:, None]
            T[e * k:(e + 1) * k] = (Ee * s).T
    return X, T, rho


def cell_assemble(mesh, p, Y, rho, k, R=None, diag=None, pou_sqrt=False, dscale=None):
    """z = (R / diag if given) + sum_e Q_e^T (w rho y) (sqrt(w) if pou_sqrt,
    divided by sqrt(dscale) at each node if given) for rows (cell, column)."""
    cmap = cell_dof_map(mesh, p)
    w = pou_weights(mesh, p)
    if pou_sqrt:
        w = np.sqrt(w)
    if dscale is not None:
        w = w / np.sqrt(dscale)[cmap]
    ndofs = constrained_mask(mesh, p).size
    Z = np.zeros((ndofs, k)) if R is None else R / diag[:, None]
    for e in range(cmap.shape[0]):
        rows = slice(e * k, (e + 1) * k)
        contrib = (Y[rows] * rho[rows, None]).T * w[e][:, None]   # F x k
        np.add.at(Z, cmap[e], contrib)
    return Z


def forward(params, X):
    """Rows of X (n x F) -> (h1, h2, y); params = [W1, b1, W2, b2, W3, b3, S]."""
    W1, b1, W2, b2, W3, b3, S = params
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3.T + b3 + X @ S.T
    return h1, h2, y


def loss_and_grads(params, X, T):
    """Mean over rows of ||y - t||^2 and its gradients (backpropagation); the
    gradient of S is the plain one (the symmetric projection is the optimizer's)."""
    W1, b1, W2, b2, W3, b3, S = params
    n = X.shape[0]
    h1, h2, y = forward(params, X)
    d = y - T
    loss = float((d * d).sum() / n)
    dy = 2.0 * d / n
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    gS = dy.T @ X
    dh2 = (dy @ W3) * (h2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (h1 > 0)
    gW1 = dh1.T @ X
    gb1 = dh1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3, gS]


def adam_step(w, g, m1, m2, lr, b1, b2, eps, step):
    """One Adam update (bias-corrected moments), FP32 like the kernel."""
    w, g, m1, m2 = (np.asarray(a, dtype=np.float32) for a in (w, g, m1, m2))
    m1 = np.float32(b1) * m1 + np.float32(1 - b1) * g
    m2 = np.float32(b2) * m2 + np.float32(1 - b2) * g * g
    c1 = np.float32(1 - b1 ** step)
    c2 = np.float32(1 - b2 ** step)
    w = w - np.float32(lr) * (m1 / c1) / (np.sqrt(m2 / c2) + np.float32(eps))
    return w, m1, m2
