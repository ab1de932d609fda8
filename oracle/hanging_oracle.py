"""FP64 CPU oracle for hanging-node constraints on a once-refined box mesh
(test infrastructure only: like fe_oracle, it may be imported by the tests, the
smoke check and the benchmark's CPU-baseline leg, never by the product path).

The mesh: a structured box of coarse hexahedra in which the coarse cells of one
index box [rlo, rhi) are each split into 2 x 2 x 2 children.  Faces between a
refined and an unrefined region are non-conforming: the fine nodes on them are
"hanging" and carry no unknown of their own.

What it computes (eq. AU with one partition; Sec. 3.2.2 for C):
  * C, the constraint matrix: identity on free nodes, zero rows for zero-Dirichlet
    nodes (constraints with empty masters), and on every hanging node the value
    of the unrefined neighbour cell's degree-p polynomial at that node, i.e. the
    tensor-product Lagrange interpolation of that cell's nodal values (the
    continuity requirement that makes the refined space conforming);
  * the constrained product Y = C^T Z (sum_e Q_e^T A^(e) Q_e) Z C X, with the
    element matrices of fe_oracle on cells of two sizes;
  * for the eigenproblem on the refined mesh (eq. shep): the GLL-lumped mass of
    the constrained space lumped by rows, m_c = C^T m_u (m_u the lumped mass of
    every cell, as in fe_oracle; row sums of C^T M_u C, since every row of C
    sums to one), and one Chebyshev filter step a D C^T A_u C D Y + b Y + c X
    with D = m_c^{-1/2} on free rows and 0 elsewhere.

Numbering (the layout the library's refined operator uses):
  * cells: unrefined coarse cells in lexicographic order (first index fastest),
    then the fine cells of the refined box, lexicographic over fine indices;
  * nodes: the coarse lattice nodes that belong to an unrefined cell,
    lexicographic, numbered consecutively; then every fine lattice node of the
    refined box, lexicographic.  A fine node on the interface is a node of its
    own even where it coincides with a coarse node (its constraint then has a
    single master of weight one).
  * zero-Dirichlet: nodes on the outer boundary (they win over hanging).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fe_oracle import (BC_DIRICHLET0, BC_PERIODIC, Oracle, _lin, gll_nodes,
                        lagrange_values)

FREE, DIRICHLET, HANGING = 0, 1, 2


class RefinedMesh:
    """A coarse box mesh (n, lo, hi, bc, lin) with the index box [rlo, rhi) refined once."""

    def __init__(self, n, lo, hi, rlo, rhi, bc=0, lin=None):
        self.n, self.lo, self.hi = list(n), list(lo), list(hi)
        self.rlo, self.rhi, self.bc, self.lin = list(rlo), list(rhi), bc, lin


def _empty(rm):
    return any(rm.rlo[d] >= rm.rhi[d] for d in range(3))


def refined_layout(rm, p):
    """Cells (origin and size in coarse-cell units), the cell-to-node map, the node kinds
    and every node's position in coarse-cell units (all in the numbering above)."""
    if rm.bc == BC_PERIODIC:
        raise ValueError("periodic refined meshes are not defined")
    n = [int(v) for v in rm.n]
    xi = gll_nodes(p)
    empty = _empty(rm)
    rlo, rhi = list(rm.rlo), list(rm.rhi)

    def refined(c):
        return (not empty) and all(rlo[d] <= c[d] < rhi[d] for d in range(3))

    origins, sizes = [], []
    for cz in range(n[2]):
        for cy in range(n[1]):
            for cx in range(n[0]):
                if not refined((cx, cy, cz)):
                    origins.append((cx, cy, cz))
                    sizes.append(1.0)
    ncoarse_cells = len(origins)
    if not empty:
        for fz in range(2 * rlo[2], 2 * rhi[2]):
            for fy in range(2 * rlo[1], 2 * rhi[1]):
                for fx in range(2 * rlo[0], 2 * rhi[0]):
                    origins.append((fx / 2, fy / 2, fz / 2))
                    sizes.append(0.5)
    E = len(origins)

    # coarse lattice nodes used by unrefined cells, numbered lexicographically
    N = [n[d] * p + 1 for d in range(3)]
    used = np.zeros((N[2], N[1], N[0]), dtype=bool)       # [z, y, x]: C order = x fastest
    for cx, cy, cz in origins[:ncoarse_cells]:
        used[cz * p:cz * p + p + 1, cy * p:cy * p + p + 1, cx * p:cx * p + p + 1] = True
    cidx = -np.ones(used.shape, dtype=np.int64)
    nc = int(used.sum())
    cidx[used] = np.arange(nc)
    F = [2 * (rhi[d] - rlo[d]) * p + 1 for d in range(3)] if not empty else [0, 0, 0]
    ndofs = nc + F[0] * F[1] * F[2]

    n1 = p + 1
    i3, i2, i1 = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    i1, i2, i3 = i1.ravel(), i2.ravel(), i3.ravel()
    cmap = np.empty((E, n1 ** 3), dtype=np.int64)
    for e in range(E):
        o = origins[e]
        if e < ncoarse_cells:
            cmap[e] = cidx[o[2] * p + i3, o[1] * p + i2, o[0] * p + i1]
        else:
            f = [int(round(2 * o[d])) - 2 * rlo[d] for d in range(3)]
            cmap[e] = nc + (f[0] * p + i1) + F[0] * ((f[1] * p + i2) + F[1] * (f[2] * p + i3))

    # node positions in coarse-cell units: lattice index g of step h/p (coarse) or
    # h/(2p) (fine): u = cell + (1 + xi_a) / 2 with g = cell * p + a
    def coord(g, fine):
        c, a = np.divmod(g, p)
        u = c + (1.0 + xi[a]) / 2.0
        return u / 2.0 if fine else u

    pos = np.zeros((ndofs, 3))
    kind = np.zeros(ndofs, dtype=np.int8)
    gz, gy, gx = np.nonzero(used)                          # C order: matches cidx numbering
    pos[:nc] = np.stack([coord(gx, False), coord(gy, False), coord(gz, False)], axis=1)
    bnd = (gx == 0) | (gx == N[0] - 1) | (gy == 0) | (gy == N[1] - 1) | (gz == 0) | (gz == N[2] - 1)
    if not empty:
        fz, fy, fx = np.meshgrid(np.arange(F[2]), np.arange(F[1]), np.arange(F[0]), indexing="ij")
        ax = [fx.ravel() + 2 * rlo[0] * p, fy.ravel() + 2 * rlo[1] * p, fz.ravel() + 2 * rlo[2] * p]
        pos[nc:] = np.stack([coord(ax[d], True) for d in range(3)], axis=1)
        fb = np.zeros(ax[0].size, dtype=bool)
        for d in range(3):
            fb |= (ax[d] == 0) | (ax[d] == 2 * n[d] * p)
        bnd = np.concatenate([bnd, fb])
    if rm.bc == BC_DIRICHLET0:
        kind[bnd] = DIRICHLET

    # hanging: fine nodes in the closure of an unrefined coarse cell
    host = -np.ones((ndofs, 3), dtype=np.int64)
    for i in range(nc, ndofs):
        if kind[i] == DIRICHLET:
            continue
        c = containing_coarse_cell(pos[i], n, refined)
        if c is not None:
            kind[i] = HANGING
            host[i] = c
    return dict(E=E, origins=np.array(origins, float), sizes=np.array(sizes), map=cmap,
                ndofs=ndofs, kind=kind, pos=pos, host=host, cidx=cidx,
                ncoarse_cells=ncoarse_cells)


def containing_coarse_cell(u, n, refined):
    """An unrefined coarse cell whose closure holds the point u (coarse units), or None."""
    cands = []
    for d in range(3):
        f = int(np.floor(u[d]))
        cands.append([c for c in (f - 1, f) if 0 <= c < n[d] and c <= u[d] <= c + 1])
    for cz in cands[2]:
        for cy in cands[1]:
            for cx in cands[0]:
                if not refined((cx, cy, cz)):
                    return (cx, cy, cz)
    return None


def constraint_matrix(lay, p):
    """C (ndofs x ndofs, sparse): rows of free nodes are unit rows, zero-Dirichlet rows are
    empty, and the row of a hanging node interpolates the host coarse cell's nodes at the
    hanging node (Dirichlet masters dropped: their values are zero)."""
    xi = gll_nodes(p)
    n1 = p + 1
    cidx, kind, pos = lay["cidx"], lay["kind"], lay["pos"]
    rows, cols, vals = [], [], []
    for i in range(lay["ndofs"]):
        if kind[i] == FREE:
            rows.append(i)
            cols.append(i)
            vals.append(1.0)
        elif kind[i] == HANGING:
            c = lay["host"][i]
            r = 2.0 * (pos[i] - np.asarray(c, float)) - 1.0     # reference coordinates in [-1, 1]
            L = [lagrange_values(xi, np.array([r[d]]))[0] for d in range(3)]
            # weight of the host node (a1, a2, a3): L_a1(r1) L_a2(r2) L_a3(r3), a1 fastest
            w = (L[2][:, None, None] * L[1][None, :, None] * L[0][None, None, :]).ravel()
            m = cidx[c[2] * p:c[2] * p + n1, c[1] * p:c[1] * p + n1, c[0] * p:c[0] * p + n1].ravel()
            keep = (w != 0.0) & (kind[m] != DIRICHLET)
            rows.extend([i] * int(keep.sum()))
            cols.extend(m[keep].tolist())
            vals.extend(w[keep].tolist())
    n = lay["ndofs"]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


class RefinedOracle(Oracle):
    """Element-matrix evaluation of the constrained product on a once-refined box."""

    def __init__(self, rmesh, p: int, q: int, mu: float, V=None, sigma: float = 0.0):
        if p < 1 or q < 1:
            raise ValueError("p >= 1 and q >= 1")
        self.mesh, self.p, self.q, self.mu, self.sigma = rmesh, p, q, float(mu), float(sigma)
        self.np1 = p + 1
        lay = refined_layout(rmesh, p)
        self.layout = lay
        self.E, self.map, self.ndofs = lay["E"], lay["map"], lay["ndofs"]
        self.kind = lay["kind"]
        self.constrained = lay["kind"] == DIRICHLET
        self.hanging = lay["kind"] == HANGING
        lo = np.asarray(rmesh.lo, float)
        h = (np.asarray(rmesh.hi, float) - lo) / np.asarray(rmesh.n, float)
        bits = np.array([[(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], float)
        y = lo + h * (lay["origins"][:, None, :] + lay["sizes"][:, None, None] * bits[None])
        self.corners = y @ _lin(rmesh).T
        self._setup(V)
        self.C = constraint_matrix(lay, p)

    def distribute(self, X):
        """The in-place action of C: hanging rows := their interpolated values; every
        other row unchanged."""
        X = np.array(X, dtype=np.float64)
        CX = self.C @ X
        X[self.hanging] = CX[self.hanging]
        return X

    def condense(self, Y):
        """C^T Y (masters accumulate their hanging nodes' weighted rows, hanging and
        Dirichlet rows become zero)."""
        return self.C.T @ np.asarray(Y, dtype=np.float64)

    def apply_constrained(self, X):
        """Y = C^T Z A_u Z C X: the operator on the conforming (constrained) space."""
        return self.condense(self.apply(self.C @ np.asarray(X, dtype=np.float64)))

    def lumped_mass_constrained(self):
        """m_c = C^T m_u: zero on hanging and zero-Dirichlet rows."""
        return self.C.T @ self.lumped_mass()

    def cheb_step_constrained(self, D, Y, Xp, a, b, c):
        """a D C^T A_u C (D Y) + b Y + c Xp on rows with D > 0; 0 on the others."""
        out = a * D[:, None] * self.apply_constrained(D[:, None] * Y) + b * Y
        if Xp is not None:
            out = out + c * Xp
        out[D == 0.0] = 0.0
        return out
