"""FP64 CPU oracle for Y = A X (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the product path never does.  It shares no code with
the HIP library: its 1D rules, basis tables, Jacobians and element matrices are
computed here, independently, from the definitions in the paper.

What it computes (Sec. 2.1-2.2 of the paper):
  * the operator A = mu*K + M^kappa (+ sigma*M), with K, M, M^kappa the
    quadrature sums of the stiffness, mass and weighted-mass integrals
    (eq. integrals; eq. stiffnessmatinteg/stiffnessmatquad; eq. mass3d), on
    tensor-product Lagrange elements of degree p with GLL nodes (eq. NTensor) and
    an n_q-point Gauss rule per direction (eq. quadTensor);
  * the product the "FE-cell level local dense matrices" way (Sec. 2.2.1): dense
    element matrices A^(e), extraction X_e = Q_e C X, batched dense products
    A^(e) X_e, assembly sum_e Q_e^T (eq. AU with a single partition);
  * for the eigenvalue problem (eq. ghep / eq. shep): the GLL-lumped diagonal
    mass M and one Chebyshev filter step a M^{-1/2} A M^{-1/2} Y + b Y + c X
    (Alg. ChFSi).

Readings of points the paper leaves open (each also listed in the design notes):
  * J is d x / d xi (reference -> physical); the stated direction of the map
    only makes the quadrature formula consistent this way round.
  * Dirichlet constraints with empty masters (Sec. 3.2.2): constrained input
    rows are treated as zero and constrained output rows are written as zero,
    i.e. Y = Z A Z X with Z the 0/1 projection onto free nodes.
  * Periodic meshes identify nodes modulo the node count per direction.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

BC_NONE = 0
BC_DIRICHLET0 = 1
BC_PERIODIC = 2


# ----------------------------------------------------------------------------
# 1D rules (Sec. 2.2.2: GLL nodal points; Gauss quadrature of n_q points)
# ----------------------------------------------------------------------------

def legendre_with_derivs(n: int, x):
    """Legendre P_n and its first two derivatives by the three-term recurrence.

    (k) P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2};  P_k' = x P_{k-1}' + k P_{k-1};
    P_k'' = x P_{k-1}'' + (k+1) P_{k-1}'.
    """
    x = np.asarray(x, dtype=np.float64)
    p_prev, p = np.zeros_like(x), np.ones_like(x)
    d_prev, d = np.zeros_like(x), np.zeros_like(x)
    dd = np.zeros_like(x)
    for k in range(1, n + 1):
        p_new = ((2 * k - 1) * x * p - (k - 1) * p_prev) / k
        d_new = x * d + k * p
        dd_new = x * dd + (k + 1) * d
        p_prev, p = p, p_new
        d, dd = d_new, dd_new
    return p, d, dd


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1]: roots of P_n by Newton; w = 2/((1-x^2) P_n'^2)."""
    if n < 1:
        raise ValueError("n >= 1")
    i = np.arange(n)
    x = -np.cos(np.pi * (i + 0.75) / (n + 0.5))
    for _ in range(100):
        p, d, _dd = legendre_with_derivs(n, x)
        dx = p / d
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, d, _dd = legendre_with_derivs(n, x)
    w = 2.0 / ((1.0 - x * x) * d * d)
    order = np.argsort(x)
    return x[order], w[order]


def gll_nodes(p: int):
    """p+1 Gauss-Lobatto-Legendre nodes: -1, the roots of P_p', and +1 (ascending)."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([-1.0, 1.0])
    i = np.arange(1, p)
    x = -np.cos(np.pi * i / p)
    for _ in range(100):
        _p, d, dd = legendre_with_derivs(p, x)
        dx = d / dd
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    return np.concatenate([[-1.0], np.sort(x), [1.0]])


def gll_weights(p: int):
    """Weights of the (p+1)-point Gauss-Lobatto-Legendre rule: 2 / (p (p+1) P_p(x_i)^2)."""
    x = gll_nodes(p)
    P, _d, _dd = legendre_with_derivs(p, x)
    return 2.0 / (p * (p + 1) * P * P)


def lagrange_values(nodes, x):
    """L[q, i] = prod_{m != i} (x_q - x_m) / (x_i - x_m)."""
    nodes = np.asarray(nodes, float)
    x = np.asarray(x, float)
    L = np.ones((x.size, nodes.size))
    for i in range(nodes.size):
        for m in range(nodes.size):
            if m != i:
                L[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return L


def lagrange_derivatives(nodes, x):
    """dL[q, i] = sum_{l != i} 1/(x_i - x_l) prod_{m != i, l} (x_q - x_m)/(x_i - x_m)."""
    nodes = np.asarray(nodes, float)
    x = np.asarray(x, float)
    n = nodes.size
    D = np.zeros((x.size, n))
    for i in range(n):
        for l in range(n):
            if l == i:
                continue
            term = np.full(x.size, 1.0 / (nodes[i] - nodes[l]))
            for m in range(n):
                if m != i and m != l:
                    term *= (x - nodes[m]) / (nodes[i] - nodes[m])
            D[:, i] += term
    return D


# ----------------------------------------------------------------------------
# Structured box mesh: numbering, constraints, geometry
# ----------------------------------------------------------------------------

def nodes_per_dir(mesh, p):
    per = mesh.bc == BC_PERIODIC
    return [int(mesh.n[d]) * p + (0 if per else 1) for d in range(3)]


def cell_dof_map(mesh, p):
    """Q: E x (p+1)^3 global node indices.  Cells with x fastest; local nodes with p1 fastest
    (the index order of Sec. 3.2.3); global node (gx, gy, gz) -> gx + Nx*(gy + Ny*gz)."""
    nx, ny, nz = (int(v) for v in mesh.n)
    Nx, Ny, Nz = nodes_per_dir(mesh, p)
    n1 = p + 1
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    i3, i2, i1 = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    i1, i2, i3 = i1.ravel(), i2.ravel(), i3.ravel()
    gx = cx[:, None] * p + i1[None, :]
    gy = cy[:, None] * p + i2[None, :]
    gz = cz[:, None] * p + i3[None, :]
    if mesh.bc == BC_PERIODIC:
        gx, gy, gz = gx % Nx, gy % Ny, gz % Nz
    return (gx + Nx * (gy + Ny * gz)).astype(np.int64)


def constrained_mask(mesh, p):
    """True for nodes on the boundary of a zero-Dirichlet mesh (constraints with empty masters)."""
    Nx, Ny, Nz = nodes_per_dir(mesh, p)
    m = np.zeros(Nx * Ny * Nz, dtype=bool)
    if mesh.bc != BC_DIRICHLET0:
        return m
    gz, gy, gx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    b = (gx == 0) | (gx == Nx - 1) | (gy == 0) | (gy == Ny - 1) | (gz == 0) | (gz == Nz - 1)
    return b.ravel()


def _lin(mesh):
    return np.eye(3) if getattr(mesh, "lin", None) is None else np.asarray(mesh.lin, float)


def cell_corners(mesh):
    """Physical coordinates of the 8 corners of every cell: E x 8 x 3, corner c = c0 + 2 c1 + 4 c2."""
    nx, ny, nz = (int(v) for v in mesh.n)
    lo = np.asarray(mesh.lo, float)
    h = (np.asarray(mesh.hi, float) - lo) / np.array([nx, ny, nz], float)
    e = np.arange(nx * ny * nz)
    c = np.stack([e % nx, (e // nx) % ny, e // (nx * ny)], axis=1).astype(float)
    bits = np.array([[(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], float)
    y = lo[None, None, :] + h[None, None, :] * (c[:, None, :] + bits[None, :, :])
    return y @ _lin(mesh).T


def trilinear(xi):
    """Values phi[k, c] and reference gradients dphi[k, c, s] of the 8 trilinear vertex functions."""
    xi = np.atleast_2d(xi)
    phi = np.ones((xi.shape[0], 8))
    dphi = np.ones((xi.shape[0], 8, 3))
    for c in range(8):
        bits = [(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1]
        f = [(1 + x) / 2 if b else (1 - x) / 2 for x, b in zip(xi.T, bits)]
        df = [np.full(xi.shape[0], 0.5 if b else -0.5) for b in bits]
        phi[:, c] = f[0] * f[1] * f[2]
        dphi[:, c, 0] = df[0] * f[1] * f[2]
        dphi[:, c, 1] = f[0] * df[1] * f[2]
        dphi[:, c, 2] = f[0] * f[1] * df[2]
    return phi, dphi


# ----------------------------------------------------------------------------
# The oracle proper
# ----------------------------------------------------------------------------

class Oracle:
    """Cell-matrix evaluation of Y = A X with A = mu K + M^V + sigma M (FP64, CPU).

    ``V`` is either a callable V(x) of physical points (..., 3), or None (V = 0).
    """

    def __init__(self, mesh, p: int, q: int, mu: float, V=None, sigma: float = 0.0):
        if p < 1 or q < 1:
            raise ValueError("p >= 1 and q >= 1")
        self.mesh, self.p, self.q, self.mu, self.sigma = mesh, p, q, float(mu), float(sigma)
        self.np1 = p + 1
        self.E = int(mesh.n[0]) * int(mesh.n[1]) * int(mesh.n[2])
        self.map = cell_dof_map(mesh, p)
        self.ndofs = int(np.prod(nodes_per_dir(mesh, p)))
        self.constrained = constrained_mask(mesh, p)
        self.corners = cell_corners(mesh)
        self._setup(V)

    def _setup(self, V):
        """Basis tables and per-point geometry; needs p, q, E, map and corners set."""
        p, q = self.p, self.q
        # 1D tables: GLL nodal basis (values, derivatives) at the Gauss points.
        self.xi_q, self.w_q = gauss_legendre(q)
        self.xi_n = gll_nodes(p)
        N1 = lagrange_values(self.xi_n, self.xi_q)        # n_q x n_p
        D1 = lagrange_derivatives(self.xi_n, self.xi_q)   # n_q x n_p

        # 3D tables by explicit triple products (eq. NTensor), q1 / i1 fastest.
        qq3, qq2, qq1 = np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij")
        ii3, ii2, ii1 = np.meshgrid(np.arange(self.np1), np.arange(self.np1), np.arange(self.np1),
                                    indexing="ij")
        Q1, Q2, Q3 = qq1.ravel(), qq2.ravel(), qq3.ravel()
        I1, I2, I3 = ii1.ravel(), ii2.ravel(), ii3.ravel()
        self.N3 = N1[Q1][:, I1] * N1[Q2][:, I2] * N1[Q3][:, I3]
        self.dN3 = np.stack([
            D1[Q1][:, I1] * N1[Q2][:, I2] * N1[Q3][:, I3],
            N1[Q1][:, I1] * D1[Q2][:, I2] * N1[Q3][:, I3],
            N1[Q1][:, I1] * N1[Q2][:, I2] * D1[Q3][:, I3],
        ])                                                  # 3 x n_q^3 x n_p^3
        self.wQ = self.w_q[Q1] * self.w_q[Q2] * self.w_q[Q3]
        self.xiQ = np.stack([self.xi_q[Q1], self.xi_q[Q2], self.xi_q[Q3]], axis=1)

        # Geometry at every quadrature point of every cell, from the trilinear map.
        phi, dphi = trilinear(self.xiQ)
        self.xq = np.einsum("kc,ecd->ekd", phi, self.corners)           # E x n_q^3 x 3
        self.J = np.einsum("kcs,ecd->ekds", dphi, self.corners)         # E x n_q^3 x 3 x 3
        self.detJ = np.linalg.det(self.J)
        self.Jinv = np.linalg.inv(self.J)

        if V is None:
            self.Vq = np.zeros((self.E, q ** 3))
        elif callable(V):
            self.Vq = np.asarray(V(self.xq), dtype=np.float64)
        else:
            self.Vq = np.asarray(V, dtype=np.float64).reshape(self.E, q ** 3)
        self._Ae = None

    # -- element matrices (eq. stiffnessmatquad, eq. mass3d) ------------------
    def element_matrices(self, cells=None):
        """Dense A^(e) = mu K^(e) + M^(e)_{V+sigma} for the given cells (all if None)."""
        cells = np.arange(self.E) if cells is None else np.asarray(cells)
        out = np.empty((cells.size, self.np1 ** 3, self.np1 ** 3))
        for k, e in enumerate(cells):
            wdet = self.wQ * self.detJ[e]
            # physical gradients: grad_x N = J^{-T} grad_xi N, component a = sum_s Jinv[s, a] dN_s
            gx = np.einsum("qsa,sqi->aqi", self.Jinv[e], self.dN3)
            K = np.zeros((self.np1 ** 3, self.np1 ** 3))
            for a in range(3):
                K += gx[a].T @ (wdet[:, None] * gx[a])
            M = self.N3.T @ ((wdet * (self.Vq[e] + self.sigma))[:, None] * self.N3)
            out[k] = self.mu * K + M
        return out

    def all_element_matrices(self):
        if self._Ae is None:
            self._Ae = self.element_matrices()
        return self._Ae

    def scatter_matrix(self, cells=None):
        """Sparse Boolean matrix of sum_e Q_e^T over the given cells (ndofs x |cells| n_p^3)."""
        cells = np.arange(self.E) if cells is None else np.asarray(cells)
        rows = self.map[cells].ravel()
        cols = np.arange(rows.size)
        return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(self.ndofs, rows.size))

    # -- the product (Sec. 2.2.1, steps 2-4) ---------------------------------
    def apply(self, X, cells=None, Ae=None):
        """Y = Z (sum_e Q_e^T A^(e) Q_e) Z X, Z = projection onto unconstrained nodes.

        With ``cells`` given, only those cells' contributions are summed (used to time
        bounded samples and to compute selected output rows)."""
        X = np.asarray(X, dtype=np.float64)
        squeeze = X.ndim == 1
        if squeeze:
            X = X[:, None]
        Xc = X.copy()
        Xc[self.constrained] = 0.0
        if cells is None:
            cells = np.arange(self.E)
            if Ae is None:
                Ae = self.all_element_matrices()
        elif Ae is None:
            Ae = self.element_matrices(cells)
        Xe = Xc[self.map[cells]]                              # |cells| x n_p^3 x nvec
        Ye = np.matmul(Ae, Xe)
        Y = self.scatter_matrix(cells) @ Ye.reshape(-1, X.shape[1])
        Y[self.constrained] = 0.0
        return Y[:, 0] if squeeze else Y

    def cells_touching(self, rows):
        rows = np.asarray(rows)
        hit = np.isin(self.map, rows).any(axis=1)
        return np.nonzero(hit)[0]

    def apply_rows(self, X, rows):
        """Selected rows of Y = A X, computed from the cells that touch them only."""
        cells = self.cells_touching(rows)
        return self.apply(X, cells=cells)[np.asarray(rows)]

    def assemble_dense(self):
        """Dense global A (tiny meshes only), with constrained rows and columns zeroed."""
        A = np.zeros((self.ndofs, self.ndofs))
        Ae = self.all_element_matrices()
        for e in range(self.E):
            idx = self.map[e]
            # np.add.at sums repeated indices (a periodic mesh with one cell per direction
            # maps several local nodes of a cell onto the same global node)
            np.add.at(A, (idx[:, None], idx[None, :]), Ae[e])
        A[self.constrained, :] = 0.0
        A[:, self.constrained] = 0.0
        return A

    # -- lumped mass and the Chebyshev filter step (eigenvalue problem) -------
    def lumped_mass(self):
        """The mass matrix with its overlap integral evaluated by the GLL rule of the
        element's own nodes, which makes it diagonal (Helmholtz eigenvalue problem,
        eq. shep): m_i = sum over cells and local nodes at i of w_a w_b w_c det J(node).
        Constrained entries zero."""
        wg = gll_weights(self.p)
        xi = self.xi_n
        n = self.np1
        i3, i2, i1 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        I1, I2, I3 = i1.ravel(), i2.ravel(), i3.ravel()
        _phi, dphi = trilinear(np.stack([xi[I1], xi[I2], xi[I3]], axis=1))
        J = np.einsum("kcs,ecd->ekds", dphi, self.corners)              # E x n^3 x 3 x 3
        vals = wg[I1] * wg[I2] * wg[I3] * np.linalg.det(J)             # E x n^3
        m = np.zeros(self.ndofs)
        np.add.at(m, self.map.ravel(), vals.ravel())
        m[self.constrained] = 0.0
        return m

    def cheb_step(self, D, Y, Xp, a, b, c):
        """a D A (D Y) + b Y + c Xp (one step of the Chebyshev filter of Alg. ChFSi on
        D A D, D = M^{-1/2}); constrained rows zero; Xp may be None."""
        out = a * D[:, None] * self.apply(D[:, None] * Y) + b * Y
        if Xp is not None:
            out = out + c * Xp
        out[self.constrained] = 0.0
        return out

    def chebyshev_filter(self, D, U, m, lam_min, lam_max, lam_u):
        """p_m(H~) U on the standard form H~ = D A D (eq. shep), see chebyshev_filter."""
        def H(Z):
            out = D[:, None] * self.apply(D[:, None] * Z)
            out[self.constrained] = 0.0
            return out
        return chebyshev_filter(H, U, m, lam_min, lam_max, lam_u)

    def diagonal(self):
        """diag(A) (constrained entries zero), from the element-matrix diagonals."""
        d = np.zeros(self.ndofs)
        Ae = self.all_element_matrices()
        np.add.at(d, self.map.ravel(), np.einsum("eii->ei", Ae).ravel())
        d[self.constrained] = 0.0
        return d


# ----------------------------------------------------------------------------
# Chebyshev filter of subspace iteration (Alg. ChFSi)
# ----------------------------------------------------------------------------
def chebyshev_filter(H, U, m, lam_min, lam_max, lam_u):
    """p_m(H) U for a symmetric operator H given by its action Z -> H Z.

    p_m is the degree-m Chebyshev polynomial of the first kind mapped so that the
    unwanted interval [lam_u, lam_max] goes to [-1, 1], normalised to 1 at lam_min
    (Alg. ChFSi):  p_m(t) = T_m((t - c) / e) / T_m((lam_min - c) / e), with c and e
    the centre and half-width of [lam_u, lam_max].  Written from the definition:
    T_0 = 1, T_1(x) = x, T_{k+1}(x) = 2 x T_k(x) - T_{k-1}(x) on the matrix argument
    L = (H - c) / e, and one division by the scalar T_m at the end (no per-step
    normalisation)."""
    if m < 1:
        raise ValueError("m >= 1")
    U = np.asarray(U, dtype=np.float64)
    c = 0.5 * (lam_max + lam_u)
    e = 0.5 * (lam_max - lam_u)

    def L(Z):
        return (H(Z) - c * Z) / e

    prev, cur = U, L(U)
    x0 = (lam_min - c) / e
    t_prev, t_cur = 1.0, x0
    for _ in range(2, m + 1):
        prev, cur = cur, 2.0 * L(cur) - prev
        t_prev, t_cur = t_cur, 2.0 * x0 * t_cur - t_prev
    return cur / t_cur
