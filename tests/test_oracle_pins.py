"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
library routines (numpy's Gauss-Legendre rule, scipy's Lagrange interpolation),
exact integrals of low-degree polynomials, invariants of the operator, and an
independent Kronecker-product assembly of the global matrices from 1D finite
element matrices.  A plausible mistake anywhere in the oracle (a dropped term,
a wrong sign or index, a transposed Jacobian) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest
import scipy.interpolate

from oracle import fe_oracle as fo
from workloads import BoxMesh, BC_NONE, BC_DIRICHLET0, BC_PERIODIC

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ---------------------------------------------------------------- 1D rules
def test_gauss3_closed_form():
    x, w = fo.gauss_legendre(3)
    np.testing.assert_allclose(x, GOLDEN["gauss3"]["points"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, GOLDEN["gauss3"]["weights"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", range(1, 17))
def test_gauss_matches_numpy_and_is_exact(n):
    x, w = fo.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-14)
    np.testing.assert_allclose(w, wr, atol=1e-14)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * n):  # exact for degree <= 2n-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_closed_form(p):
    np.testing.assert_allclose(fo.gll_nodes(p), GOLDEN["gll"][f"p{p}"], atol=1e-15)


@pytest.mark.parametrize("p", range(2, 11))
def test_gll_matches_library_roots(p):
    inner = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
    np.testing.assert_allclose(fo.gll_nodes(p), np.concatenate([[-1.0], inner, [1.0]]), atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_lagrange_basis(p):
    nodes = fo.gll_nodes(p)
    np.testing.assert_allclose(fo.lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-14)
    x = np.linspace(-1, 1, 23)
    L = fo.lagrange_values(nodes, x)
    D = fo.lagrange_derivatives(nodes, x)
    np.testing.assert_allclose(L.sum(axis=1), 1.0, atol=1e-13)      # partition of unity
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11)      # its derivative
    for k in range(p + 1):                                          # interpolation is exact
        np.testing.assert_allclose(L @ nodes ** k, x ** k, atol=1e-12)
        np.testing.assert_allclose(D @ nodes ** k, k * x ** max(k - 1, 0) if k else 0 * x, atol=1e-10)
    # against scipy's Lagrange polynomial
    for i in range(p + 1):
        poly = scipy.interpolate.lagrange(nodes, np.eye(p + 1)[i])
        np.testing.assert_allclose(L[:, i], poly(x), atol=1e-9)
        np.testing.assert_allclose(D[:, i], poly.deriv()(x), atol=1e-8)


# ------------------------------------------------------ element matrices
def test_q1_brick_textbook():
    mesh = BoxMesh(n=(1, 1, 1), bc=BC_NONE)
    for q in (2, 3):
        K = fo.Oracle(mesh, 1, q, mu=1.0).element_matrices()[0]
        M = fo.Oracle(mesh, 1, q, mu=0.0, sigma=1.0).element_matrices()[0]
        for a in range(8):
            for b in range(8):
                nd = bin(a ^ b).count("1")
                assert abs(K[a, b] - GOLDEN["q1_brick"]["K_by_ndiff"][nd]) < 1e-14
                assert abs(M[a, b] - GOLDEN["q1_brick"]["M_by_ndiff"][nd]) < 1e-15
        np.testing.assert_allclose(M.sum(axis=1), 1.0 / 8.0, atol=1e-15)


def _kron_reference(mesh, p, q, mu, c):
    """Global mu K + c M built as Kronecker products of 1D FE matrices (library rules only)."""
    gll = np.concatenate([[-1.0], np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real),
                          [1.0]]) if p > 1 else np.array([-1.0, 1.0])
    xg, wg = np.polynomial.legendre.leggauss(q)
    polys = [scipy.interpolate.lagrange(gll, np.eye(p + 1)[i]) for i in range(p + 1)]
    Lq = np.array([[pl(x) for pl in polys] for x in xg])
    Dq = np.array([[pl.deriv()(x) for pl in polys] for x in xg])
    K1s, M1s = [], []
    for d in range(3):
        n = int(mesh.n[d])
        h = (mesh.hi[d] - mesh.lo[d]) / n
        per = mesh.bc == BC_PERIODIC
        N = n * p + (0 if per else 1)
        ke = (2.0 / h) * Dq.T @ (wg[:, None] * Dq)
        me = (h / 2.0) * Lq.T @ (wg[:, None] * Lq)
        K1 = np.zeros((N, N))
        M1 = np.zeros((N, N))
        for c_ in range(n):
            idx = (c_ * p + np.arange(p + 1)) % N if per else c_ * p + np.arange(p + 1)
            for a in range(p + 1):
                for b in range(p + 1):
                    K1[idx[a], idx[b]] += ke[a, b]
                    M1[idx[a], idx[b]] += me[a, b]
        K1s.append(K1)
        M1s.append(M1)
    kron3 = lambda z, y, x: np.kron(z, np.kron(y, x))  # x fastest
    K = (kron3(M1s[2], M1s[1], K1s[0]) + kron3(M1s[2], K1s[1], M1s[0]) + kron3(K1s[2], M1s[1], M1s[0]))
    A = mu * K + c * kron3(M1s[2], M1s[1], M1s[0])
    if mesh.bc == BC_DIRICHLET0:
        Ns = [int(mesh.n[d]) * p + 1 for d in range(3)]
        gz, gy, gx = np.meshgrid(*[np.arange(v) for v in Ns[::-1]], indexing="ij")
        b = ((gx == 0) | (gx == Ns[0] - 1) | (gy == 0) | (gy == Ns[1] - 1) | (gz == 0) | (gz == Ns[2] - 1)).ravel()
        A[b, :] = 0.0
        A[:, b] = 0.0
    return A


@pytest.mark.parametrize("bc", [BC_NONE, BC_DIRICHLET0, BC_PERIODIC])
@pytest.mark.parametrize("p,q,n", [(1, 2, (2, 1, 2)), (2, 3, (2, 2, 1)), (3, 4, (1, 2, 2)), (2, 4, (2, 1, 1)),
                                   (3, 5, (1, 1, 1))])
def test_global_matrix_equals_kronecker_assembly(bc, p, q, n):
    mesh = BoxMesh(n=n, lo=(0.0, -1.0, 0.5), hi=(1.0, 0.5, 2.5), bc=bc)
    c = 0.7
    orc = fo.Oracle(mesh, p, q, mu=0.5, V=lambda x: np.full(x.shape[:-1], c))
    A = orc.assemble_dense()
    Aref = _kron_reference(mesh, p, q, 0.5, c)
    scale = np.abs(Aref).max()
    np.testing.assert_allclose(A, Aref, atol=1e-13 * scale)
    # the cell-matrix apply equals the dense product
    X = np.random.default_rng(5).uniform(-1, 1, (orc.ndofs, 3))
    np.testing.assert_allclose(orc.apply(X), Aref @ X, atol=1e-12 * scale * orc.ndofs ** 0.5)


# ------------------------------------------------------------- invariants
SHEAR = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])


@pytest.mark.parametrize("bc", [BC_NONE, BC_DIRICHLET0, BC_PERIODIC])
@pytest.mark.parametrize("lin", [None, SHEAR])
def test_symmetry(bc, lin):
    mesh = BoxMesh(n=(2, 3, 2), hi=(1.0, 1.5, 0.8), bc=bc, lin=lin)
    orc = fo.Oracle(mesh, 3, 4, mu=0.5, V=lambda x: np.sin(x[..., 0]) + x[..., 1] * x[..., 2], sigma=0.3)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(orc.ndofs), rng.standard_normal(orc.ndofs)
    a, b = x @ orc.apply(y), y @ orc.apply(x)
    assert abs(a - b) < 1e-13 * max(abs(a), 1.0)
    if bc == BC_DIRICHLET0:
        Y = orc.apply(rng.standard_normal(orc.ndofs))
        assert np.all(Y[orc.constrained] == 0.0)
        X2 = rng.standard_normal(orc.ndofs)
        X3 = X2.copy()
        X3[orc.constrained] = rng.standard_normal(orc.constrained.sum())
        np.testing.assert_array_equal(orc.apply(X2), orc.apply(X3))


@pytest.mark.parametrize("bc", [BC_NONE, BC_PERIODIC])
@pytest.mark.parametrize("lin", [None, SHEAR])
@pytest.mark.parametrize("p", [1, 2, 4])
def test_stiffness_annihilates_constants_and_mass_volume(bc, lin, p):
    mesh = BoxMesh(n=(2, 2, 3), lo=(0, 0, 0), hi=(1.0, 2.0, 1.5), bc=bc, lin=lin)
    K = fo.Oracle(mesh, p, p + 1, mu=1.0)
    one = np.ones(K.ndofs)
    assert np.abs(K.apply(one)).max() < 1e-12
    M = fo.Oracle(mesh, p, p + 1, mu=0.0, sigma=1.0)
    assert abs(one @ M.apply(one) - mesh.volume()) < 1e-12 * mesh.volume()
    # V == c on a periodic mesh: 1^T A 1 = c |Omega|
    A = fo.Oracle(mesh, p, p + 1, mu=0.5, V=lambda x: np.full(x.shape[:-1], -2.5))
    assert abs(one @ A.apply(one) - (-2.5) * mesh.volume()) < 1e-12 * mesh.volume()


def _node_coords(orc):
    """Physical coordinates of every global node (test-side, from GLL positions)."""
    X = np.zeros((orc.ndofs, 3))
    phi, _ = fo.trilinear(np.stack(np.meshgrid(orc.xi_n, orc.xi_n, orc.xi_n, indexing="ij")[::-1], -1)
                          .reshape(-1, 3))
    for e in range(orc.E):
        X[orc.map[e]] = phi @ orc.corners[e]
    return X


@pytest.mark.parametrize("p", [2, 3, 4])
def test_exact_energies_unit_cube(p):
    g = GOLDEN["energies_unit_cube"]
    mesh = BoxMesh(n=(2, 3, 2), bc=BC_NONE)
    K = fo.Oracle(mesh, p, p + 1, mu=1.0)
    M = fo.Oracle(mesh, p, p + 1, mu=0.0, sigma=1.0)
    x = _node_coords(K)
    u = x[:, 0]
    assert abs(u @ K.apply(u) - g["u=x"]["K"]) < 1e-13
    assert abs(u @ M.apply(u) - g["u=x"]["M"]) < 1e-13
    u = x[:, 0] ** 2 + x[:, 1] * x[:, 2]
    assert abs(u @ K.apply(u) - g["u=x^2+yz"]["K"]) < 1e-13
    assert abs(u @ M.apply(u) - g["u=x^2+yz"]["M"]) < 1e-13
    MV = fo.Oracle(mesh, p, p + 1, mu=0.0, V=lambda x: x[..., 0])
    one = np.ones(K.ndofs)
    assert abs(one @ MV.apply(one) - g["V=x1"]["oneMV1"]) < 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_bubble_energy_dirichlet_config1_operator(p):
    g = GOLDEN["energies_unit_cube"]["bubble"]
    mesh = BoxMesh(n=(4, 4, 4), bc=BC_DIRICHLET0)
    c = -0.8
    A = fo.Oracle(mesh, p, p + 1, mu=0.5, V=lambda x: np.full(x.shape[:-1], c))
    x = _node_coords(A)
    u = np.prod(x * (1 - x), axis=1)
    assert abs(u @ A.apply(u) - (0.5 * g["K"] + c * g["M"])) < 1e-15


def test_sheared_linear_energy():
    mesh = BoxMesh(n=(2, 2, 2), hi=(1.0, 1.2, 0.9), bc=BC_NONE, lin=SHEAR)
    K = fo.Oracle(mesh, 2, 3, mu=1.0)
    x = _node_coords(K)
    a = np.array([0.3, -1.1, 0.7])
    u = x @ a
    assert abs(u @ K.apply(u) - a @ a * mesh.volume()) < 1e-12


@pytest.mark.parametrize("p,ns", [(2, (8, 16)), (3, (4, 8))])
def test_rayleigh_quotient_converges(p, ns):
    """Periodic [0,L]^3, V = 0: the Rayleigh quotient of the interpolant of sin(2 pi x / L)
    tends to (2 pi / L)^2 with error O(h^{2p}) (energy-norm interpolation error squared)."""
    L = 2.0
    errs = []
    for n in ns:
        mesh = BoxMesh(n=(n, 1, 1), hi=(L, L, L), bc=BC_PERIODIC)
        K = fo.Oracle(mesh, p, p + 1, mu=1.0)
        M = fo.Oracle(mesh, p, p + 1, mu=0.0, sigma=1.0)
        u = np.sin(2 * np.pi * _node_coords(K)[:, 0] / L)
        errs.append(abs((u @ K.apply(u)) / (u @ M.apply(u)) - (2 * np.pi / L) ** 2))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - 2 * p) < 0.25, rate


def test_apply_rows_and_diagonal():
    mesh = BoxMesh(n=(3, 2, 2), bc=BC_DIRICHLET0)
    orc = fo.Oracle(mesh, 2, 3, mu=0.5, V=lambda x: -np.exp(-np.sum((x - 0.5) ** 2, -1) / 0.05))
    X = np.random.default_rng(3).uniform(-1, 1, (orc.ndofs, 4))
    rows = np.array([0, 17, 40, orc.ndofs - 1, 55])
    np.testing.assert_allclose(orc.apply_rows(X, rows), orc.apply(X)[rows], atol=1e-14)
    np.testing.assert_allclose(orc.diagonal(), np.diag(orc.assemble_dense()), atol=1e-15)


def test_periodic_single_cell_repeated_dofs():
    """n = 1 periodic: every cell node appears 8/4/2 times in the map; assembly must add all copies."""
    mesh = BoxMesh(n=(1, 1, 1), bc=BC_PERIODIC)
    orc = fo.Oracle(mesh, 2, 3, mu=0.5, V=lambda x: np.full(x.shape[:-1], 1.0))
    Aref = _kron_reference(mesh, 2, 3, 0.5, 1.0)
    np.testing.assert_allclose(orc.assemble_dense(), Aref, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_weighted_mass_orientation(p):
    """u^T M_V u for V = x_a, u = x_b: int x_1^3 = 1/4 but int x_2 x_1^2 = 1/6, so a permuted
    quadrature-point ordering of V (q1 <-> q3, say) fails this pin, unlike a constant V."""
    mesh = BoxMesh(n=(2, 2, 3), bc=BC_NONE)
    for a, b, exact in [(0, 0, 0.25), (1, 0, 1.0 / 6.0), (2, 2, 0.25), (2, 0, 1.0 / 6.0)]:
        MV = fo.Oracle(mesh, p, p + 1, mu=0.0, V=lambda x, a=a: x[..., a])
        u = _node_coords(MV)[:, b]
        assert abs(u @ MV.apply(u) - exact) < 1e-14
