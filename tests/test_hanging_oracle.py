"""Pins of the hanging-node oracle (once-refined box mesh, Sec. 3.2.2 constraints).

Each test checks the oracle against something other than itself: the uniform-mesh
oracle where the refined mesh degenerates to a uniform one, exact reproduction of
polynomials of the element degree at hanging nodes (node coordinates taken from
the cells' own geometry), closed-form bilinear forms of polynomials on the box
(numpy polynomial integration), symmetry and the one-dimensional null space of
the constrained stiffness.  A wrong child offset, a swapped tangential axis, a
missing C^T term or a dropped Dirichlet row fails one of them.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle import fe_oracle as fo
from oracle.hanging_oracle import RefinedMesh, RefinedOracle, HANGING, DIRICHLET
from workloads import BoxMesh, BC_NONE, BC_DIRICHLET0

LO, HI = [0.0, 0.0, 0.0], [2.0, 1.0, 1.5]


def node_coords(orc):
    """Physical coordinates of every node, from each cell's own trilinear map at its GLL nodes."""
    xi = fo.gll_nodes(orc.p)
    n1 = orc.p + 1
    i3, i2, i1 = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    ref = np.stack([xi[i1.ravel()], xi[i2.ravel()], xi[i3.ravel()]], axis=1)
    phi, _ = fo.trilinear(ref)
    x = np.full((orc.ndofs, 3), np.nan)
    pts = np.einsum("kc,ecd->ekd", phi, orc.corners)
    for e in range(orc.E):
        x[orc.map[e]] = pts[e]
    return x


def poly_field(coefs, x):
    return np.prod([P.polyval(x[:, d], coefs[d]) for d in range(3)], axis=0)


def exact_forms(cu, cw, mu, sigma):
    """mu * int grad w . grad u + sigma * int w u over the box [LO, HI], u and w separable."""
    def integ(c):
        ci = P.polyint(c)
        return lambda d: P.polyval(HI[d], ci) - P.polyval(LO[d], ci)
    mass = [integ(P.polymul(cu[d], cw[d]))(d) for d in range(3)]
    grad = [integ(P.polymul(P.polyder(cu[d]), P.polyder(cw[d])))(d) for d in range(3)]
    stiff = sum(grad[d] * np.prod([mass[e] for e in range(3) if e != d]) for d in range(3))
    return mu * stiff + sigma * np.prod(mass)


MESHES = [
    dict(n=[3, 3, 3], rlo=[1, 1, 1], rhi=[2, 2, 2]),     # refined core: hanging on all six faces
    dict(n=[3, 2, 2], rlo=[0, 1, 0], rhi=[2, 2, 1]),     # refined block touching the boundary
]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_empty_refinement_is_the_uniform_mesh(p):
    box = BoxMesh([3, 2, 2], LO, HI, BC_DIRICHLET0)
    rm = RefinedMesh([3, 2, 2], LO, HI, [1, 0, 0], [1, 2, 2], bc=BC_DIRICHLET0)
    V = lambda x: 1.0 + x[..., 0]
    ref, orc = fo.Oracle(box, p, p + 1, 0.5, V, 0.3), RefinedOracle(rm, p, p + 1, 0.5, V, 0.3)
    assert orc.ndofs == ref.ndofs and not orc.hanging.any()
    np.testing.assert_array_equal(orc.map, ref.map)
    X = np.random.default_rng(1).standard_normal((ref.ndofs, 3))
    np.testing.assert_allclose(orc.apply_constrained(X), ref.apply(X), rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_full_refinement_is_the_uniform_fine_mesh(p):
    rm = RefinedMesh([2, 1, 2], LO, HI, [0, 0, 0], [2, 1, 2], bc=BC_DIRICHLET0)
    box = BoxMesh([4, 2, 4], LO, HI, BC_DIRICHLET0)
    V = lambda x: np.cos(x[..., 1])
    ref, orc = fo.Oracle(box, p, p + 1, 1.0, V, 0.0), RefinedOracle(rm, p, p + 1, 1.0, V, 0.0)
    assert orc.ndofs == ref.ndofs and not orc.hanging.any()
    np.testing.assert_array_equal(orc.map, ref.map)
    X = np.random.default_rng(2).standard_normal((ref.ndofs, 2))
    np.testing.assert_allclose(orc.apply_constrained(X), ref.apply(X), rtol=0, atol=1e-12)


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_hanging_values_reproduce_degree_p_polynomials(mesh, p):
    rm = RefinedMesh(mesh["n"], LO, HI, mesh["rlo"], mesh["rhi"])
    orc = RefinedOracle(rm, p, p + 1, 1.0)
    assert orc.hanging.sum() > 0
    x = node_coords(orc)
    rng = np.random.default_rng(p)
    coefs = [rng.standard_normal(p + 1) for _ in range(3)]
    u = poly_field(coefs, x)
    X = np.where(orc.hanging, 1e3, u)[:, None]          # garbage on hanging rows: C overwrites
    got = orc.distribute(X)[:, 0]
    np.testing.assert_allclose(got, u, rtol=0, atol=1e-12 * np.abs(u).max())
    # one degree too many is not reproduced on the interface (the pin has teeth)
    if p >= 1:
        c2 = [np.concatenate([c, [1.0]]) for c in coefs]
        u2 = poly_field(c2, x)
        assert np.abs(orc.distribute(np.where(orc.hanging, 0.0, u2)[:, None])[:, 0] - u2).max() > 1e-6


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("p", [2, 3])
def test_constrained_bilinear_form_is_exact(mesh, p):
    mu, sigma = 0.75, 0.4
    rm = RefinedMesh(mesh["n"], LO, HI, mesh["rlo"], mesh["rhi"])
    orc = RefinedOracle(rm, p, p + 1, mu, None, sigma)
    x = node_coords(orc)
    rng = np.random.default_rng(10 + p)
    cu = [rng.standard_normal(p + 1) for _ in range(3)]
    cw = [rng.standard_normal(p + 1) for _ in range(3)]
    U = np.where(orc.hanging, -7.0, poly_field(cu, x))
    W = np.where(orc.hanging, 0.0, poly_field(cw, x))
    Y = orc.apply_constrained(U[:, None])[:, 0]
    assert np.all(Y[orc.hanging] == 0.0)
    want = exact_forms(cu, cw, mu, sigma)
    assert abs(W @ Y - want) <= 1e-11 * max(1.0, abs(want))


@pytest.mark.parametrize("p", [2, 3])
def test_dirichlet_bilinear_form_is_exact(p):
    mu, sigma = 1.3, 0.0
    m = MESHES[0]
    rm = RefinedMesh(m["n"], LO, HI, m["rlo"], m["rhi"], bc=BC_DIRICHLET0)
    orc = RefinedOracle(rm, p, p + 1, mu, None, sigma)
    x = node_coords(orc)
    # fields vanishing on the boundary: x_d (L_d - x_d) times a degree p-2 factor
    rng = np.random.default_rng(20 + p)

    def bubble(d):
        return P.polymul([0.0, HI[d], -1.0], rng.standard_normal(p - 1))
    cu = [bubble(d) for d in range(3)]
    cw = [bubble(d) for d in range(3)]
    U = poly_field(cu, x)
    W = poly_field(cw, x)
    Y = orc.apply_constrained(U[:, None])[:, 0]
    assert np.all(Y[orc.constrained] == 0.0) and np.all(Y[orc.hanging] == 0.0)
    want = exact_forms(cu, cw, mu, sigma)
    assert abs(W @ Y - want) <= 1e-11 * max(1.0, abs(want))


@pytest.mark.parametrize("p", [1, 2])
def test_constrained_stiffness_symmetric_with_constant_null_space(p):
    m = MESHES[0]
    rm = RefinedMesh(m["n"], LO, HI, m["rlo"], m["rhi"])
    orc = RefinedOracle(rm, p, p + 1, 1.0)
    A = orc.apply_constrained(np.eye(orc.ndofs))
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-12)
    free = ~orc.hanging
    ev = np.linalg.eigvalsh(A[np.ix_(free, free)])
    assert ev[0] > -1e-10
    assert np.sum(ev < 1e-9 * ev[-1]) == 1                  # only the constants
    ones = np.where(orc.hanging, 0.0, 1.0)
    assert np.abs(orc.apply_constrained(ones[:, None])).max() < 1e-12


# ------------------------------------------------- eigenproblem on the refined mesh
def test_constrained_lumped_mass_volume_and_uniform_limit():
    rm = RefinedMesh([3, 3, 3], LO, HI, [1, 1, 1], [2, 2, 2])
    orc = RefinedOracle(rm, 3, 4, 0.5)
    m = orc.lumped_mass_constrained()
    assert abs(m.sum() - np.prod(np.subtract(HI, LO))) < 1e-13      # rows of C sum to one
    assert np.all(m[orc.hanging] == 0.0) and np.all(m[~orc.hanging] > 0.0)
    box = BoxMesh([3, 2, 2], LO, HI, BC_DIRICHLET0)
    empty = RefinedMesh([3, 2, 2], LO, HI, [1, 0, 0], [1, 2, 2], bc=BC_DIRICHLET0)
    np.testing.assert_allclose(RefinedOracle(empty, 3, 4, 0.5).lumped_mass_constrained(),
                               fo.Oracle(box, 3, 4, 0.5).lumped_mass(), rtol=0, atol=1e-15)


@pytest.mark.parametrize("p,tol", [(3, 1e-4), (4, 1e-6)])
def test_lowest_dirichlet_eigenvalue_on_refined_mesh(p, tol):
    """Standard form D C^T A_u C D (D = m_c^{-1/2}) of (1/2) K on the box with zero Dirichlet:
    the lowest eigenvalue converges to (1/2) pi^2 sum_d L_d^-2."""
    rm = RefinedMesh([3, 3, 3], LO, HI, [1, 1, 1], [2, 2, 2], bc=BC_DIRICHLET0)
    orc = RefinedOracle(rm, p, p + 1, 0.5)
    m = orc.lumped_mass_constrained()
    free = m > 0
    D = np.zeros_like(m)
    D[free] = 1.0 / np.sqrt(m[free])
    S = orc.cheb_step_constrained(D, np.eye(orc.ndofs)[:, free], None, 1.0, 0.0, 0.0)[free]
    lam = np.linalg.eigvalsh(0.5 * (S + S.T))[0]
    exact = 0.5 * np.pi ** 2 * sum(1.0 / (HI[d] - LO[d]) ** 2 for d in range(3))
    assert abs(lam - exact) <= tol * exact
