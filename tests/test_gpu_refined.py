"""GPU parity of hanging-node constraints on once-refined box meshes
(include/mfrefine.h) against the FP64 hanging-node oracle.

- Small meshes (several degrees, both boundary conditions, refined blocks in
  the core, on the boundary, everything and nothing refined, 1 to 70 columns,
  so the 64-column tiles have a ragged tail): C (distribute), A_u (mf_apply on
  the refined map), C^T (condense) and the composition, element by element,
  relative error <= 1e-12 per column.
- The full refined workload (12^3 coarse cells, central 6^3 refined, p = 6,
  64 columns, the launch the benchmark times) on sampled rows that include
  interface masters and hanging rows; the closed-form bilinear form of two
  degree-6 polynomials vanishing on the boundary; the adjoint identity
  <C^T Y, Z> = <Y, C Z> over every set; the symmetry of C^T A_u C.
- The eigenproblem on the constrained space: the row-lumped mass C^T m_u and its
  inverse square root (1e-13), the Chebyshev step a D C^T A_u C D Y + b Y + c X
  (Xp absent, separate, in place), and Chebyshev-filtered subspace iteration
  against a dense eigen-solve of the oracle's standard form.
- The grid-based calls refuse a refined operator.
"""
import ctypes

import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import workloads as W
from oracle.hanging_oracle import RefinedOracle, refined_layout
from paper_2208_07129_amd import mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def dev():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def vfun(x):
    return np.sin(x[..., 0]) + x[..., 1] * x[..., 2] - 0.3


def colrel(Y, R):
    den = np.maximum(np.linalg.norm(R, axis=0), 1e-300)
    return float((np.linalg.norm(Y - R, axis=0) / den).max())


LO, HI = (0.0, -0.5, 0.25), (1.0, 1.0, 1.5)
CASES = [  # p, n, rlo, rhi, bc, nvec
    (1, (3, 3, 3), (1, 1, 1), (2, 2, 2), W.BC_NONE, 130),           # no cell-interior rows
    (2, (3, 3, 3), (1, 1, 1), (2, 2, 2), W.BC_DIRICHLET0, 5),
    (3, (4, 3, 2), (0, 1, 0), (2, 3, 1), W.BC_NONE, 70),
    (4, (3, 3, 2), (1, 0, 0), (3, 2, 1), W.BC_DIRICHLET0, 1),
    (6, (3, 2, 2), (1, 0, 1), (2, 1, 2), W.BC_NONE, 64),
    (6, (2, 2, 2), (0, 0, 0), (2, 2, 2), W.BC_DIRICHLET0, 8),     # everything refined
    (5, (2, 2, 2), (1, 1, 1), (1, 2, 2), W.BC_NONE, 4),           # nothing refined
    (8, (2, 2, 1), (1, 1, 0), (2, 2, 1), W.BC_DIRICHLET0, 3),
]


@pytest.mark.parametrize("p,n,rlo,rhi,bc,nvec", CASES)
def test_constraints_and_apply_match_oracle(p, n, rlo, rhi, bc, nvec):
    print(f"refined case p={p} n={n} box=[{rlo},{rhi}) bc={bc} nvec={nvec}", flush=True)
    rm = W.RefinedMesh(n, LO, HI, rlo, rhi, bc)
    q = p + 1
    op = mfmv.RefinedOperator(rm, p, q, 0.5, vfun(mfmv.refined_quad_points(rm, q)), 0.2)
    orc = RefinedOracle(rm, p, q, 0.5, vfun, 0.2)
    assert op.ndofs == orc.ndofs
    rng = np.random.default_rng(p * 1000 + nvec)
    X = rng.uniform(-1, 1, (orc.ndofs, nvec))
    # C: hanging rows replaced, every other row untouched
    Xd = T(X)
    op.distribute(Xd)
    np.testing.assert_array_equal(Xd.cpu().numpy()[~orc.hanging], X[~orc.hanging])
    assert colrel(Xd.cpu().numpy(), orc.distribute(X)) <= TOL
    # A_u on the distributed multivector
    Y = op.apply(Xd)
    Yref = orc.apply(orc.distribute(X))
    assert colrel(Y.cpu().numpy(), Yref) <= TOL
    # C^T in place (zero-Dirichlet rows were written 0 by the apply)
    op.condense(Y)
    assert colrel(Y.cpu().numpy(), orc.condense(Yref)) <= TOL
    assert colrel(Y.cpu().numpy(), orc.apply_constrained(X)) <= TOL
    # C^T of an arbitrary multivector leaves zero-Dirichlet rows unchanged
    R = rng.uniform(-1, 1, (orc.ndofs, nvec))
    Rd = T(R)
    op.condense(Rd)
    got = Rd.cpu().numpy()
    want = orc.condense(R)
    free = ~orc.constrained
    assert colrel(got[free], want[free]) <= TOL
    np.testing.assert_array_equal(got[orc.constrained], R[orc.constrained])
    # the one-call product (zero fill and C fused) and the three-call sequence
    for steps in (False, True):
        Xc = T(X)
        Yc = op.apply_constrained(Xc, steps=steps)
        assert colrel(Yc.cpu().numpy(), orc.apply_constrained(X)) <= TOL
        np.testing.assert_allclose(Xc.cpu().numpy(), orc.distribute(X), rtol=0, atol=1e-13)


SHEAR = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])


@pytest.mark.parametrize("p,general,lin", [(3, True, None), (6, True, None), (4, False, SHEAR),
                                           (2, False, SHEAR)])
def test_general_kernel_and_sheared_cells(p, general, lin):
    """The general-geometry kernel (forced, or chosen for sheared cells) on a refined map."""
    print(f"refined general p={p} forced={general} sheared={lin is not None}", flush=True)
    rm = W.RefinedMesh((3, 3, 2), LO, HI, (1, 0, 0), (3, 2, 1), W.BC_DIRICHLET0, lin)
    q = p + 1
    op = mfmv.RefinedOperator(rm, p, q, 0.5, vfun(mfmv.refined_quad_points(rm, q)), 0.2)
    if general:
        op.set_launch(general=True)
    orc = RefinedOracle(rm, p, q, 0.5, vfun, 0.2)
    X = np.random.default_rng(p).uniform(-1, 1, (orc.ndofs, 6))
    Y = op.apply_constrained(T(X)).cpu().numpy()
    assert colrel(Y, orc.apply_constrained(X)) <= TOL
    # accumulate form: Y + A_u X
    Xd = T(orc.distribute(X))
    Y0 = np.random.default_rng(p + 1).uniform(-1, 1, X.shape)
    Ya = op.apply(Xd, T(Y0), accumulate=True).cpu().numpy()
    want = Y0 + orc.apply(orc.distribute(X))
    free = ~orc.constrained
    assert colrel(Ya[free], want[free]) <= TOL


@pytest.mark.parametrize("p,nvec", [(2, 5), (4, 16), (6, 64), (8, 3)])
def test_fp32_apply_on_refined_map(p, nvec):
    """FP32 cell arrays through the map: per-column relative error <= 1e-6 against the
    FP64 oracle, with column magnitudes from 1e-30 to 1e30 (power-of-two scaling)."""
    print(f"refined fp32 p={p} nvec={nvec}", flush=True)
    rm = W.RefinedMesh((3, 2, 2), LO, HI, (1, 0, 0), (2, 2, 1), W.BC_DIRICHLET0)
    q = p + 1
    op = mfmv.RefinedOperator(rm, p, q, 0.5, vfun(mfmv.refined_quad_points(rm, q)), 0.2)
    orc = RefinedOracle(rm, p, q, 0.5, vfun, 0.2)
    rng = np.random.default_rng(300 + p)
    X = rng.uniform(-1, 1, (orc.ndofs, nvec)) * np.logspace(-30, 30, nvec)[None, :]
    Xd = orc.distribute(X)
    Y = op.apply(T(Xd), precision="fp32").cpu().numpy()
    assert colrel(Y, orc.apply(Xd)) <= 1e-6
    # the accumulating form
    Ya = op.apply(T(Xd), T(np.zeros_like(Xd)), precision="fp32", accumulate=True).cpu().numpy()
    free = ~orc.constrained
    assert colrel(Ya[free], orc.apply(Xd)[free]) <= 1e-6


@pytest.mark.parametrize("q", [11, 12])
def test_degree_10(q):
    """The largest degree: FP64 (B = 4 map tiles), FP32, and the constraint kernels
    with 121 masters per set."""
    print(f"refined p=10 q={q}", flush=True)
    rm = W.RefinedMesh((2, 1, 1), LO, HI, (1, 0, 0), (2, 1, 1), W.BC_NONE)
    op = mfmv.RefinedOperator(rm, 10, q, 0.5, vfun(mfmv.refined_quad_points(rm, q)), 0.2)
    orc = RefinedOracle(rm, 10, q, 0.5, vfun, 0.2)
    X = np.random.default_rng(q).uniform(-1, 1, (orc.ndofs, 5))
    want = orc.apply_constrained(X)
    assert colrel(op.apply_constrained(T(X)).cpu().numpy(), want) <= TOL
    if q == 11:
        Xd = orc.distribute(X)
        assert colrel(op.apply(T(Xd), precision="fp32").cpu().numpy(), orc.apply(Xd)) <= 1e-6


def test_constrained_call_on_uniform_operator_is_the_apply():
    mesh = W.BoxMesh(n=(3, 2, 2), lo=LO, hi=HI, bc=W.BC_DIRICHLET0)
    op = mfmv.Operator(mesh, 3, 4, 0.5, None, 0.3)
    X = T(np.random.default_rng(9).uniform(-1, 1, (op.ndofs, 6)))
    X0 = X.clone()
    Y = torch.empty_like(X)
    rc = mfmv.lib().mf_apply_constrained(op._h, X.data_ptr(), Y.data_ptr(), 6, 6, 6, None)
    assert rc == mfmv.MF_OK
    Yr = op.apply(X0)
    torch.cuda.synchronize()
    assert torch.equal(X, X0)                     # no constraint sets: X untouched
    assert colrel(Y.cpu().numpy(), Yr.cpu().numpy()) <= TOL


def test_strided_single_column():
    rm = W.RefinedMesh((3, 3, 3), LO, HI, (1, 1, 1), (2, 2, 2), W.BC_NONE)
    op = mfmv.RefinedOperator(rm, 3, 4, 0.5, None, 0.1)
    orc = RefinedOracle(rm, 3, 4, 0.5, None, 0.1)
    X = np.random.default_rng(5).uniform(-1, 1, (orc.ndofs, 3))
    big = T(X)
    col = big[:, 1:2]                     # ld = 3, nvec = 1
    op.distribute(col)
    np.testing.assert_allclose(big.cpu().numpy()[:, 1], orc.distribute(X[:, 1:2])[:, 0],
                               rtol=0, atol=1e-13)
    np.testing.assert_array_equal(big.cpu().numpy()[:, [0, 2]], X[:, [0, 2]])


def _full_operator(with_v=True):
    w = W.refined_config()
    op = mfmv.RefinedOperator.from_workload(w) if with_v else \
        mfmv.RefinedOperator(w.mesh, w.p, w.q, w.mu, None, 0.35)
    return w, op


def test_full_size_sampled_rows():
    w, op = _full_operator()
    print(f"full refined workload ndofs={op.ndofs} sets={op.nsets}", flush=True)
    orc = RefinedOracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    X = w.X(op.ndofs)
    Xd = T(X)
    Y = op.apply_constrained(Xd).cpu().numpy()
    rng = np.random.default_rng(77)
    CT = orc.C.T.tocsr()
    masters = np.unique(orc.C[orc.hanging].indices)
    rows = np.concatenate([rng.choice(op.ndofs, 6, replace=False),
                           rng.choice(masters, 6, replace=False),
                           rng.choice(np.nonzero(orc.hanging)[0], 2, replace=False),
                           np.nonzero(orc.constrained)[0][:2]])
    S = CT[rows]                                      # rows of C^T
    needed = np.unique(S.indices)
    CX = orc.C @ X
    Yn = orc.apply(CX, cells=orc.cells_touching(needed))[needed]
    ref = S[:, needed] @ Yn
    scale = np.abs(ref).max()
    assert np.abs(Y[rows] - ref).max() <= 1e-12 * scale
    assert np.all(Y[orc.hanging] == 0.0) and np.all(Y[orc.constrained] == 0.0)


def test_full_size_bilinear_form_of_polynomials():
    w, op = _full_operator(with_v=False)
    mu, sigma = w.mu, 0.35
    lay = refined_layout(w.mesh, w.p)
    lo, hi = np.asarray(w.mesh.lo, float), np.asarray(w.mesh.hi, float)
    L = hi - lo
    t = lay["pos"] / np.asarray(w.mesh.n, float)      # node coordinates scaled to [0, 1]
    rng = np.random.default_rng(31)

    def bubble():  # t (1 - t) r(t), r of degree p - 2: zero on the boundary, degree p
        return P.polymul([0.0, 1.0, -1.0], rng.standard_normal(w.p - 1))
    cu = [bubble() for _ in range(3)]
    cv = [bubble() for _ in range(3)]
    U = np.prod([P.polyval(t[:, d], cu[d]) for d in range(3)], axis=0)
    V = np.prod([P.polyval(t[:, d], cv[d]) for d in range(3)], axis=0)
    hang = lay["kind"] == 2
    Ud = T(np.where(hang, 0.0, U)[:, None])
    Y = op.apply_constrained(Ud).cpu().numpy()[:, 0]
    # C reproduced the polynomial at every hanging node
    np.testing.assert_allclose(Ud.cpu().numpy()[:, 0], U, rtol=0, atol=1e-12 * np.abs(U).max())

    def integ01(c):
        ci = P.polyint(c)
        return P.polyval(1.0, ci) - P.polyval(0.0, ci)
    # x = lo + L t: int f g dx = L int f g dt, d/dx = (1/L) d/dt
    mass = [L[d] * integ01(P.polymul(cu[d], cv[d])) for d in range(3)]
    grad = [integ01(P.polymul(P.polyder(cu[d]), P.polyder(cv[d]))) / L[d] for d in range(3)]
    want = mu * sum(grad[d] * np.prod([mass[e] for e in range(3) if e != d]) for d in range(3)) \
        + sigma * np.prod(mass)
    got = float(np.where(hang, 0.0, V) @ Y)
    assert abs(got - want) <= 1e-11 * abs(want)


def test_full_size_adjoint_and_symmetry():
    w, op = _full_operator()
    rng = np.random.default_rng(41)
    nvec = 8
    Yh = rng.uniform(-1, 1, (op.ndofs, nvec))
    Zh = rng.uniform(-1, 1, (op.ndofs, nvec))
    # <C^T Y, Z> = <Y, C Z> with C Z the distributed Z (every row but the hanging kept)
    cty = op.condense(T(Yh)).cpu().numpy()
    cz = op.distribute(T(Zh)).cpu().numpy()
    _, kind = mfmv.refined_layout(w.mesh, w.p)
    cz[kind == 1] = 0.0                     # C has empty zero-Dirichlet rows
    cty[kind == 1] = 0.0
    lhs = np.einsum("ij,ij->j", cty, Zh)
    rhs = np.einsum("ij,ij->j", Yh, cz)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)
    # symmetry of C^T A_u C
    U = rng.uniform(-1, 1, (op.ndofs, nvec))
    V = rng.uniform(-1, 1, (op.ndofs, nvec))
    AU = op.apply_constrained(T(U)).cpu().numpy()
    AV = op.apply_constrained(T(V)).cpu().numpy()
    hang = kind == 2
    U[hang] = 0.0
    V[hang] = 0.0
    np.testing.assert_allclose(np.einsum("ij,ij->j", V, AU), np.einsum("ij,ij->j", U, AV),
                               rtol=1e-11)


def test_grid_calls_refuse_refined_operator():
    rm = W.RefinedMesh((2, 2, 2), LO, HI, (0, 0, 0), (1, 1, 1), W.BC_NONE)
    op = mfmv.RefinedOperator(rm, 2, 3)
    L = mfmv.lib()
    buf = torch.zeros((op.ndofs, 2), dtype=torch.float64, device=dev())
    p = buf.data_ptr()
    assert L.mf_diagonal(op._h, p, None) == mfmv.MF_ERR_UNSUPPORTED
    out = torch.zeros_like(buf)
    assert L.mf_cheb_step(op._h, p, p, None, out.data_ptr(), 2, 2, 1.0, 0.0, 0.0,
                          None) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_apply(op._h, p, out.data_ptr(), 2, 2, 2, mfmv.MF_BF16,
                      None) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_apply_constrained(op._h, p, p, 2, 2, 2, None) == mfmv.MF_ERR_ARG  # overlap
    nv = (ctypes.c_int * 1)(2)
    hs = (ctypes.c_void_p * 1)(op._h)
    b = ctypes.c_void_p()
    assert L.mf_batch_create(1, hs, nv, 0, ctypes.byref(b)) == mfmv.MF_ERR_UNSUPPORTED
    torch.cuda.synchronize()


# ------------------------------------------- eigenproblem on the refined mesh (Alg. ChFSi)
@pytest.mark.parametrize("p,bc,lin", [(3, W.BC_DIRICHLET0, None), (4, W.BC_NONE, None),
                                      (6, W.BC_DIRICHLET0, None), (2, W.BC_DIRICHLET0, SHEAR)])
def test_lumped_mass_and_cheb_step_on_refined_mesh(p, bc, lin):
    """Axis-aligned cells take the D-scaled map kernel; sheared cells the composed path."""
    print(f"refined cheb p={p} bc={bc} sheared={lin is not None}", flush=True)
    rm = W.RefinedMesh((3, 2, 2), LO, HI, (1, 0, 0), (2, 2, 1), bc, lin)
    q = p + 1
    op = mfmv.RefinedOperator(rm, p, q, 0.5, vfun(mfmv.refined_quad_points(rm, q)), 0.2)
    orc = RefinedOracle(rm, p, q, 0.5, vfun, 0.2)
    m_ref = orc.lumped_mass_constrained()
    np.testing.assert_allclose(mfmv.gll_mass(op).cpu().numpy(), m_ref, rtol=1e-13, atol=0)
    D = mfmv.gll_mass(op, inv_sqrt=True)
    Dr = np.zeros_like(m_ref)
    Dr[m_ref > 0] = 1.0 / np.sqrt(m_ref[m_ref > 0])
    np.testing.assert_allclose(D.cpu().numpy(), Dr, rtol=1e-13, atol=0)
    rng = np.random.default_rng(40 + p)
    nvec = 6
    Y = rng.uniform(-1, 1, (orc.ndofs, nvec))
    Xp = rng.uniform(-1, 1, (orc.ndofs, nvec))
    a, b, c = 1.3, -0.4, 0.25
    for xp_mode in ("none", "separate", "in place"):
        Out = T(Xp.copy()) if xp_mode == "in place" else torch.empty((orc.ndofs, nvec),
                                                                     dtype=torch.float64,
                                                                     device=dev())
        Xd = None if xp_mode == "none" else (Out if xp_mode == "in place" else T(Xp))
        mfmv.cheb_step(op, D, T(Y), Xd, Out, a, b, c)
        want = orc.cheb_step_constrained(Dr, Y, None if xp_mode == "none" else Xp, a, b, c)
        assert colrel(Out.cpu().numpy(), want) <= TOL, xp_mode


def test_subspace_iteration_on_refined_mesh():
    """Chebyshev-filtered subspace iteration on the constrained space of a refined mesh
    against a dense eigen-solve of the oracle's standard form D C^T A_u C D."""
    from paper_2208_07129_amd.chebyshev import SubspaceIteration
    rm = W.RefinedMesh((3, 3, 3), (0, 0, 0), (3.0, 3.0, 3.0), (1, 1, 1), (2, 2, 2),
                       W.BC_DIRICHLET0)
    Vf = W.gaussian_wells(8, L=3.0, k=3, width=0.6)
    op = mfmv.RefinedOperator(rm, 3, 4, 0.5, Vf(mfmv.refined_quad_points(rm, 4)), 0.0)
    orc = RefinedOracle(rm, 3, 4, 0.5, Vf, 0.0)
    m = orc.lumped_mass_constrained()
    free = m > 0
    Dr = np.zeros_like(m)
    Dr[free] = 1.0 / np.sqrt(m[free])
    S = orc.cheb_step_constrained(Dr, np.eye(orc.ndofs)[:, free], None, 1.0, 0.0, 0.0)[free]
    ref = np.linalg.eigvalsh(0.5 * (S + S.T))
    k, nev = 16, 10
    U0 = np.random.default_rng(2).uniform(-1, 1, (orc.ndofs, k))
    U0[~free] = 0.0
    si = SubspaceIteration(op, k)
    out = si.solve(T(U0), nev, degree=12, tol=2e-7, maxit=60)
    print(out["iterations"], out["residual"])
    assert out["converged"], out["history"][-5:]
    np.testing.assert_allclose(out["eigenvalues"], ref[:nev], rtol=0,
                               atol=1e-9 * max(1.0, abs(ref[:nev]).max()))
