"""GPU parity of the Chebyshev-filter building blocks (include/mfcheb.h)
against the FP64 CPU oracle.

- mf_gll_mass: the lumped mass diagonal and its inverse square root (1e-13).
- mf_cheb_step: a D A (D Y) + b Y + c Xp on small meshes of every boundary
  condition and several degrees, with Xp absent, separate, and the output
  itself (the in-place recurrence); per-column relative error <= 1e-12.
- Config 2 (16^3, p = 6, 64 columns) on sampled rows, in place.
- The standard-form matrix D A D is symmetric (u^T S v = v^T S u).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fe_oracle as fo
from paper_2208_07129_amd import mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def vfun(x):
    return np.sin(x[..., 0]) + x[..., 1] * x[..., 2] - 0.3


def colrel(Y, R):
    return float((np.linalg.norm(Y - R, axis=0) / np.linalg.norm(R, axis=0)).max())


# the periodic and free one-cell directions check that every face row has one
# owner cell when Out is not Xp (a periodic cell meets itself; the last cell of
# a free direction owns its far face)
CASES = [(2, 3, (3, 2, 2), W.BC_DIRICHLET0, 5), (3, 4, (2, 2, 3), W.BC_PERIODIC, 8),
         (4, 5, (2, 2, 2), W.BC_NONE, 3), (6, 7, (2, 2, 2), W.BC_PERIODIC, 16),
         (8, 9, (2, 1, 1), W.BC_DIRICHLET0, 9), (3, 4, (1, 2, 3), W.BC_PERIODIC, 7),
         (5, 6, (3, 1, 2), W.BC_NONE, 11), (6, 7, (1, 1, 1), W.BC_PERIODIC, 8)]


@pytest.mark.parametrize("p,q,n,bc,nvec", CASES)
def test_gll_mass_and_cheb_step_match_oracle(p, q, n, bc, nvec):
    mesh = W.BoxMesh(n=n, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc)
    op = mfmv.Operator(mesh, p, q, 0.5, vfun(mfmv.quad_points(mesh, q)), 0.2)
    orc = fo.Oracle(mesh, p, q, 0.5, vfun, 0.2)
    m_ref = orc.lumped_mass()
    m = mfmv.gll_mass(op).cpu().numpy()
    np.testing.assert_allclose(m, m_ref, rtol=1e-13, atol=0)
    D = mfmv.gll_mass(op, inv_sqrt=True)
    free = ~orc.constrained
    D_ref = np.zeros_like(m_ref)
    D_ref[free] = 1.0 / np.sqrt(m_ref[free])
    np.testing.assert_allclose(D.cpu().numpy(), D_ref, rtol=1e-13, atol=0)
    rng = np.random.default_rng(p * 100 + nvec)
    Y = rng.uniform(-1, 1, (orc.ndofs, nvec))
    Xp = rng.uniform(-1, 1, (orc.ndofs, nvec))
    a, b, c = 1.7, -0.6, 0.35
    for mode in ("none", "separate", "inplace"):
        Yd = T(Y)
        Out = T(Xp) if mode == "inplace" else torch.full_like(Yd, float("nan"))
        Xd = None if mode == "none" else (Out if mode == "inplace" else T(Xp))
        mfmv.cheb_step(op, D, Yd, Xd, Out, a, b, c)
        torch.cuda.synchronize()
        ref = orc.cheb_step(D_ref, Y, None if mode == "none" else Xp, a, b, c)
        assert colrel(Out.cpu().numpy(), ref) <= 1e-12, mode
        assert np.all(Out.cpu().numpy()[orc.constrained] == 0.0)


def test_cheb_step_rejects_bad_arguments():
    mesh = W.BoxMesh(n=(2, 2, 2), bc=W.BC_PERIODIC)
    op = mfmv.Operator(mesh, 2, 3, 0.5, None, 0.0)
    D = mfmv.gll_mass(op, inv_sqrt=True)
    Y = torch.zeros((op.ndofs, 4), dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        mfmv.cheb_step(op, D, Y, None, Y, 1.0, 0.0, 0.0)     # Out overlaps Y
    assert e.value.status == mfmv.MF_ERR_ARG
    sheared = W.BoxMesh(n=(2, 2, 2), bc=W.BC_NONE,
                        lin=np.array([[1.0, 0.3, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    op2 = mfmv.Operator(sheared, 2, 3, 0.5, None, 0.0)
    with pytest.raises(mfmv.MfError) as e:
        mfmv.gll_mass(op2)
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED


def test_standard_form_is_symmetric():
    w = W.config2()
    w.nvec = 2
    op = mfmv.Operator.from_workload(w)
    D = mfmv.gll_mass(op, inv_sqrt=True)
    rng = np.random.default_rng(3)
    U = T(rng.standard_normal((op.ndofs, 2)))
    S = torch.empty_like(U)
    mfmv.cheb_step(op, D, U, None, S, 1.0, 0.0, 0.0)
    uSv = float((U[:, 0] * S[:, 1]).sum())
    vSu = float((U[:, 1] * S[:, 0]).sum())
    assert abs(uSv - vSu) <= 1e-12 * float(S.abs().max()) * op.ndofs ** 0.5


@pytest.mark.parametrize("in_place", [True, False])
def test_config2_cheb_step_sampled_rows(in_place):
    """Config 2 at full size, in place (face rows initialised to b Y + c Xp) and
    into a separate array (face rows zeroed, b Y + c Xp added by the owner cell),
    on sampled rows that include cell-face rows."""
    w = W.config2()
    op = mfmv.Operator.from_workload(w)
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    m_ref = orc.lumped_mass()
    D = mfmv.gll_mass(op, inv_sqrt=True)
    np.testing.assert_allclose(D.cpu().numpy(), 1.0 / np.sqrt(m_ref), rtol=1e-13, atol=0)
    Y = w.X()
    Xp = np.random.default_rng(7).uniform(-1, 1, Y.shape)
    a, b, c = 0.9, 0.25, -0.5
    Out = T(Xp) if in_place else torch.full((orc.ndofs, Y.shape[1]), float("nan"),
                                            dtype=torch.float64, device=dev())
    mfmv.cheb_step(op, D, T(Y), Out if in_place else T(Xp), Out, a, b, c)
    N = 16 * w.p   # periodic 16^3 cells: a node on a cell face has a coordinate index divisible by p
    face = [int(i + N * (j + N * k)) for i, j, k in ((0, 3, 5), (6, 12, 1), (6, 12, 90),
                                                   (12, 18, 24), (95, 0, 7))]
    rows = np.concatenate([np.random.default_rng(11).choice(orc.ndofs, 12, replace=False), face])
    Dr = 1.0 / np.sqrt(m_ref)
    ref = a * Dr[rows, None] * orc.apply_rows(Dr[:, None] * Y, rows) + b * Y[rows] + c * Xp[rows]
    got = Out[torch.from_numpy(rows).to(dev())].cpu().numpy()
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-12, rel


def test_chebyshev_filter_matches_oracle_polynomial():
    """The library's filter (scaled three-term steps) against the oracle's p_m(H~) U,
    computed from the plain Chebyshev recurrence and one final normalisation."""
    from paper_2208_07129_amd.chebyshev import chebyshev_filter
    mesh = W.BoxMesh(n=(2, 2, 2), lo=(0, 0, 0), hi=(2.0, 2.0, 2.0), bc=W.BC_PERIODIC)
    op = mfmv.Operator(mesh, 4, 5, 0.5, vfun(mfmv.quad_points(mesh, 5)), 0.0)
    orc = fo.Oracle(mesh, 4, 5, 0.5, vfun, 0.0)
    D_ref = 1.0 / np.sqrt(orc.lumped_mass())
    D = mfmv.gll_mass(op, inv_sqrt=True)
    U = np.random.default_rng(5).standard_normal((orc.ndofs, 6))
    m, lmin, lmax, lu = 7, -2.0, 60.0, 5.0
    Ud = T(U)
    Yd = chebyshev_filter(op, D, Ud, m, lmin, lmax, lu)
    torch.cuda.synchronize()
    assert np.array_equal(Ud.cpu().numpy(), U)        # the input is left unmodified
    ref = orc.chebyshev_filter(D_ref, U, m, lmin, lmax, lu)
    assert colrel(Yd.cpu().numpy(), ref) <= 1e-11


@pytest.mark.parametrize("k", [1, 2, 5, 33, 64, 65, 96, 128, 200, 320])
def test_sym_eig_matches_numpy(k):
    """Small blocks take the one-workgroup Jacobi kernel, k > 64 the block
    Jacobi method (padded to a multiple of 64 at k = 65, 200).  Both this and
    LAPACK are backward stable: each eigenvalue is within c k eps ||A|| of the
    exact one, so the bound grows with k (at least 1e-13 ||A||)."""
    rng = np.random.default_rng(k)
    Z = rng.standard_normal((k, k))
    A = Z + Z.T
    w, V, st = mfmv.sym_eig(T(A))
    assert int(st.item()) == 0
    wh, Vh = w.cpu().numpy(), V.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    eps = np.finfo(np.float64).eps
    scale = max(1e-13, 4 * k * eps)
    np.testing.assert_allclose(wh, ref, rtol=0, atol=scale * np.abs(ref).max())
    assert np.abs(A @ Vh - Vh * wh).max() <= 10 * scale * np.abs(ref).max()
    assert np.abs(Vh.T @ Vh - np.eye(k)).max() <= scale
    # the orthonormalising factor of an SPD block, and the status of an indefinite one
    Gs = Z @ Z.T + k * np.eye(k)
    _, Mh, st = mfmv.sym_eig(T(Gs), vpow=-0.5)
    assert int(st.item()) == 0
    Mh = Mh.cpu().numpy()
    np.testing.assert_allclose(Mh.T @ Gs @ Mh, np.eye(k), rtol=0, atol=1e-12)
    if k > 1:
        _, _, st = mfmv.sym_eig(T(A), vpow=-0.5)
        assert int(st.item()) == 2


def test_sym_eig_block_jacobi_on_clustered_and_diagonal_blocks():
    """k = 384: a clustered spectrum (cubes of uniform numbers, the shape of a
    Rayleigh-Ritz block near convergence) in a random orthonormal basis, and a
    block that is diagonal already (no sweep), with a strided A and V."""
    k = 384
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    lam = np.sort(rng.random(k)) ** 3
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    Ab = torch.zeros((k, k + 3), dtype=torch.float64, device=dev())
    Ab[:, :k] = T(A)
    Vb = torch.zeros((k, k + 5), dtype=torch.float64, device=dev())
    w, V, st = mfmv.sym_eig(Ab[:, :k], V=Vb[:, :k])
    assert int(st.item()) == 0
    wh, Vh = w.cpu().numpy(), V.cpu().numpy()
    tol = 4 * k * np.finfo(np.float64).eps  # ||A|| < 1
    np.testing.assert_allclose(wh, np.linalg.eigvalsh(A), rtol=0, atol=tol)
    assert np.abs(A @ Vh - Vh * wh).max() <= 10 * tol
    assert np.abs(Vh.T @ Vh - np.eye(k)).max() <= tol
    d = rng.standard_normal(200)
    w, V, st = mfmv.sym_eig(T(np.diag(d)))
    assert int(st.item()) == 0
    assert np.array_equal(w.cpu().numpy(), np.sort(d))
    assert np.array_equal(np.abs(V.cpu().numpy()), np.eye(200)[np.argsort(d)].T)


def test_sym_eig_rejects_large_blocks_and_short_work():
    with pytest.raises(mfmv.MfError) as e:
        mfmv.sym_eig(torch.eye(2049, dtype=torch.float64, device=dev()))
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED
    short = torch.empty(10, dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        mfmv.sym_eig(torch.eye(100, dtype=torch.float64, device=dev()), work=short)
    assert e.value.status == mfmv.MF_ERR_ARG


@pytest.mark.parametrize("bc,k,nev,tol", [(W.BC_PERIODIC, 16, 10, 2e-7),
                                          (W.BC_DIRICHLET0, 16, 10, 2e-7),
                                          (W.BC_PERIODIC, 96, 72, 1e-6)])
def test_subspace_iteration_finds_the_lowest_eigenpairs(bc, k, nev, tol):
    """Chebyshev-filtered subspace iteration against a dense eigen-solve of the
    oracle's standard-form matrix: the nev lowest eigenvalues to 1e-9 once every
    residual norm is below tol (k = 96: the block-Jacobi eigen-solver in the
    orthogonalisation and Rayleigh-Ritz steps; its wanted eigenvalues reach ~50,
    where the residual estimate resolves ~1e-8 |theta|, hence the looser tol)."""
    from paper_2208_07129_amd.chebyshev import SubspaceIteration
    mesh = W.BoxMesh(n=(3, 3, 3), lo=(0, 0, 0), hi=(3.0, 3.0, 3.0), bc=bc)
    Vf = W.gaussian_wells(8, L=3.0, k=3, width=0.6)
    op = mfmv.Operator(mesh, 3, 4, 0.5, Vf(mfmv.quad_points(mesh, 4)), 0.0)
    orc = fo.Oracle(mesh, 3, 4, 0.5, Vf, 0.0)
    free = ~orc.constrained
    m = orc.lumped_mass()
    Dr = np.zeros_like(m)
    Dr[free] = 1.0 / np.sqrt(m[free])
    S = Dr[:, None] * orc.assemble_dense() * Dr[None, :]
    ref = np.linalg.eigvalsh(S[np.ix_(free, free)])
    U0 = np.random.default_rng(2).uniform(-1, 1, (orc.ndofs, k))
    U0[orc.constrained] = 0.0
    si = SubspaceIteration(op, k)
    # residual norms come from ||H~ u||^2 - theta^2 (resolution ~1e-8 |theta|); the
    # eigenvalues then carry errors of order residual^2 / gap
    out = si.solve(T(U0), nev, degree=12, tol=tol, maxit=60)
    print(out["iterations"], out["residual"])
    assert out["converged"], out["history"][-5:]
    np.testing.assert_allclose(out["eigenvalues"], ref[:nev], rtol=0,
                               atol=1e-9 * max(1.0, abs(ref[:nev]).max()))
