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


CASES = [(2, 3, (3, 2, 2), W.BC_DIRICHLET0, 5), (3, 4, (2, 2, 3), W.BC_PERIODIC, 8),
         (4, 5, (2, 2, 2), W.BC_NONE, 3), (6, 7, (2, 2, 2), W.BC_PERIODIC, 16),
         (8, 9, (2, 1, 1), W.BC_DIRICHLET0, 9)]


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


def test_config2_cheb_step_sampled_rows_in_place():
    w = W.config2()
    op = mfmv.Operator.from_workload(w)
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    m_ref = orc.lumped_mass()
    D = mfmv.gll_mass(op, inv_sqrt=True)
    np.testing.assert_allclose(D.cpu().numpy(), 1.0 / np.sqrt(m_ref), rtol=1e-13, atol=0)
    Y = w.X()
    Xp = np.random.default_rng(7).uniform(-1, 1, Y.shape)
    a, b, c = 0.9, 0.25, -0.5
    Out = T(Xp)
    mfmv.cheb_step(op, D, T(Y), Out, Out, a, b, c)
    rows = np.random.default_rng(11).choice(orc.ndofs, 12, replace=False)
    Dr = 1.0 / np.sqrt(m_ref)
    ref = a * Dr[rows, None] * orc.apply_rows(Dr[:, None] * Y, rows) + b * Y[rows] + c * Xp[rows]
    got = Out[torch.from_numpy(rows).to(dev())].cpu().numpy()
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-12, rel


def test_chebyshev_filter_matches_oracle_recurrence():
    from paper_2208_07129_amd.chebyshev import chebyshev_filter, filter_coefficients
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
    steps = filter_coefficients(m, lmin, lmax, lu)
    a, b, _ = steps[0]
    prev, cur = U, orc.cheb_step(D_ref, U, None, a, b, 0.0)
    for a, b, c in steps[1:]:
        prev, cur = cur, orc.cheb_step(D_ref, cur, prev, a, b, c)
    assert colrel(Yd.cpu().numpy(), cur) <= 1e-11
