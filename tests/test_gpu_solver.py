"""GPU tests of the block-CG building blocks (include/mfsolve.h) and of the
block-CG solve.

- mf_diagonal against the oracle's assembled element-matrix diagonal (1e-12,
  every boundary condition, box and sheared cells).
- Gram, paired Gram, block update (also with the column norms of its
  result), column dots, axpby, Jacobi and the small SPD solve against numpy
  in FP64 on seeded inputs with ragged sizes.
- Block PCG (Jacobi) on small meshes: the true FP64 residual reaches 1e-10 in
  every column and the solution agrees with a dense direct solve of the
  oracle's assembled matrix to within cond(A) * 1e-10; the mixed-precision
  apply inside FP64 iterative refinement reaches the same residual.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fe_oracle as fo
from paper_2208_07129_amd import blockcg, mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHEAR = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])


def dev():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def vfun(x):
    return np.sin(x[..., 0]) + x[..., 1] * x[..., 2] - 0.3


@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC])
@pytest.mark.parametrize("p,q,lin", [(1, 2, None), (2, 3, SHEAR), (3, 5, None), (5, 6, None),
                                     (6, 7, SHEAR)])
def test_diagonal_matches_oracle(bc, p, q, lin):
    mesh = W.BoxMesh(n=(2, 3, 2), lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc, lin=lin)
    orc = fo.Oracle(mesh, p, q, 0.5, vfun, 0.2)
    op = mfmv.Operator(mesh, p, q, 0.5, vfun(mfmv.quad_points(mesh, q)), 0.2)
    d = mfmv.diagonal(op).cpu().numpy()
    ref = orc.diagonal()
    free = ~orc.constrained
    rel = np.abs(d[free] - ref[free]).max() / np.abs(ref[free]).max()
    assert rel <= 1e-12
    np.testing.assert_array_equal(d[orc.constrained], 1.0)


@pytest.mark.parametrize("n,k,kp", [(0, 3, 3), (1, 1, 1), (997, 7, 5), (5000, 64, 64),
                                    (3001, 128, 128), (2049, 300, 17), (600011, 128, 130)])
def test_dense_blocks_match_numpy(n, k, kp):
    rng = np.random.default_rng(n + k)
    A = rng.standard_normal((n, k))
    B = rng.standard_normal((n, k))
    P = rng.standard_normal((n, kp))
    M = rng.standard_normal((kp, k))
    Y = rng.standard_normal((n, k))
    C0 = rng.standard_normal((k, k))
    tol = 1e-13 * max(1, n) ** 0.5
    C = mfmv.block_gram(T(A), T(B), T(C0), alpha=0.5, beta=2.0).cpu().numpy()
    np.testing.assert_allclose(C, 0.5 * A.T @ B + 2.0 * C0, rtol=0, atol=tol * 10)
    Yd = mfmv.block_update(T(P), T(M), T(Y), alpha=-1.5, beta=0.25).cpu().numpy()
    np.testing.assert_allclose(Yd, 0.25 * Y - 1.5 * P @ M, rtol=0, atol=tol * 10)
    d = mfmv.col_dots(T(A), T(B)).cpu().numpy()
    np.testing.assert_allclose(d, (A * B).sum(axis=0), rtol=0, atol=tol * 10)
    Yd = mfmv.axpby(-2.0, T(A), 0.5, T(Y)).cpu().numpy()
    np.testing.assert_array_equal(Yd, -2.0 * A + 0.5 * Y)
    Yn = torch.full((n, k), float("nan"), dtype=torch.float64, device=dev())
    np.testing.assert_array_equal(mfmv.axpby(3.0, T(A), 0.0, Yn).cpu().numpy(), 3.0 * A)
    diag = rng.uniform(0.5, 2.0, n)
    np.testing.assert_array_equal(mfmv.jacobi(T(diag), T(A)).cpu().numpy(), A / diag[:, None])


@pytest.mark.parametrize("n,k,kp", [(0, 3, 3), (1, 1, 1), (997, 7, 5), (5000, 64, 64),
                                    (3001, 128, 128), (2049, 300, 17), (600011, 128, 120),
                                    (70001, 100, 33)])
def test_paired_gram_and_update_with_norms_match_numpy(n, k, kp):
    """block_gram2 (A^T B1 and A^T B2 in one pass over A) and block_update_norms
    (Y := beta Y + alpha P M with the squared column norms of the new Y) against
    numpy in FP64, over ragged row counts (partial chunks, partial 16-row strips),
    k not a multiple of 16 and k above one 128-column block."""
    rng = np.random.default_rng(7 * n + k)
    A = rng.standard_normal((n, k))
    B1 = rng.standard_normal((n, k))
    B2 = rng.uniform(-3, 1, (n, k))
    C10 = rng.standard_normal((k, k))
    C20 = rng.standard_normal((k, k))
    tol = 1e-12 * max(1, n) ** 0.5
    C1 = torch.full((k, k), float("nan"), dtype=torch.float64, device=dev())
    C1, C2 = mfmv.block_gram2(T(A), T(B1), T(B2), C1, T(C20), alpha=-0.75, beta=0.0)
    np.testing.assert_allclose(C1.cpu().numpy(), -0.75 * A.T @ B1, rtol=0, atol=tol * 3)
    np.testing.assert_allclose(C2.cpu().numpy(), -0.75 * A.T @ B2, rtol=0, atol=tol * 3)
    C1, C2 = mfmv.block_gram2(T(A), T(B1), T(B2), T(C10), T(C20), alpha=0.5, beta=2.0)
    np.testing.assert_allclose(C1.cpu().numpy(), 0.5 * A.T @ B1 + 2.0 * C10, rtol=0, atol=tol * 3)
    np.testing.assert_allclose(C2.cpu().numpy(), 0.5 * A.T @ B2 + 2.0 * C20, rtol=0, atol=tol * 3)
    P = rng.standard_normal((n, kp))
    M = rng.standard_normal((kp, k))
    Y = rng.standard_normal((n, k))
    if k > 128 or kp > 128:
        with pytest.raises(mfmv.MfError) as e:
            mfmv.block_update_norms(T(P), T(M), T(Y))
        assert e.value.status == mfmv.MF_ERR_UNSUPPORTED
        return
    for alpha, beta in ((-1.0, 1.0), (2.5, 0.0)):
        Yn = T(Y) if beta != 0.0 else torch.full((n, k), float("nan"), dtype=torch.float64,
                                                 device=dev())
        nrm = torch.full((k,), float("nan"), dtype=torch.float64, device=dev())
        Yd, nrm = mfmv.block_update_norms(T(P), T(M), Yn, nrm, alpha=alpha, beta=beta)
        Yd, nrm = Yd.cpu().numpy(), nrm.cpu().numpy()
        ref = beta * Y + alpha * P @ M
        np.testing.assert_allclose(Yd, ref, rtol=0, atol=1e-12 * kp * 10)
        # the norms are those of the values stored, to the rounding of a sum of n squares
        np.testing.assert_allclose(nrm, (Yd * Yd).sum(axis=0), rtol=1e-13 * max(1, n) ** 0.5,
                                   atol=0)
        np.testing.assert_allclose(nrm, (ref * ref).sum(axis=0), rtol=1e-12, atol=0)
        # the same update as block_update, bit for bit
        Yb = mfmv.block_update(T(P), T(M), T(Y), alpha=alpha, beta=beta).cpu().numpy()
        np.testing.assert_array_equal(Yd, Yb)


def test_paired_gram_and_update_norms_strided_and_repeatable():
    """Column blocks of wider arrays (ld > k), results repeat bit for bit (fixed
    summation order), and bad arguments are refused."""
    rng = np.random.default_rng(21)
    n, k = 123457, 80
    Wh = rng.standard_normal((n, 3 * k + 5))
    Wd = T(Wh)
    A, B1, B2 = Wd[:, 0:k], Wd[:, k + 2:2 * k + 2], Wd[:, 2 * k + 5:3 * k + 5]
    C1, C2 = mfmv.block_gram2(A, B1, B2)
    D1, D2 = mfmv.block_gram2(A, B1, B2)
    assert torch.equal(C1, D1) and torch.equal(C2, D2)
    np.testing.assert_allclose(C1.cpu().numpy(), Wh[:, 0:k].T @ Wh[:, k + 2:2 * k + 2], rtol=0,
                               atol=1e-11 * n ** 0.5)
    np.testing.assert_allclose(C2.cpu().numpy(), Wh[:, 0:k].T @ Wh[:, 2 * k + 5:3 * k + 5],
                               rtol=0, atol=1e-11 * n ** 0.5)
    M = T(rng.standard_normal((k, k)))
    Yw = torch.zeros((n, k + 7), dtype=torch.float64, device=dev())
    Yv = Yw[:, 3:k + 3]
    _, n1 = mfmv.block_update_norms(A, M, Yv, alpha=1.0, beta=0.0)
    _, n2 = mfmv.block_update_norms(A, M, Yv, alpha=1.0, beta=0.0)
    assert torch.equal(n1, n2)
    ref = Wh[:, 0:k] @ M.cpu().numpy()
    np.testing.assert_allclose(Yv.cpu().numpy(), ref, rtol=0, atol=1e-12 * k * 10)
    np.testing.assert_allclose(n1.cpu().numpy(), (ref * ref).sum(axis=0), rtol=1e-12)
    assert float(Yw[:, :3].abs().max()) == 0.0 and float(Yw[:, k + 3:].abs().max()) == 0.0
    with pytest.raises(mfmv.MfError) as e:      # C1 overlapping B1
        mfmv.block_gram2(A, B1, B2, C1=Wd[:k, k + 2:2 * k + 2])
    assert e.value.status == mfmv.MF_ERR_ARG
    with pytest.raises(mfmv.MfError) as e:      # work too short
        mfmv.block_gram2(A, B1, B2, work=torch.empty(10, dtype=torch.float64, device=dev()))
    assert e.value.status == mfmv.MF_ERR_ARG
    with pytest.raises(mfmv.MfError) as e:      # Y overlapping P
        mfmv.block_update_norms(A, M, Wd[:, 1:k + 1])
    assert e.value.status == mfmv.MF_ERR_ARG


def test_dense_blocks_strided_and_symmetric():
    """Leading dimensions larger than k (column blocks of wider arrays), a Gram block of a
    multivector with itself (symmetric to rounding), and beta = 0 with a NaN-filled C."""
    rng = np.random.default_rng(9)
    n, k = 40000, 96
    W = rng.standard_normal((n, 2 * k + 3))
    A, B = W[:, 1:k + 1], W[:, k + 3:2 * k + 3]
    Wd = T(W)
    Ad, Bd = Wd[:, 1:k + 1], Wd[:, k + 3:2 * k + 3]
    C = torch.full((k, k), float("nan"), dtype=torch.float64, device=dev())
    C = mfmv.block_gram(Ad, Bd, C, alpha=1.0, beta=0.0).cpu().numpy()
    np.testing.assert_allclose(C, A.T @ B, rtol=0, atol=1e-12 * n ** 0.5 * 10)
    G = mfmv.block_gram(Ad, Ad).cpu().numpy()
    np.testing.assert_allclose(G, A.T @ A, rtol=0, atol=1e-12 * n ** 0.5 * 10)
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
    M = rng.standard_normal((k, k))
    Yw = torch.zeros((n, 2 * k + 3), dtype=torch.float64, device=dev())
    Yv = Yw[:, 2:k + 2]
    mfmv.block_update(Ad, T(M), Yv, alpha=2.0, beta=0.0)
    np.testing.assert_allclose(Yv.cpu().numpy(), 2.0 * A @ M, rtol=0, atol=1e-12 * k * 10)
    assert float(Yw[:, :2].abs().max()) == 0.0 and float(Yw[:, k + 2:].abs().max()) == 0.0


def test_dense_blocks_reject_bad_arguments():
    X = torch.zeros(10, 4, dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        mfmv.block_update(X, torch.zeros(4, 4, dtype=torch.float64, device=dev()), X)
    assert e.value.status == mfmv.MF_ERR_ARG  # Y overlaps P
    with pytest.raises(mfmv.MfError) as e:
        mfmv.axpby(1.0, X[1:], 1.0, X[:-1])
    assert e.value.status == mfmv.MF_ERR_ARG
    G = torch.eye(200, dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        mfmv.spd_solve(G, G)
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED


@pytest.mark.parametrize("k,m", [(1, 1), (5, 3), (13, 7), (64, 64), (128, 128), (97, 200)])
def test_spd_solve(k, m):
    rng = np.random.default_rng(k * 1000 + m)
    Z = rng.standard_normal((k, k))
    G = Z @ Z.T + k * np.eye(k)
    S = rng.standard_normal((k, m))
    X, st = mfmv.spd_solve(T(G), T(S))
    assert int(st.item()) == 0
    ref = np.linalg.solve(G, S)
    np.testing.assert_allclose(X.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # an indefinite block reports the first bad pivot (in the first and in a later
    # 8-column block of the blocked factorisation)
    for piv in sorted({2 % k, 11 % k}):
        Gi = G.copy()
        Gi[piv, piv] = -1.0 - np.abs(G).sum()
        _, st = mfmv.spd_solve(T(Gi), T(S))
        assert int(st.item()) == piv + 1


def small_problem(bc, p=3, n=(3, 3, 3), k=6, seed=7):
    mesh = W.BoxMesh(n=n, lo=(0.0, 0.0, 0.0), hi=(2.0, 2.0, 2.0), bc=bc)
    V = W.gaussian_wells(seed, L=2.0, k=3, width=0.5, depth=(-2.0, -0.5))
    sigma = 1.0
    orc = fo.Oracle(mesh, p, p + 1, 0.5, V, sigma)
    op = mfmv.Operator(mesh, p, p + 1, 0.5, V(mfmv.quad_points(mesh, p + 1)), sigma)
    Bh = np.random.default_rng(seed).uniform(-1, 1, (orc.ndofs, k))
    Bh[orc.constrained] = 0.0
    return op, orc, Bh


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET0])
@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_block_pcg_jacobi_solves(bc, inner):
    op, orc, Bh = small_problem(bc)
    diag = mfmv.diagonal(op)
    X, st = blockcg.solve(op, T(Bh), blockcg.jacobi_preconditioner(diag), tol=1e-10,
                          maxit=3000, inner_precision=inner)
    assert st.converged and st.rel_residual <= 1e-10, st
    A = orc.assemble_dense()
    free = ~orc.constrained
    Af = A[np.ix_(free, free)]
    Xref = np.linalg.solve(Af, Bh[free])
    ev = np.linalg.eigvalsh(Af)
    assert ev[0] > 0, "test operator must be SPD"
    cond = ev[-1] / ev[0]
    Xd = X.cpu().numpy()
    err = np.linalg.norm(Xd[free] - Xref, axis=0) / np.linalg.norm(Xref, axis=0)
    assert err.max() <= cond * 1e-10
    assert np.all(Xd[orc.constrained] == 0.0) or bc == W.BC_PERIODIC
    # FP64 residual recomputed independently on the host
    Rh = Bh - orc.apply(Xd)
    assert (np.linalg.norm(Rh, axis=0) / np.linalg.norm(Bh, axis=0)).max() <= 1.5e-10


def test_block_pcg_fewer_iterations_than_single_column_cg():
    """The block method shares Krylov information across right-hand sides: it needs
    no more iterations than the same method on one column at a time."""
    op, orc, Bh = small_problem(W.BC_PERIODIC, k=8)
    diag = mfmv.diagonal(op)
    M = blockcg.jacobi_preconditioner(diag)
    _, st_block = blockcg.solve(op, T(Bh), M, tol=1e-10, maxit=3000)
    its = []
    for j in range(2):
        _, st1 = blockcg.solve(op, T(Bh[:, j:j + 1]), M, tol=1e-10, maxit=3000)
        assert st1.converged
        its.append(st1.iterations)
    assert st_block.converged
    assert st_block.iterations <= min(its)


def test_lanczos_extremes_match_dense_eigenvalues():
    op, orc, _ = small_problem(W.BC_DIRICHLET0)
    lam = blockcg.lanczos_extremes(op, steps=200)
    free = ~orc.constrained
    A = orc.assemble_dense()[np.ix_(free, free)]
    ev = np.linalg.eigvalsh(A)
    assert abs(lam["lambda_max"] - ev[-1]) <= 1e-6 * ev[-1]
    assert ev[0] - 1e-9 * ev[-1] <= lam["lambda_min"] <= ev[0] * 1.05
