"""GPU tests of the learned-preconditioner kernels (include/mfmlp.h) against
the numpy FP64 oracle (oracle/mlp_oracle.py):

- the BF16 matrix-core GEMM in its three operand forms with every epilogue and
  the split batch dimension, against FP64 products of the same BF16 values
  (FP32 accumulation: 1e-5 relative);
- the cell gather (network inputs, targets, scales) and the partition-of-unity
  assembly (with and without the Jacobi term);
- loss and gradients of the whole network against the oracle's backward pass
  on the same BF16-rounded weights and inputs (BF16 activations: 2e-2);
- Adam against the oracle's FP32 update;
- training reduces the loss, and the trained step is judged against Jacobi.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp_oracle as mo
from oracle.fe_oracle import constrained_mask
from paper_2208_07129_amd import blockcg, mfmv, mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch.device("cuda:0")


def bf(a):
    """(device BF16 bits, FP64 values of the rounded numbers)"""
    bits = mlp._host_bf16(a)
    return torch.from_numpy(bits).to(dev()), mo.bf16_round(a)


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("M,N,K", [(8, 8, 8), (72, 136, 40), (256, 344, 352), (344, 200, 256)])
def test_gemm_forms(ta, tb, M, N, K):
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    Ad, Ar = bf(A)
    Bd, Br = bf(B)
    ref = (Ar.T if ta else Ar) @ (Br.T if tb else Br)
    out = torch.full((M, N), float("nan"), dtype=torch.float32, device=dev())
    mlp.CellMLP._gemm(M, N, K, ta, tb, Ad, A.shape[1], Bd, B.shape[1], out_f32=out, ld_f32=N)
    scale = np.abs(Ar).max() * np.abs(Br).max() * K
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=0, atol=1e-6 * scale)


def test_gemm_epilogues_and_split():
    rng = np.random.default_rng(5)
    M, N, K = 64, 128, 96
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    bias = rng.standard_normal(M).astype(np.float32)
    mask = rng.standard_normal((M, N)).astype(np.float32)
    Ad, Ar = bf(A)
    Bd, Br = bf(B)
    md, mr = bf(mask)
    ref = Ar @ Br
    tol = 1e-6 * np.abs(Ar).max() * np.abs(Br).max() * K
    f32 = torch.empty(M, N, dtype=torch.float32, device=dev())
    b16 = torch.empty(M, N, dtype=torch.int16, device=dev())
    bt = torch.from_numpy(bias).to(dev())
    mlp.CellMLP._gemm(M, N, K, False, False, Ad, K, Bd, N, bias=bt, relu=True, out_f32=f32,
                      ld_f32=N, out_bf16=b16, ld_bf16=N)
    want = np.maximum(ref + bias[:, None], 0)
    np.testing.assert_allclose(f32.cpu().numpy(), want, rtol=0, atol=tol)
    got16 = mo.bf16_round(f32.cpu().numpy())
    np.testing.assert_array_equal(mlp._host_bf16(f32.cpu().numpy()), b16.cpu().numpy())
    assert np.all(np.abs(got16 - want) <= np.abs(want) * 2 ** -8 + tol)
    mlp.CellMLP._gemm(M, N, K, False, False, Ad, K, Bd, N, mask=md, ldmask=N, out_f32=f32, ld_f32=N)
    np.testing.assert_allclose(f32.cpu().numpy(), ref * (mr > 0), rtol=0, atol=tol)
    f32.zero_()
    mlp.CellMLP._gemm(M, N, K, False, False, Ad, K, Bd, N, kchunk=32, out_f32=f32, ld_f32=N,
                      atomic=True)
    np.testing.assert_allclose(f32.cpu().numpy(), ref, rtol=0, atol=tol)
    with pytest.raises(mfmv.MfError):
        mlp.CellMLP._gemm(M, N, K, False, False, Ad, K, Bd, N, kchunk=32, bias=bt, out_f32=f32,
                          ld_f32=N, atomic=True)


def small_op(bc, p=3, n=(2, 3, 2), sigma=1.0):
    mesh = W.BoxMesh(n=n, lo=(0.0, 0.0, 0.0), hi=(2.0, 2.0, 2.0), bc=bc)
    V = W.gaussian_wells(11, L=2.0, k=3, width=0.5, depth=(-2.0, -0.5))
    op = mfmv.Operator(mesh, p, p + 1, 0.5, V(mfmv.quad_points(mesh, p + 1)), sigma)
    return mesh, op


@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC])
def test_cell_gather_and_scatter_match_oracle(bc):
    mesh, op = small_op(bc)
    p, k = op.p, 9
    cons = constrained_mask(mesh, p)
    rng = np.random.default_rng(3)
    R = rng.uniform(-1, 1, (op.ndofs, k))
    E = rng.uniform(-1, 1, (op.ndofs, k))
    R[cons] = 0.0
    net = mlp.CellMLP(op, hidden=16, seed=1)
    Rt, Et = torch.from_numpy(R).to(dev()), torch.from_numpy(E).to(dev())
    bs = net.gather(Rt, pou_sqrt=True)
    Xs, _, rhos = mo.cell_inputs(mesh, p, R, pou_sqrt=True)
    rows = op.ncells * k
    np.testing.assert_allclose(bs["rho"].cpu().numpy()[:rows], rhos, rtol=1e-6)
    xs = (bs["X0"].cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.all(np.abs(xs.astype(np.float64)[:net.F, :rows].T - Xs) <= np.abs(Xs) * 2 ** -8 + 1e-30)
    b = net.gather(Rt, Et)
    X, T, rho = mo.cell_inputs(mesh, p, R, E)
    F = net.F
    x0 = b["X0"].cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    X0 = x0.view(np.float32).astype(np.float64)
    rows = op.ncells * k
    np.testing.assert_allclose(b["rho"].cpu().numpy()[:rows], rho, rtol=1e-6)
    assert np.all(np.abs(X0[:F, :rows].T - X) <= np.abs(X) * 2 ** -8 + 1e-30)
    assert np.all(X0[F:] == 0.0) and np.all(X0[:, rows:] == 0.0)
    np.testing.assert_allclose(b["T"].cpu().numpy()[:F, :rows].T, T, rtol=1e-6,
                               atol=1e-6 * np.abs(T).max())
    # assembly of arbitrary outputs, with and without the Jacobi term
    Y = rng.standard_normal((net.Fp, b["ld"])).astype(np.float32)
    b["Y"].copy_(torch.from_numpy(Y))
    diag = rng.uniform(1.0, 2.0, op.ndofs)
    Rd, dd = torch.from_numpy(R).to(dev()), torch.from_numpy(diag).to(dev())
    Z = torch.empty_like(Rd)
    for with_j in (False, True):
        for sq in (0, 1):
            for ds in (None, dd):
                mfmv._check(mfmv.lib().mf_cell_scatter(
                    op._h, k, b["Y"].data_ptr(), b["ld"], b["rho"].data_ptr(),
                    dd.data_ptr() if with_j else None, Rd.data_ptr() if with_j else None, k,
                    Z.data_ptr(), k, sq, None if ds is None else ds.data_ptr(), 0, None))
                ref = mo.cell_assemble(mesh, p, Y[:F, :rows].T.astype(np.float64),
                                       b["rho"].cpu().numpy()[:rows].astype(np.float64), k,
                                       R if with_j else None, diag if with_j else None,
                                       pou_sqrt=bool(sq), dscale=None if ds is None else diag)
                np.testing.assert_allclose(Z.cpu().numpy(), ref, rtol=0,
                                           atol=1e-10 * np.abs(ref).max())
    # the assembly is taken node by node in a fixed order: bitwise reproducible
    Z2 = torch.empty_like(Z)
    mfmv._check(mfmv.lib().mf_cell_scatter(
        op._h, k, b["Y"].data_ptr(), b["ld"], b["rho"].data_ptr(), dd.data_ptr(), Rd.data_ptr(),
        k, Z2.data_ptr(), k, 1, dd.data_ptr(), 0, None))
    assert torch.equal(Z, Z2)
    # without rho: the gather does not normalise and the assembly takes rho = 1
    b1 = net.gather(Rt, pou_sqrt=True, normalise=False)
    x1 = (b1["X0"].cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    U = Xs * rhos[:, None]
    assert np.all(np.abs(x1.astype(np.float64)[:F, :rows].T - U) <= np.abs(U) * 2 ** -8 + 1e-30)
    mfmv._check(mfmv.lib().mf_cell_scatter(
        op._h, k, b["Y"].data_ptr(), b["ld"], None, dd.data_ptr(), Rd.data_ptr(), k,
        Z.data_ptr(), k, 1, dd.data_ptr(), 0, None))
    ref = mo.cell_assemble(mesh, p, Y[:F, :rows].T.astype(np.float64), np.ones(rows), k, R, diag,
                           pou_sqrt=True, dscale=diag)
    np.testing.assert_allclose(Z.cpu().numpy(), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # diagonally scaled network inputs and targets
    net.dscale = dd
    bd = net.gather(Rt, Et, pou_sqrt=True)
    Xd, Td, rhod = mo.cell_inputs(mesh, p, R, E, pou_sqrt=True, dscale=diag)
    np.testing.assert_allclose(bd["rho"].cpu().numpy()[:rows], rhod, rtol=1e-6)
    xd = (bd["X0"].cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.all(np.abs(xd.astype(np.float64)[:F, :rows].T - Xd) <= np.abs(Xd) * 2 ** -8 + 1e-30)
    np.testing.assert_allclose(bd["T"].cpu().numpy()[:F, :rows].T, Td, rtol=1e-6,
                               atol=1e-6 * np.abs(Td).max())


@pytest.mark.parametrize("n", [(1, 3, 2), (1, 1, 1)])
def test_node_assembly_with_one_cell_periodic_directions(n):
    """A one-cell periodic direction: the vertex nodes meet the same cell twice
    (local 0 and local p), each incidence with weight 1/2."""
    mesh, op = small_op(W.BC_PERIODIC, p=2, n=n)
    k, F = 5, 27
    net = mlp.CellMLP(op, hidden=8, seed=2)
    b = net._buffers(k)
    rows = op.ncells * k
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((net.Fp, b["ld"])).astype(np.float32)
    b["Y"].copy_(torch.from_numpy(Y))
    rho = rng.uniform(0.5, 2.0, b["ld"]).astype(np.float32)
    b["rho"].copy_(torch.from_numpy(rho))
    R = rng.standard_normal((op.ndofs, k))
    diag = rng.uniform(1.0, 2.0, op.ndofs)
    Rd, dd = torch.from_numpy(R).to(dev()), torch.from_numpy(diag).to(dev())
    Z = torch.empty_like(Rd)
    for sq in (0, 1):
        mfmv._check(mfmv.lib().mf_cell_scatter(
            op._h, k, b["Y"].data_ptr(), b["ld"], b["rho"].data_ptr(), dd.data_ptr(),
            Rd.data_ptr(), k, Z.data_ptr(), k, sq, dd.data_ptr(), 0, None))
        ref = mo.cell_assemble(mesh, op.p, Y[:F, :rows].T.astype(np.float64),
                               rho[:rows].astype(np.float64), k, R, diag, pou_sqrt=bool(sq),
                               dscale=diag)
        np.testing.assert_allclose(Z.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_skip_floor_rebuilds_the_spectrum():
    """mf_skip_floor on a random symmetric skip block with eigenvalues below -1:
    the rebuilt block has the eigenvalues max(w, floor) (floor from the block's
    own norm), is exactly symmetric, and its BF16 copy is its rounding."""
    mesh, op = small_op(W.BC_PERIODIC, p=3, n=(2, 2, 2))
    net = mlp.CellMLP(op, hidden=16, seed=3)
    H, F = net.H, net.F
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((F, F)))
    w = np.linspace(-3.0, 2.0, F)
    S = ((Q * w) @ Q.T).astype(np.float32)
    with torch.no_grad():
        net.params[4][:F, H:H + F] = torch.from_numpy(S).to(dev())
    assert net.floor_skip(margin=0.05) == 0
    Sd = net.params[4][:F, H:H + F].cpu().numpy()
    assert np.array_equal(Sd, Sd.T)
    S64 = (S.astype(np.float64) + S.T.astype(np.float64)) / 2
    ws = np.linalg.eigvalsh(S64)
    floor = -1.0 + 0.05 + 2.0 ** -8 * (np.sqrt((ws ** 2).sum()) + np.sqrt(F))
    np.testing.assert_allclose(np.linalg.eigvalsh(Sd.astype(np.float64)), np.maximum(ws, floor),
                               rtol=0, atol=2e-6 * np.abs(ws).max())
    bf = net.wbf[4][:F, H:H + F].cpu().numpy()
    assert np.array_equal(bf, mlp._host_bf16(Sd))
    # the rest of the last layer is untouched
    assert np.all(net.params[4][:F, :H].cpu().numpy() == 0.0)


def test_floored_skip_gives_a_positive_definite_preconditioner():
    """The linear preconditioner with S = -4 I is indefinite; after the floor it
    is D^-1/2 (1 + floor) D^-1/2 (partition of unity), positive definite.  Built
    densely by applying it to the unit vectors (up to the BF16 rounding of its
    input, so the symmetric part is judged)."""
    mesh, op = small_op(W.BC_PERIODIC, p=2, n=(2, 2, 2))
    diag = mfmv.diagonal(op)
    net = mlp.CellMLP(op, hidden=8, seed=1, dscale=diag)
    H, F, n = net.H, net.F, op.ndofs
    with torch.no_grad():
        net.params[4].zero_()
        net.params[4][:F, H:H + F] = -4.0 * torch.eye(F, device=dev())
        net.wbf[4].copy_(torch.from_numpy(mlp._host_bf16(net.params[4].cpu().numpy())))
    I = torch.eye(n, dtype=torch.float64, device=dev())
    Z = torch.empty_like(I)
    dh = np.sqrt(diag.cpu().numpy())

    def scaled_sym():
        net.precondition(I, Z, diag, linear=True)
        M = Z.cpu().numpy()
        M = dh[:, None] * M * dh[None, :]
        return np.linalg.eigvalsh((M + M.T) / 2)

    assert scaled_sym().min() < -1.0
    assert net.floor_skip(margin=0.02) == 0
    floor = -1.0 + 0.02 + 2.0 ** -8 * (4.0 * np.sqrt(F) + np.sqrt(F))
    ev = scaled_sym()
    assert ev.min() > 0.0
    # BF16 rounding of the floored block (2^-9 of 0.88) and of the input
    np.testing.assert_allclose(ev, 1.0 + floor, rtol=0.03)


@pytest.mark.parametrize("bc,k", [(W.BC_PERIODIC, 16), (W.BC_DIRICHLET0, 16), (W.BC_PERIODIC, 9)])
def test_linear_preconditioner_matches_oracle(bc, k):
    """The deployed linear map z = D^-1 r + sum_e Q_e^T W^1/2 D^-1/2 S D^-1/2 W^1/2 Q_e r
    against the oracle's gather and assembly with the same BF16 rounding of the
    input and of S (k = 16: cell-blocked activations; k = 9: feature-major).  The
    blocked path equals the feature-major one bitwise."""
    mesh, op = small_op(bc, p=3, n=(2, 3, 2))
    diag = mfmv.diagonal(op)
    net = mlp.CellMLP(op, hidden=16, seed=5, dscale=diag)
    H, F = net.H, net.F
    rng = np.random.default_rng(21)
    Q, _ = np.linalg.qr(rng.standard_normal((F, F)))
    S = ((Q * rng.uniform(-0.9, 2.0, F)) @ Q.T).astype(np.float32)
    S = (S + S.T) / 2
    with torch.no_grad():
        net.params[4][:F, H:H + F] = torch.from_numpy(S).to(dev())
        net.wbf[4].copy_(torch.from_numpy(mlp._host_bf16(net.params[4].cpu().numpy())))
    cons = constrained_mask(mesh, op.p)
    R = rng.uniform(-1, 1, (op.ndofs, k))
    R[cons] = 0.0
    Rt = torch.from_numpy(R).to(dev())
    Z = torch.empty_like(Rt)
    net.precondition(Rt, Z, diag, linear=True)
    dg = diag.cpu().numpy()
    X, _, rho = mo.cell_inputs(mesh, op.p, R, pou_sqrt=True, dscale=dg)
    U = mo.bf16_round(X * rho[:, None])
    Sb = mo.bf16_round(S)
    ref = mo.cell_assemble(mesh, op.p, U @ Sb.T, np.ones(len(rho)), k, R, dg, pou_sqrt=True,
                           dscale=dg)
    bound = mo.cell_assemble(mesh, op.p, np.abs(X * rho[:, None]) @ np.abs(Sb).T,
                             np.ones(len(rho)), k, pou_sqrt=True, dscale=dg)
    assert np.all(np.abs(Z.cpu().numpy() - ref) <= 2 ** -8 * np.abs(bound) + 1e-12 * np.abs(ref).max())
    if k % 8 == 0:  # the same map through the feature-major layout
        b = net.gather(Rt, pou_sqrt=True, normalise=False, blocked=False)
        Fp, n = net.Fp, b["ld"]
        net._gemm(Fp, n, Fp, False, False, net.wbf[4][:, H:], H + Fp, b["X0"], n,
                  out_f32=b["Y"], ld_f32=n)
        Z2 = torch.empty_like(Rt)
        mfmv._check(mfmv.lib().mf_cell_scatter(
            op._h, k, b["Y"].data_ptr(), n, None, diag.data_ptr(), Rt.data_ptr(), k,
            Z2.data_ptr(), k, 1, diag.data_ptr(), 0, None))
        assert torch.equal(Z, Z2)


def test_forward_backward_match_oracle():
    mesh, op = small_op(W.BC_PERIODIC, p=2, n=(2, 2, 2))
    k = 8
    net = mlp.CellMLP(op, hidden=32, seed=4, out_scale=1.0)
    rng = np.random.default_rng(9)
    R = torch.from_numpy(rng.uniform(-1, 1, (op.ndofs, k))).to(dev())
    E = torch.from_numpy(rng.uniform(-1, 1, (op.ndofs, k))).to(dev())
    b = net.gather(R, E)
    net.forward(b)
    net._loss.zero_()
    net.loss_grad(b)
    net.backward(b, kchunk=32)
    F, Fp = net.F, net.Fp
    rows = op.ncells * k
    x0 = (b["X0"].cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    X = x0.astype(np.float64)[:F, :rows].T
    T = b["T"].cpu().numpy().astype(np.float64)[:F, :rows].T
    H = net.H
    W1, b1, W2, b2, W3S, b3 = [p.cpu().numpy().astype(np.float64) for p in net.params]
    params = [mo.bf16_round(W1[:, :F]), b1, mo.bf16_round(W2), b2, mo.bf16_round(W3S[:F, :H]),
              b3[:F], mo.bf16_round(W3S[:F, H:H + F])]
    loss, grads = mo.loss_and_grads(params, X, T)
    assert abs(net._loss.item() - loss) <= 2e-2 * loss
    gW1, gb1, gW2, gb2, gW3S, gb3 = [g.cpu().numpy().astype(np.float64) for g in net.grads]
    got = [gW1[:, :F], gb1, gW2, gb2, gW3S[:F, :H], gb3[:F], gW3S[:F, H:H + F]]
    for name, g, r in zip(["W1", "b1", "W2", "b2", "W3", "b3", "S"], got, grads):
        rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
        assert rel <= 2e-2, (name, rel)
    assert np.all(gW1[:, F:] == 0) and np.all(gW3S[F:] == 0) and np.all(gb3[F:] == 0)
    assert np.all(gW3S[:, H + F:] == 0)


def test_symmetric_projection():
    mesh, op = small_op(W.BC_PERIODIC, p=2, n=(1, 1, 2))
    net = mlp.CellMLP(op, hidden=16, seed=2)
    rng = np.random.default_rng(8)
    H, F = net.H, net.F
    Wh = rng.standard_normal(net.params[4].shape).astype(np.float32)
    net.params[4].copy_(torch.from_numpy(Wh))
    net.project()
    got = net.params[4].cpu().numpy()
    Sref = 0.5 * (Wh[:F, H:H + F] + Wh[:F, H:H + F].T)
    np.testing.assert_allclose(got[:F, H:H + F], Sref, rtol=1e-6)
    np.testing.assert_array_equal(got[:, :H], Wh[:, :H])
    np.testing.assert_array_equal(net.wbf[4].cpu().numpy()[:F, H:H + F], mlp._host_bf16(Sref))


def test_adam_matches_oracle():
    mesh, op = small_op(W.BC_PERIODIC, p=2, n=(1, 1, 2))
    net = mlp.CellMLP(op, hidden=16, seed=2, out_scale=1.0)
    rng = np.random.default_rng(1)
    w0 = [p.cpu().numpy().copy() for p in net.params]
    g = [rng.standard_normal(p.shape).astype(np.float32) for p in net.params]
    for gd, gh in zip(net.grads, g):
        gd.copy_(torch.from_numpy(gh))
    net.adam(1e-2)
    H, F = net.H, net.F
    for i, (w, gh) in enumerate(zip(w0, g)):
        ref, _, _ = mo.adam_step(w, gh, np.zeros_like(w), np.zeros_like(w), 1e-2, 0.9, 0.999, 1e-8, 1)
        if i == 4:  # the skip block is projected onto symmetric matrices after the step
            S = ref[:F, H:H + F]
            ref[:F, H:H + F] = 0.5 * (S + S.T)
        np.testing.assert_allclose(net.params[i].cpu().numpy(), ref, rtol=1e-6, atol=1e-7)
    for i in (0, 2, 4):
        np.testing.assert_array_equal(net.wbf[i].cpu().numpy(),
                                      mlp._host_bf16(net.params[i].cpu().numpy()))


def test_adam_kernel_three_steps_match_the_hand_derivation():
    """mf_adam over three steps (moment decay and bias correction at t = 2, 3) against
    the hand-derived values of tests/golden/adam_three_steps.json, and against the
    oracle's Adam on a random vector over five steps."""
    import ctypes
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "adam_three_steps.json")) as f:
        g = json.load(f)
    L = mfmv.lib()
    s = torch.cuda.current_stream().cuda_stream
    f32 = dict(dtype=torch.float32, device=dev())
    w = torch.tensor(g["w0"], **f32)
    m1, m2 = torch.zeros(2, **f32), torch.zeros(2, **f32)
    wbf = torch.zeros(2, dtype=torch.int16, device=dev())
    for t, grad in enumerate(g["grads"], start=1):
        gd = torch.tensor(grad, **f32)
        assert L.mf_adam(2, w.data_ptr(), gd.data_ptr(), m1.data_ptr(), m2.data_ptr(),
                         wbf.data_ptr(), ctypes.c_float(g["lr"]), ctypes.c_float(g["b1"]),
                         ctypes.c_float(g["b2"]), ctypes.c_float(g["eps"]), t, s) == 0
        torch.cuda.synchronize()
        np.testing.assert_allclose(w.cpu().numpy(), [g["w_after"][0][t - 1], g["w_after"][1][t - 1]],
                                   rtol=1e-6, atol=0)
        bf = (wbf.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
        np.testing.assert_array_equal(bf, mo.bf16_round(w.cpu().numpy()).astype(np.float32))
    rng = np.random.default_rng(3)
    n = 1000
    wh = rng.standard_normal(n).astype(np.float32)
    w = torch.from_numpy(wh.copy()).to(dev())
    m1, m2 = torch.zeros(n, **f32), torch.zeros(n, **f32)
    r1, r2 = np.zeros(n, np.float32), np.zeros(n, np.float32)
    # the C ABI takes the hyper-parameters as FP32: the oracle gets the same values
    lr, b1, b2, eps = (float(np.float32(v)) for v in (1e-2, 0.9, 0.999, 1e-8))
    for t in range(1, 6):
        gh = rng.standard_normal(n).astype(np.float32) * (0.0 if t == 3 else 1.0)
        gd = torch.from_numpy(gh).to(dev())
        assert L.mf_adam(n, w.data_ptr(), gd.data_ptr(), m1.data_ptr(), m2.data_ptr(), None,
                         ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2),
                         ctypes.c_float(eps), t, s) == 0
        wh, r1, r2 = mo.adam_step(wh, gh, r1, r2, lr, b1, b2, eps, t)
    torch.cuda.synchronize()
    np.testing.assert_allclose(w.cpu().numpy(), wh, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(m2.cpu().numpy(), r2, rtol=1e-5, atol=1e-12)


def test_training_reduces_loss_and_fits_the_cell_blocks():
    mesh, op = small_op(W.BC_PERIODIC, p=3, n=(4, 4, 4))
    diag = mfmv.diagonal(op)
    net = mlp.CellMLP(op, hidden=128, seed=0)
    losses = mlp.train(net, diag, steps=300, k=16)
    first, last = np.mean(losses[:5]), np.mean(losses[-10:])
    assert np.isfinite(last) and last < 0.3 * first, (first, last)
    fit = mlp.local_fit(net, diag, k=16)
    assert fit < 0.3, fit           # held out: close to the cell-block inverse
    for linear in (True, False):
        j = mlp.judge(net, diag, k=8, linear=linear)
        assert np.isfinite(j["ratio"]) and j["jacobi"] > 0


def test_learned_preconditioner_gain_over_jacobi():
    """The trained network against Jacobi in block PCG on the same problem (FP64
    apply): both reach 1e-10; the judge prefers the learned step on held-out pairs
    and the learned preconditioner needs fewer iterations (the gain the network
    brings).  The whole nonlinear network also converges (flexible iteration)."""
    mesh, op = small_op(W.BC_PERIODIC, p=3, n=(4, 4, 4))
    diag = mfmv.diagonal(op)
    net = mlp.CellMLP(op, hidden=128, seed=0, dscale=diag)
    mlp.train(net, diag, steps=1000, k=16)
    B = torch.from_numpy(np.random.default_rng(4).uniform(-1, 1, (op.ndofs, 8))).to(dev())
    jac = blockcg.jacobi_preconditioner(diag)
    _, sj = blockcg.solve(op, B, jac, tol=1e-10, maxit=3000)
    _, sl = blockcg.solve(op, B, net.preconditioner(diag), tol=1e-10, maxit=3000, fallback=jac)
    _, sf = blockcg.solve(op, B, net.preconditioner(diag, linear=False), tol=1e-10, maxit=3000,
                          fallback=jac)
    jd = mlp.judge(net, diag, k=8)
    print("jacobi", sj.iterations, "learned", sl.iterations, "full", sf.iterations, "judge", jd)
    assert sj.converged and sl.converged and sf.converged
    assert jd["ratio"] < 1.0
    assert sl.iterations < sj.iterations


@pytest.mark.parametrize("corruption", ["nan", "negated"])
def test_corrupted_network_falls_back_to_jacobi(corruption):
    """A broken network (NaN weights, or a skip block that makes the learned step an
    ascent direction) is caught by the descent check: the solve switches to Jacobi
    and still reaches 1e-10 in every column."""
    mesh, op = small_op(W.BC_PERIODIC, p=3, n=(3, 3, 3))
    diag = mfmv.diagonal(op)
    net = mlp.CellMLP(op, hidden=64, seed=1, dscale=diag)
    H, F = net.H, net.F
    with torch.no_grad():
        if corruption == "nan":
            net.params[4].fill_(float("nan"))
        else:  # S = -4 I: z = D^-1 r - 4 (D^-1/2 sqrt(w) ...) pushes z^T r below zero
            net.params[4].zero_()
            net.params[4][:F, H:H + F] = -4.0 * torch.eye(F, device=dev())
        net.wbf[4].copy_(torch.from_numpy(mlp._host_bf16(net.params[4].cpu().numpy())))
    B = torch.from_numpy(np.random.default_rng(6).uniform(-1, 1, (op.ndofs, 4))).to(dev())
    jac = blockcg.jacobi_preconditioner(diag)
    _, st = blockcg.solve(op, B, net.preconditioner(diag), tol=1e-10, maxit=3000, fallback=jac)
    assert st.converged and st.rel_residual <= 1e-10, st
    assert st.precond_switches >= 1


def test_checkpoint_resume_continues_training(tmp_path):
    """save/load round-trips the whole training state bitwise (weights, BF16 copies,
    Adam moments, step); a run resumed from a step-5 checkpoint draws the same pairs
    and reproduces the uninterrupted run's losses (to the rounding of the FP32
    atomic weight-gradient sums); a checkpoint of another shape is refused."""
    mesh, op = small_op(W.BC_PERIODIC, p=2, n=(2, 2, 2))
    diag = mfmv.diagonal(op)
    ck = str(tmp_path / "net.safetensors")
    full = mlp.CellMLP(op, hidden=16, seed=3, dscale=diag)
    losses_full = mlp.train(full, diag, steps=10, k=8, refresh=2)
    part = mlp.CellMLP(op, hidden=16, seed=3, dscale=diag)
    mlp.train(part, diag, steps=5, k=8, refresh=2, checkpoint=ck, every=5)
    assert part.step == 5
    resumed = mlp.CellMLP(op, hidden=16, seed=99, dscale=diag)   # other initial weights
    resumed.load(ck)
    a, b = part.state(), resumed.state()
    assert a.keys() == b.keys() and all(torch.equal(a[key], b[key]) for key in a)
    assert resumed.step == 5
    losses_tail = mlp.train(resumed, diag, steps=10, k=8, refresh=2)
    assert resumed.step == 10 and len(losses_tail) == 5
    np.testing.assert_allclose(losses_tail, losses_full[5:], rtol=1e-3)
    other = mlp.CellMLP(op, hidden=8, seed=0, dscale=diag)
    with pytest.raises(ValueError):
        other.load(ck)
