"""GPU tests of the deterministic (colour-ordered) assembly, mf_set_deterministic:
the apply still matches the oracle, repeated applies are bitwise equal (the
atomic assembly's shared rows vary in their last bits from run to run), and the
meshes that cannot be coloured are refused."""
import numpy as np
import pytest

import workloads as W
from oracle import fe_oracle as fo
from paper_2208_07129_amd import mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def dev():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch.device("cuda:0")


def colrel(Y, Yref):
    num = np.linalg.norm(Y - Yref, axis=0)
    den = np.linalg.norm(Yref, axis=0)
    return float((num / np.maximum(den, 1e-300)).max())


def vfun(x):
    return np.sin(x[..., 0]) + x[..., 1] * x[..., 2] - 0.3


@pytest.mark.parametrize("p,n,bc", [
    (3, (3, 4, 2), W.BC_PERIODIC),     # an odd periodic direction: three colours there
    (4, (2, 3, 3), W.BC_DIRICHLET0),
    (2, (1, 2, 3), W.BC_NONE),         # one cell in a non-periodic direction is fine
])
def test_deterministic_apply_matches_oracle_and_repeats_bitwise(p, n, bc):
    q = p + 1
    mesh = W.BoxMesh(n=n, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc)
    op = mfmv.Operator(mesh, p, q, 0.5, vfun(mfmv.quad_points(mesh, q)), 0.2)
    orc = fo.Oracle(mesh, p, q, 0.5, vfun, 0.2)
    op.set_deterministic(True)
    for nv in (7, 8):
        X = np.random.default_rng(p + nv).uniform(-1, 1, (orc.ndofs, nv))
        Yref = orc.apply(X)
        Xd = torch.from_numpy(X).to(dev())
        ran = 0
        for cfg in range(mfmv.BOX_CFGS):
            try:
                op.set_launch(False, cfg)
            except mfmv.MfError as e:
                assert e.status == mfmv.MF_ERR_UNSUPPORTED
                continue
            Y1 = op.apply(Xd, torch.full_like(Xd, float("nan")))
            Y2 = op.apply(Xd, torch.full_like(Xd, float("nan")))
            torch.cuda.synchronize()
            assert torch.equal(Y1, Y2), (nv, cfg)
            assert colrel(Y1.cpu().numpy(), Yref) <= TOL, (nv, cfg)
            ran += 1
        assert ran >= 1
        # accumulate: Y += A X on top of a given Y, also in colour order
        op.set_launch(False, -1)
        Y0 = torch.from_numpy(np.random.default_rng(9).uniform(-1, 1, X.shape)).to(dev())
        Ya = Y0.clone()
        op.apply(Xd, Ya, accumulate=True)
        torch.cuda.synchronize()
        assert colrel(Ya.cpu().numpy(), Y0.cpu().numpy() + Yref) <= TOL


def test_deterministic_at_config2_size_is_bitwise_stable():
    """Config 2 (16^3 cells, p = 6, 64 columns): three deterministic applies are
    bitwise equal, in FP64 and in the FP32 vector apply; they agree with the
    atomic assembly to rounding, and switching back restores the atomic path."""
    w = W.config2()
    op = mfmv.Operator.from_workload(w)
    X = torch.from_numpy(w.X()).to(dev())
    Ya = op.apply(X, torch.empty_like(X))
    op.set_deterministic(True)
    for prec in ("fp64", "fp32"):
        runs = [op.apply(X, torch.empty_like(X), precision=prec) for _ in range(3)]
        torch.cuda.synchronize()
        assert all(torch.equal(runs[0], r) for r in runs[1:]), prec
    Yd = op.apply(X, torch.empty_like(X))
    torch.cuda.synchronize()
    rel = float(((Yd - Ya).norm(dim=0) / Ya.norm(dim=0)).max())
    assert rel <= 1e-14
    op.set_deterministic(False)
    Yb = op.apply(X, torch.empty_like(X))
    torch.cuda.synchronize()
    assert float(((Yb - Ya).norm(dim=0) / Ya.norm(dim=0)).max()) <= 1e-14


def test_deterministic_refuses_meshes_it_cannot_colour():
    mesh = W.BoxMesh(n=(1, 2, 2), bc=W.BC_PERIODIC)     # a cell that meets itself
    op = mfmv.Operator(mesh, 2, 3, 1.0, None, 0.0)
    with pytest.raises(mfmv.MfError) as e:
        op.set_deterministic(True)
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED
    lin = np.array([[1.0, 0.3, 0.0], [0.0, 1.0, 0.2], [0.1, 0.0, 1.0]])
    sheared = W.BoxMesh(n=(2, 2, 2), bc=W.BC_PERIODIC, lin=lin)
    op = mfmv.Operator(sheared, 2, 3, 1.0, None, 0.0)
    with pytest.raises(mfmv.MfError) as e:
        op.set_deterministic(True)
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED
