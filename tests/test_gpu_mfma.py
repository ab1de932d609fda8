"""GPU parity of the FP64 matrix-core body (launch shape 10: v_mfma_f64_4x4x4_4b
even-odd contractions, q = p + 1 <= 8) against the CPU oracle, per column at 1e-12.

Covers every degree the body is built for (p = 1 .. 7), all three boundary conditions,
one-cell periodic meshes (nodes repeated inside a cell), column counts that leave
ragged tiles, the accumulating form, and the benchmark workloads on sampled rows over
every XCD range.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fe_oracle as fo
from paper_2208_07129_amd import mfmv

from test_gpu_apply import _sampled_parity, build_pair, colrel, gpu_apply, TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET0, W.BC_NONE])
def test_mfma_every_degree(p, bc):
    mesh = W.BoxMesh(n=(2, 3, 2), lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc)
    op, orc = build_pair(mesh, p, p + 1)
    for nv in (5, 8, 13):
        X = np.random.default_rng(100 * p + nv + bc).uniform(-1, 1, (orc.ndofs, nv))
        Yref = orc.apply(X)
        for cfg in mfmv.BOX_MFMA_CFGS:
            op.set_launch(False, cfg)
            assert colrel(gpu_apply(op, X), Yref) <= TOL, (p, bc, nv, cfg)


@pytest.mark.parametrize("p", [2, 6, 7])
def test_mfma_one_cell_periodic(p):
    """One cell per direction on a periodic mesh: every face node of the cell is the same
    global node as the opposite face's, so the assembly adds several local rows into one."""
    mesh = W.BoxMesh(n=(1, 1, 2), lo=(0, 0, 0), hi=(1.0, 0.8, 1.4), bc=W.BC_PERIODIC)
    op, orc = build_pair(mesh, p, p + 1)
    X = np.random.default_rng(p).uniform(-1, 1, (orc.ndofs, 11))
    Yref = orc.apply(X)
    for cfg in mfmv.BOX_MFMA_CFGS:
        op.set_launch(False, cfg)
        assert colrel(gpu_apply(op, X), Yref) <= TOL, (p, cfg)


def test_mfma_accumulate():
    mesh = W.BoxMesh(n=(3, 2, 2), lo=(0, 0, 0), hi=(1.5, 1.0, 1.0), bc=W.BC_DIRICHLET0)
    op, orc = build_pair(mesh, 6, 7)
    X = np.random.default_rng(3).uniform(-1, 1, (orc.ndofs, 16))
    Y0 = np.random.default_rng(4).uniform(-1, 1, (orc.ndofs, 16))
    ref = Y0 + orc.apply(X)
    ref[orc.constrained] = Y0[orc.constrained]   # constrained rows are left unchanged
    for cfg in mfmv.BOX_MFMA_CFGS:
        op.set_launch(False, cfg)
        Xd = torch.from_numpy(X).to(dev())
        Yd = torch.from_numpy(Y0.copy()).to(dev())
        op.apply(Xd, Yd, accumulate=True)
        torch.cuda.synchronize()
        assert colrel(Yd.cpu().numpy(), ref) <= TOL, cfg


def test_mfma_shapes_need_q_equal_p_plus_1_and_at_most_8_points():
    mesh = W.BoxMesh(n=(2, 2, 2), bc=W.BC_PERIODIC)
    for p, q in ((3, 5), (8, 9), (6, 8)):
        op = mfmv.Operator(mesh, p, q, 0.5, None, 0.0)
        for cfg in mfmv.BOX_MFMA_CFGS:
            with pytest.raises(mfmv.MfError) as e:
                op.set_launch(False, cfg)
            assert e.value.status == mfmv.MF_ERR_UNSUPPORTED


class _Forced:
    """Operator factory that forces a launch shape on every operator it builds."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.orig = mfmv.Operator.from_workload

    def __enter__(self):
        cfg, orig = self.cfg, self.orig

        def build(w):
            op = orig(w)
            op.set_launch(False, cfg)
            return op
        mfmv.Operator.from_workload = build
        return self

    def __exit__(self, *a):
        mfmv.Operator.from_workload = self.orig


@pytest.mark.parametrize("cfg", [10])
def test_mfma_config2_sampled_rows(cfg):
    """The benchmark workload (16^3 periodic cells, p = 6, 64 columns) on the matrix
    cores: sampled rows over every XCD range, per column, at 1e-12."""
    with _Forced(cfg):
        _sampled_parity(W.config2(), 128, 70 + cfg)


def test_mfma_config5_sampled_rows():
    with _Forced(10):
        _sampled_parity(W.config5(), 128, 75)
