"""GPU tests of the batched apply (persistent and per-degree launch shapes, the
latter forking onto side streams) and its graph replay.

Each batched result must equal the single-operator apply of the same mesh
(FP64: per-column relative difference <= 1e-12), for every launch shape; a
captured graph replayed several times, with unrelated eager work between the
replays, must reproduce the eager result every time.  The single-operator
apply itself is pinned to the oracle in test_gpu_apply.py; one mesh of the
batch is also checked against the oracle here.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fe_oracle as fo
from paper_2208_07129_amd import mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def small_batch(seed=4, count=6):
    rng = np.random.default_rng(seed)
    ws = []
    for i in range(count):
        n = int(rng.integers(2, 5))
        p = int(rng.choice([2, 4, 6, 8]))
        nvec = int(rng.choice([3, 8, 16, 21]))
        bc = [W.BC_PERIODIC, W.BC_DIRICHLET0, W.BC_NONE][i % 3]
        m = W.BoxMesh(n=(n, n + 1, n), lo=(0, 0, 0), hi=(1.0, 1.5, 1.2), bc=bc)
        ws.append(W.Workload(f"b{i}", m, p, p + 1, 0.5, W.gaussian_wells((7, i), L=1.0, width=0.3),
                             0.1, nvec, (7, 100 + i)))
    return ws


def colrel(a, b):
    return float((torch.linalg.norm(a - b, dim=0) / torch.linalg.norm(b, dim=0)).max())


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_batch_equals_single_applies_every_shape(prec, tol):
    ws = small_batch()
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    ref = [op.apply(X, precision="fp64") for op, X in zip(ops, Xs)]
    b = mfmv.Batch(ops, [w.nvec for w in ws], prec)
    for cfg in range(mfmv.BATCH_CFGS):
        b.set_launch(cfg)
        Ys = [torch.full_like(X, float("nan")) for X in Xs]
        b.apply(Xs, Ys)
        torch.cuda.synchronize()
        for Y, R in zip(Ys, ref):
            assert colrel(Y, R) <= tol, (prec, cfg)
    # one mesh against the oracle directly
    w = ws[0]
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    Yref = orc.apply(Xs[0].cpu().numpy())
    err = np.linalg.norm(Ys[0].cpu().numpy() - Yref, axis=0) / np.linalg.norm(Yref, axis=0)
    assert err.max() <= tol


@pytest.mark.parametrize("prec,tol,cfg", [("fp64", 1e-12, 0), ("fp64", 1e-12, 3),
                                          ("fp64", 1e-12, 4), ("fp64", 1e-12, 5),
                                          ("fp32", 1e-6, 5)])
def test_batch_graph_replays(prec, tol, cfg):
    ws = small_batch(seed=9, count=5)
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    ref = [op.apply(X) for op, X in zip(ops, Xs)]
    b = mfmv.Batch(ops, [w.nvec for w in ws], prec)
    b.set_launch(cfg)
    Ys = [torch.full_like(X, float("nan")) for X in Xs]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    b.capture(Xs, Ys, s)
    for rep in range(4):
        for Y in Ys:
            Y.fill_(float("nan"))           # eager work between replays
        torch.cuda.synchronize()
        b.replay(s)
        s.synchronize()
        for Y, R in zip(Ys, ref):
            assert colrel(Y, R) <= tol, rep
    # a new launch shape drops the graph captured with the old one
    b.set_launch((cfg + 1) % mfmv.BATCH_CFGS)
    with pytest.raises(mfmv.MfError) as e:
        b.replay(s)
    assert e.value.status == mfmv.MF_ERR_ARG


def test_batch_rejects_unsupported():
    m = W.BoxMesh(n=(2, 2, 2), bc=W.BC_PERIODIC)
    op = mfmv.Operator(m, 2, 4, 0.5, None, 0.0)  # q != p + 1
    with pytest.raises(mfmv.MfError) as e:
        mfmv.Batch([op], [4])
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED
    op2 = mfmv.Operator(m, 2, 3, 0.5, None, 0.0)
    b = mfmv.Batch([op2, op2], [4, 4])
    X = torch.zeros((op2.ndofs, 4), dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        b.apply([X, X], [X, torch.zeros_like(X)])   # output overlaps an input
    assert e.value.status == mfmv.MF_ERR_ARG


def test_config4_batch_matches_single_sampled():
    """The 32-mesh batch (6^3..16^3 cells, p in {4,6,8}, nvec in {16..128}): batched FP64
    equals per-mesh applies on every mesh (checked on 8 of them for time)."""
    ws = W.config4_meshes()
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    b = mfmv.Batch(ops, [w.nvec for w in ws], "fp64")
    Ys = [torch.empty_like(X) for X in Xs]
    b.apply(Xs, Ys)
    torch.cuda.synchronize()
    for i in range(0, 32, 4):
        R = ops[i].apply(Xs[i])
        assert colrel(Ys[i], R) <= 1e-12, i
