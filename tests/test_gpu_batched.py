"""GPU tests of the batched apply (persistent and per-degree launch shapes, the
latter forking onto side streams) and its graph replay.

Every batched result is compared with the CPU oracle (FP64: per-column
relative error <= 1e-12; FP32: <= 1e-6), for every launch shape, every graph
replay and every mesh of the small batches (which hold every degree the batch
kernels are built for); the 32-mesh config-4 batch is compared on sampled rows
of every mesh.  A captured graph is replayed several times, with unrelated
eager work between the replays.
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


def oracle_results(ws, Xs):
    """Full oracle products of every mesh of a small batch (device tensors)."""
    out = []
    for w, X in zip(ws, Xs):
        orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
        out.append(torch.from_numpy(orc.apply(X.cpu().numpy())).to(dev()))
    return out


def test_small_batches_hold_every_degree():
    degrees = {w.p for w in small_batch()} | {w.p for w in small_batch(seed=9, count=5)}
    assert {2, 4, 6, 8} <= degrees


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_batch_matches_oracle_every_shape(prec, tol):
    ws = small_batch()
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    ref = oracle_results(ws, Xs)
    b = mfmv.Batch(ops, [w.nvec for w in ws], prec)
    for cfg in range(mfmv.BATCH_CFGS):
        b.set_launch(cfg)
        Ys = [torch.full_like(X, float("nan")) for X in Xs]
        b.apply(Xs, Ys)
        torch.cuda.synchronize()
        for i, (Y, R) in enumerate(zip(Ys, ref)):
            assert colrel(Y, R) <= tol, (prec, cfg, i, ws[i].p)


@pytest.mark.parametrize("prec,tol,cfg", [("fp64", 1e-12, 0), ("fp64", 1e-12, 1),
                                          ("fp64", 1e-12, 2), ("fp64", 1e-12, 3),
                                          ("fp64", 1e-12, 4), ("fp64", 1e-12, 5),
                                          ("fp32", 1e-6, 0), ("fp32", 1e-6, 5)])
def test_batch_graph_replays(prec, tol, cfg):
    ws = small_batch(seed=9, count=5)
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    ref = oracle_results(ws, Xs)
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
        for i, (Y, R) in enumerate(zip(Ys, ref)):
            assert colrel(Y, R) <= tol, (rep, i)
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


@pytest.fixture(scope="module")
def config4_oracle_rows():
    """Six sampled rows of every config-4 mesh and their oracle values (the oracle runs
    once for both precisions)."""
    ws = W.config4_meshes()
    out = []
    for i, w in enumerate(ws):
        orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
        rows = np.random.default_rng((5, i)).choice(orc.ndofs, 6, replace=False)
        out.append((rows, orc.apply_rows(w.X(), rows)))
    return ws, out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_config4_batch_matches_oracle_sampled(prec, tol, config4_oracle_rows):
    """The 32-mesh batch (6^3..16^3 cells, p in {4,6,8}, nvec in {16..128}) in its default
    launch shape: sampled rows of every mesh against the oracle, per column."""
    ws, sampled = config4_oracle_rows
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    b = mfmv.Batch(ops, [w.nvec for w in ws], prec)
    Ys = [torch.full_like(X, float("nan")) for X in Xs]
    b.apply(Xs, Ys)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (w, Y, (rows, ref)) in enumerate(zip(ws, Ys, sampled)):
        assert not torch.isnan(Y).any(), i
        got = Y[torch.from_numpy(rows).to(dev())].cpu().numpy()
        rel = float((np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())
        worst = max(worst, rel)
        assert rel <= tol, (i, w.p, w.mesh.n, w.nvec, rel)
    print(f"config 4 {prec}: worst sampled column rel err {worst:.3e}")
