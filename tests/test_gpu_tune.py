"""GPU tests of the launch-shape tuner (mf_tune, mf_batch_tune) and the one-call
batched apply (mf_apply_batched), through the C ABI.

The tuner times every launch shape built for the operator and keeps the fastest
(the analogue of the paper's sweep of its kernel's batch size and thread-block
shape, Sec. 4, tbl:batchsizeStudy); its JSON cache is keyed by architecture, p,
q, cells, columns and precision.  Whatever shape it picks, the product must
still match the oracle.
"""
import json

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


def colrel(a, b):
    return float((torch.linalg.norm(a - b, dim=0) / torch.linalg.norm(b, dim=0)).max())


def small(seed, p, n, nvec, bc=W.BC_PERIODIC):
    m = W.BoxMesh(n=(n, n, n + 1), lo=(0, 0, 0), hi=(1.0, 1.0, 1.3), bc=bc)
    return W.Workload(f"t{seed}", m, p, p + 1, 0.5, W.gaussian_wells((3, seed), L=1.0, width=0.3),
                      0.2, nvec, (3, seed))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16", 3e-2)])
def test_tune_writes_cache_and_keeps_parity(tmp_path, prec, tol):
    w = small(1, 4, 3, 24)
    op = mfmv.Operator.from_workload(w)
    cache = str(tmp_path / "tune.json")
    rec = op.tune(w.nvec, prec, cache)
    assert rec["cfg"] >= 0 and str(rec["cfg"]) in rec["ms"]
    assert rec["ms"][str(rec["cfg"])] == min(rec["ms"].values())
    db = json.load(open(cache))
    (key, val), = db.items()
    assert key.endswith(f"/p4q5/cells{op.ncells}/nvec24/{prec}") and val["cfg"] == rec["cfg"]
    X = torch.from_numpy(w.X()).to(dev())
    Y = op.apply(X, torch.full_like(X, float("nan")), precision=prec)
    ref = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma).apply(w.X())
    assert colrel(Y, torch.from_numpy(ref).to(dev())) <= tol
    # a second operator of the same shape takes the cached choice without timing
    op2 = mfmv.Operator.from_workload(w)
    rec2 = op2.tune(w.nvec, prec, cache)
    assert rec2["cfg"] == rec["cfg"] and rec2["ms"] == {}


def test_tune_uses_a_planted_cache_entry(tmp_path):
    """A cache entry is taken as it stands: plant a shape that differs from the
    default choice and check that the apply runs it (its result still matches)."""
    w = small(2, 6, 2, 16)
    op = mfmv.Operator.from_workload(w)
    cache = tmp_path / "planted.json"
    probe = mfmv.Operator.from_workload(w)
    key = None
    rec = probe.tune(w.nvec, "fp64", str(tmp_path / "probe.json"))
    key = next(iter(json.load(open(tmp_path / "probe.json"))))
    other = [int(c) for c in rec["ms"] if int(c) != rec["cfg"]][0]
    cache.write_text(json.dumps({key: {"cfg": other, "ms": []}}))
    rec2 = op.tune(w.nvec, "fp64", str(cache))
    assert rec2["cfg"] == other
    X = torch.from_numpy(w.X()).to(dev())
    ref = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma).apply(w.X())
    Y = op.apply(X, torch.full_like(X, float("nan")))
    assert colrel(Y, torch.from_numpy(ref).to(dev())) <= 1e-12


def test_tune_errors(tmp_path):
    w = small(3, 2, 2, 4)
    op = mfmv.Operator.from_workload(w)
    L = mfmv.lib()
    assert L.mf_tune(op._h, 0, 0, None) == mfmv.MF_ERR_ARG
    assert L.mf_tune(op._h, 4, 7, None) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_tune(None, 4, 0, None) == mfmv.MF_ERR_ARG
    bad = str(tmp_path / "no_such_dir" / "t.json").encode()
    assert L.mf_tune(op._h, 4, 0, bad) == mfmv.MF_ERR_ARG
    sheared = W.BoxMesh(n=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1), bc=W.BC_NONE,
                        lin=((1.0, 0.2, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)))
    opg = mfmv.Operator(sheared, 2, 3, 0.5, None, 0.1)
    assert L.mf_tune(opg._h, 4, 0, None) == 0                       # one shape: nothing to time
    assert L.mf_tune(opg._h, 4, 1, None) == mfmv.MF_ERR_UNSUPPORTED  # mixed: box cells only


def test_apply_batched_one_call_matches_oracle_and_reuses_its_batch(tmp_path):
    ws = [small(10 + i, p, n, nv) for i, (p, n, nv) in
          enumerate([(8, 2, 16), (4, 3, 8), (6, 2, 21), (2, 4, 5)])]
    ops = [mfmv.Operator.from_workload(w) for w in ws]
    Xs = [torch.from_numpy(w.X()).to(dev()) for w in ws]
    refs = [torch.from_numpy(fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma).apply(w.X())).to(dev())
            for w in ws]
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
        for rep in range(2):                     # the second call reuses the cached batch
            Ys = [torch.full_like(X, float("nan")) for X in Xs]
            mfmv.apply_batched(ops, Xs, Ys, prec)
            torch.cuda.synchronize()
            for i, (Y, R) in enumerate(zip(Ys, refs)):
                assert colrel(Y, R) <= tol, (prec, rep, i)
    # a tuned shape is remembered for the one-call form of the same batch
    b = mfmv.Batch(ops, [w.nvec for w in ws], "fp64")
    Ys = [torch.empty_like(X) for X in Xs]
    cfg = b.tune(Xs, Ys, str(tmp_path / "batch.json"))
    db = json.load(open(tmp_path / "batch.json"))
    (key, val), = db.items()
    assert "/batch/fp64/" in key and val["cfg"] == cfg and len(val["ms"]) == mfmv.BATCH_CFGS
    Ys = [torch.full_like(X, float("nan")) for X in Xs]
    mfmv.apply_batched(ops, Xs, Ys, "fp64")
    torch.cuda.synchronize()
    for Y, R in zip(Ys, refs):
        assert colrel(Y, R) <= 1e-12
    # destroying an operator drops the cached batches that use it; a new list works
    ops[1].close()
    w2 = small(20, 4, 3, 8)
    op2 = mfmv.Operator.from_workload(w2)
    X2 = torch.from_numpy(w2.X()).to(dev())
    ops2 = [ops[0], op2]
    Ys = [torch.full_like(Xs[0], float("nan")), torch.full_like(X2, float("nan"))]
    mfmv.apply_batched(ops2, [Xs[0], X2], Ys, "fp64")
    torch.cuda.synchronize()
    ref2 = torch.from_numpy(fo.Oracle(w2.mesh, w2.p, w2.q, w2.mu, w2.V, w2.sigma).apply(w2.X())).to(dev())
    assert colrel(Ys[0], refs[0]) <= 1e-12 and colrel(Ys[1], ref2) <= 1e-12


def test_apply_batched_errors():
    w = small(30, 2, 2, 4)
    op = mfmv.Operator.from_workload(w)
    X = torch.zeros((op.ndofs, 4), dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        mfmv.apply_batched([op, op], [X, X], [X, torch.zeros_like(X)])   # output overlaps input
    assert e.value.status == mfmv.MF_ERR_ARG
    m = W.BoxMesh(n=(2, 2, 2), bc=W.BC_PERIODIC)
    opq = mfmv.Operator(m, 2, 4, 0.5, None, 0.0)                           # q != p + 1
    Xq = torch.zeros((opq.ndofs, 4), dtype=torch.float64, device=dev())
    with pytest.raises(mfmv.MfError) as e:
        mfmv.apply_batched([opq], [Xq], [torch.zeros_like(Xq)])
    assert e.value.status == mfmv.MF_ERR_UNSUPPORTED
