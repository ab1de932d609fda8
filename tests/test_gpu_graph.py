"""GPU tests of the fused apply under HIP graph capture: mf_apply enqueues
kernels only (the shared-row zero fill is a kernel, no memset, no allocation,
no host synchronisation), so a captured apply replays like the eager call.
Each graph is replayed several times, with eager work that changes X in
between, and every replay is checked against the eager apply of the current X
(and the first against the oracle)."""
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


def vfun(x):
    return np.sin(x[..., 0]) + x[..., 1] * x[..., 2] - 0.3


def colrel(Y, R):
    num = (Y - R).norm(dim=0)
    den = R.norm(dim=0).clamp_min(1e-300)
    return float((num / den).max())


@pytest.mark.parametrize("precision,deterministic,tol", [
    ("fp64", False, 1e-13),     # shared rows summed by atomics: equal to rounding
    ("fp64", True, 0.0),        # colour-ordered assembly: bitwise
    ("fp32", False, 1e-6),
])
def test_captured_apply_replays_like_eager(precision, deterministic, tol):
    p, q, nvec = 4, 5, 16
    mesh = W.BoxMesh(n=(4, 3, 4), lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=W.BC_PERIODIC)
    op = mfmv.Operator(mesh, p, q, 0.5, vfun(mfmv.quad_points(mesh, q)), 0.2)
    if deterministic:
        op.set_deterministic(True)
    orc = fo.Oracle(mesh, p, q, 0.5, vfun, 0.2)
    rng = np.random.default_rng(17)
    X = torch.from_numpy(rng.uniform(-1, 1, (op.ndofs, nvec))).to(dev())
    Y = torch.full_like(X, float("nan"))
    op.apply(X, Y, precision=precision)   # eager warm-up (per-device launch facts cached)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            op.apply(X, Y, precision=precision)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for r in range(4):
        Y.fill_(float("nan"))
        g.replay()
        ref = op.apply(X, torch.empty_like(X), precision=precision)   # eager, same X
        torch.cuda.synchronize()
        assert not torch.isnan(Y).any(), r
        err = colrel(Y, ref)
        assert err <= tol, (r, err)
        if r == 0:
            Yref = orc.apply(X.cpu().numpy())
            assert colrel(Y.cpu(), torch.from_numpy(Yref)) <= (1e-12 if precision == "fp64" else 1e-6)
        X.mul_(-0.5).add_(0.25)          # eager work on the graph's input between replays
