"""GPU parity of the FP64 fused apply against the CPU oracle (through the C ABI).

Bar: per-column relative error max_j |Y_j - Yref_j|_2 / |Yref_j|_2 <= 1e-12
(FP64 atomics reorder the assembly sums, so results agree to rounding only).
Small meshes are compared in full, over every degree the library builds, all
three boundary conditions, sheared cells (full 3x3 Jacobian scaling), ragged
vector tiles and strided layouts; the benchmark-size workloads are compared
on sampled rows the oracle computes from the cells that touch them, plus
properties that hold at any size.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import fe_oracle as fo
from paper_2208_07129_amd import mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
SHEAR = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])


def dev():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch.device("cuda:0")


def colrel(Y, Yref):
    num = np.linalg.norm(Y - Yref, axis=0)
    den = np.linalg.norm(Yref, axis=0)
    return float((num / np.maximum(den, 1e-300)).max())


def nan_like(X):
    """Output buffer full of NaN: mf_apply must overwrite every row it owns."""
    return torch.full(X.shape, float("nan"), dtype=torch.float64, device=X.device)


def gpu_apply(op, X, precision="fp64"):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev())
    Yd = op.apply(Xd, nan_like(Xd), precision=precision)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


def vfun(x):
    return np.sin(x[..., 0]) + x[..., 1] * x[..., 2] - 0.3


def build_pair(mesh, p, q, mu=0.5, V=vfun, sigma=0.2):
    op = mfmv.Operator(mesh, p, q, mu, V(mfmv.quad_points(mesh, q)) if V else None, sigma)
    orc = fo.Oracle(mesh, p, q, mu, V, sigma)
    return op, orc


def test_config1_full():
    w = W.config1()
    op = mfmv.Operator.from_workload(w)
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    X = w.X()
    Y = gpu_apply(op, X)
    Yref = orc.apply(X)
    assert colrel(Y, Yref) <= TOL
    assert np.all(Y[orc.constrained] == 0.0)


CASES = [
    # p, q, cells, bc, lin, nvec
    (1, 2, (3, 2, 2), W.BC_NONE, None, 5),
    (2, 3, (2, 3, 2), W.BC_DIRICHLET0, SHEAR, 7),
    (2, 5, (1, 1, 1), W.BC_PERIODIC, None, 3),
    (3, 4, (2, 2, 2), W.BC_PERIODIC, SHEAR, 13),
    (3, 6, (2, 1, 3), W.BC_NONE, None, 1),
    (4, 5, (2, 2, 2), W.BC_DIRICHLET0, None, 9),
    (5, 7, (2, 2, 1), W.BC_PERIODIC, SHEAR, 17),
    (6, 7, (2, 2, 2), W.BC_PERIODIC, None, 11),
    (6, 9, (2, 1, 1), W.BC_DIRICHLET0, SHEAR, 4),
    (7, 8, (2, 1, 2), W.BC_NONE, SHEAR, 6),
    (8, 9, (2, 2, 1), W.BC_PERIODIC, None, 10),
    (9, 10, (1, 2, 1), W.BC_DIRICHLET0, None, 3),
    (10, 11, (2, 1, 1), W.BC_PERIODIC, SHEAR, 2),
    (10, 12, (1, 1, 1), W.BC_NONE, None, 5),
]


@pytest.mark.parametrize("p,q,n,bc,lin,nvec", CASES)
def test_small_meshes_full(p, q, n, bc, lin, nvec):
    mesh = W.BoxMesh(n=n, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc, lin=lin)
    op, orc = build_pair(mesh, p, q)
    X = np.random.default_rng(p * 100 + q).uniform(-1, 1, (orc.ndofs, nvec))
    assert colrel(gpu_apply(op, X), orc.apply(X)) <= TOL


def test_strided_layout_and_accumulate():
    mesh = W.BoxMesh(n=(3, 2, 2), bc=W.BC_DIRICHLET0, lin=SHEAR)
    op, orc = build_pair(mesh, 3, 4)
    nvec = 6
    rng = np.random.default_rng(11)
    Xbig = torch.from_numpy(rng.uniform(-1, 1, (orc.ndofs, nvec + 5))).to(dev())
    Ybig = torch.full((orc.ndofs, nvec + 3), 7.0, dtype=torch.float64, device=dev())
    X, Y = Xbig[:, :nvec], Ybig[:, :nvec]
    op.apply(X, Y)
    torch.cuda.synchronize()
    Yref = orc.apply(Xbig[:, :nvec].cpu().numpy())
    assert colrel(Y.cpu().numpy(), Yref) <= TOL
    assert torch.all(Ybig[:, nvec:] == 7.0)           # columns past nvec untouched
    # accumulate: Y0 + A X; constrained rows keep Y0
    Y0 = rng.uniform(-1, 1, (orc.ndofs, nvec))
    Yd = torch.from_numpy(Y0.copy()).to(dev())
    op.apply(X, Yd, accumulate=True)
    torch.cuda.synchronize()
    expect = Y0 + Yref
    assert colrel(Yd.cpu().numpy(), expect) <= TOL
    np.testing.assert_array_equal(Yd.cpu().numpy()[orc.constrained], Y0[orc.constrained])


def test_dirichlet_rows_ignored_and_zeroed():
    w = W.config1()
    op = mfmv.Operator.from_workload(w)
    mask = mfmv.constrained_mask(w.mesh, w.p)
    X = w.X()
    X2 = X.copy()
    X2[mask] = 1e6
    Y, Y2 = gpu_apply(op, X), gpu_apply(op, X2)
    np.testing.assert_array_equal(Y[mask], 0.0)
    assert colrel(Y2, Y) <= TOL


def test_argument_errors_on_device():
    w = W.config1()
    op = mfmv.Operator.from_workload(w)
    X = torch.zeros((op.ndofs, 8), dtype=torch.float64, device=dev())
    L = mfmv.lib()
    s = torch.cuda.current_stream().cuda_stream
    assert L.mf_apply(op._h, X.data_ptr(), X.data_ptr(), 8, 8, 8, 0, s) == mfmv.MF_ERR_ARG     # overlap
    Y = torch.zeros_like(X)
    assert L.mf_apply(op._h, X.data_ptr(), Y.data_ptr(), 8, 4, 8, 0, s) == mfmv.MF_ERR_ARG     # ldx < nvec
    assert L.mf_apply(op._h, X.data_ptr(), Y.data_ptr(), 0, 8, 8, 0, s) == mfmv.MF_ERR_ARG     # nvec < 1
    assert L.mf_apply(op._h, X.data_ptr(), Y.data_ptr(), 8, 8, 8, 9, s) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_apply(op._h, None, Y.data_ptr(), 8, 8, 8, 0, s) == mfmv.MF_ERR_ARG


def chunk_rows(op, orc, nrandom, seed):
    """Rows that cover every XCD range of the launch: for the first and the last cell of
    each of the 8 contiguous ranges of the library's cell order, one cell-interior, one
    face-interior and one vertex node (free nodes only), plus nrandom random rows."""
    order = op.cell_order()
    E = order.size
    n = op.p + 1
    mid = n // 2
    picks = []
    for x in range(8):
        lo, hi = (x * E) // 8, ((x + 1) * E) // 8 - 1
        for c in {int(order[lo]), int(order[hi])}:
            for loc in ((mid, mid, mid), (0, mid, mid), (0, 0, 0)):
                g = int(orc.map[c][loc[0] + n * (loc[1] + n * loc[2])])
                if g >= 0 and not orc.constrained[g]:
                    picks.append(g)
    rng = np.random.default_rng(seed)
    free = np.nonzero(~orc.constrained)[0]
    picks.extend(rng.choice(free, nrandom, replace=False).tolist())
    return np.unique(np.asarray(picks))


def _sampled_parity(w, nrows, seed, precision="fp64", tol=TOL):
    """Sampled rows of the full-size product against the oracle, judged per column, over
    rows from every XCD range's first and last cell plus random rows."""
    op = mfmv.Operator.from_workload(w)
    orc = fo.Oracle(w.mesh, w.p, w.q, w.mu, w.V, w.sigma)
    X = w.X()
    Xd = torch.from_numpy(X).to(dev())
    Yd = op.apply(Xd, nan_like(Xd), precision=precision)
    torch.cuda.synchronize()
    assert not torch.isnan(Yd).any()
    rows = chunk_rows(op, orc, nrows, seed)
    Yrows = Yd[torch.from_numpy(rows).to(dev())].cpu().numpy()
    Yref = orc.apply_rows(X, rows)
    rel = colrel(Yrows, Yref)
    print(f"{w.name} {precision}: {rows.size} rows, max column rel err {rel:.3e}")
    assert rel <= tol, rel
    return op, Xd, Yd


def test_config2_sampled_rows_and_symmetry():
    """Periodic [0,10]^3, 16^3 cells, p=6, q=7, nvec=64 (the benchmark workload)."""
    w = W.config2()
    op, Xd, Yd = _sampled_parity(w, 256, 7)
    # X^T A X is symmetric (A = A^T) at full size
    G = (Xd.T @ Yd).cpu().numpy()
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
    # linearity: A(2 X0 - 3 X1) = 2 A X0 - 3 A X1 on two column blocks
    Z = 2.0 * Xd[:, :32] - 3.0 * Xd[:, 32:]
    YZ = op.apply(Z.contiguous())
    ref = 2.0 * Yd[:, :32] - 3.0 * Yd[:, 32:]
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(YZ - ref) / torch.linalg.norm(ref)) <= 1e-13


def test_config2_stiffness_kernel_at_full_size():
    """V = 0, sigma = 0 on the periodic config-2 mesh: K 1 = 0, so 1^T (A X) = 0 for every X."""
    w = W.config2()
    op = mfmv.Operator(w.mesh, w.p, w.q, w.mu, None, 0.0)
    X = torch.from_numpy(w.X(8)).to(dev())
    Y = op.apply(X)
    colsum = Y.sum(dim=0).abs().max().item()
    assert colsum <= 1e-10 * Y.abs().max().item() * op.ndofs ** 0.5
    one = torch.ones((op.ndofs, 1), dtype=torch.float64, device=dev())
    assert op.apply(one).abs().max().item() <= 1e-12


@pytest.mark.parametrize("nvec", [16, 64, 256])
def test_config3_sampled_rows(nvec):
    """Periodic unit cube, 12^3 cells, p=8, q=9 (nvec 256: the largest multivector of the
    benchmark configurations, 1.8 GB per operand)."""
    _sampled_parity(W.config3(nvec), 16, nvec)


def test_config5_sampled_rows():
    """Periodic [0,10]^3, 20^3 cells, p=6, q=7, sigma=0.5, 128 columns (the solve operator)."""
    _sampled_parity(W.config5(), 256, 5)


BOX_CASES = [
    # p, q, cells, bc, nvec
    (2, 3, (3, 2, 2), W.BC_DIRICHLET0, 19),
    (3, 5, (2, 2, 2), W.BC_PERIODIC, 33),
    (4, 5, (1, 2, 2), W.BC_NONE, 17),
    (6, 7, (2, 2, 2), W.BC_PERIODIC, 21),
    (6, 8, (2, 1, 2), W.BC_DIRICHLET0, 9),
    (8, 9, (2, 1, 1), W.BC_PERIODIC, 13),
    (10, 11, (1, 1, 2), W.BC_NONE, 3),
]


@pytest.mark.parametrize("p,q,n,bc,nvec", BOX_CASES)
def test_box_kernel_every_launch_shape(p, q, n, bc, nvec):
    """Every built launch shape of the axis-aligned-cell kernel, plus the general kernel
    forced on the same box mesh, against the oracle (ragged column tiles).  Each case
    runs with the odd column count given (one column per thread everywhere) and the
    next even one (two-column shapes take their 16-byte path)."""
    mesh = W.BoxMesh(n=n, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc)
    op, orc = build_pair(mesh, p, q)
    cases = []
    for nv in (nvec, nvec + 1):
        X = np.random.default_rng(p * 7 + q + nv).uniform(-1, 1, (orc.ndofs, nv))
        cases.append((X, orc.apply(X)))
    for X, Yref in cases:
        ran = 0
        for cfg in range(mfmv.BOX_CFGS):
            try:
                op.set_launch(False, cfg)
            except mfmv.MfError as e:
                assert e.status == mfmv.MF_ERR_UNSUPPORTED
                continue
            assert colrel(gpu_apply(op, X), Yref) <= TOL, (X.shape[1], cfg)
            ran += 1
        assert ran >= 1
    op.set_launch(True, -1)  # the general kernel on the same box mesh (irreversible)
    for X, Yref in cases:
        assert colrel(gpu_apply(op, X), Yref) <= TOL


@pytest.mark.parametrize("layout", ["odd_ld", "unaligned"])
def test_box_two_column_shapes_fall_back(layout):
    """A two-column launch shape on a call that cannot take 16-byte column pairs (odd
    leading dimension, 8-byte aligned multivectors) runs the one-column shape."""
    mesh = W.BoxMesh(n=(2, 2, 2), bc=W.BC_PERIODIC)
    op, orc = build_pair(mesh, 5, 6)
    nvec = 10
    X = np.random.default_rng(5).uniform(-1, 1, (orc.ndofs, nvec))
    Yref = orc.apply(X)
    ld = nvec + 1 if layout == "odd_ld" else nvec
    off = 0 if layout == "odd_ld" else 1
    Xb = torch.zeros(orc.ndofs * ld + off, dtype=torch.float64, device=dev())
    Yb = torch.full_like(Xb, float("nan"))
    Xb[off:].view(orc.ndofs, ld)[:, :nvec] = torch.from_numpy(X).to(dev())
    for cfg in (0, 2, 3):
        op.set_launch(False, cfg)
        Yb.fill_(float("nan"))
        op.apply_ptr(Xb.data_ptr() + 8 * off, Yb.data_ptr() + 8 * off, nvec, ld, ld)
        torch.cuda.synchronize()
        Y = Yb[off:].view(orc.ndofs, ld)[:, :nvec].cpu().numpy()
        assert colrel(Y, Yref) <= TOL, (layout, cfg)


def test_box_accumulate_and_timing():
    mesh = W.BoxMesh(n=(3, 3, 2), bc=W.BC_DIRICHLET0)
    op, orc = build_pair(mesh, 4, 5)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (orc.ndofs, 12))
    Y0 = rng.uniform(-1, 1, (orc.ndofs, 12))
    Yref = orc.apply(X)
    Xd = torch.from_numpy(X).to(dev())
    Yd = torch.from_numpy(Y0.copy()).to(dev())
    op.timing(8)
    op.apply(Xd, Yd, accumulate=True)
    Y1 = op.apply(Xd, nan_like(Xd))
    n, zero_ms, kern_ms = op.timing_read()
    assert n == 2 and kern_ms > 0.0 and zero_ms >= 0.0
    op.timing(0)
    assert colrel(Yd.cpu().numpy(), Y0 + Yref) <= TOL
    np.testing.assert_array_equal(Yd.cpu().numpy()[orc.constrained], Y0[orc.constrained])
    assert colrel(Y1.cpu().numpy(), Yref) <= TOL


def test_config2_general_kernel_matches_box_kernel():
    """The general-geometry kernel (full 3x3 factor) and the box kernel agree at full size."""
    w = W.config2()
    op = mfmv.Operator.from_workload(w)
    X = torch.from_numpy(w.X(16)).to(dev())
    Yb = op.apply(X, nan_like(X))
    op.set_launch(True, -1)
    Yg = op.apply(X, nan_like(X))
    torch.cuda.synchronize()
    rel = (torch.linalg.norm(Yb - Yg, dim=0) / torch.linalg.norm(Yg, dim=0)).max().item()
    assert rel <= TOL


# ------------------------------------------------ seeded random draws (properties)
def _draws(count=10, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        p = int(rng.integers(1, 9))
        q = p + int(rng.integers(1, 4))
        if p >= 7:
            q = p + 1            # keep the oracle's dense cell matrices small
        bc = int(rng.choice([W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC]))
        n = tuple(int(v) for v in rng.integers(1, 4 if p <= 4 else 3, size=3))
        nvec = int(rng.choice([1, 3, 17, 64, 129, 300]))
        out.append((p, q, bc, n, nvec, int(rng.integers(0, 1 << 30))))
    return out


@pytest.mark.parametrize("p,q,bc,n,nvec,seed", _draws())
def test_random_draws_parity_linearity_permutation(p, q, bc, n, nvec, seed):
    """Seeded draws of degree, quadrature, boundary condition, mesh (one-cell-wide
    periodic meshes included) and column count (ragged tiles up to 300): parity with
    the oracle, linearity, and equivariance under a permutation of the columns."""
    mesh = W.BoxMesh(n=n, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.5), bc=bc)
    op, orc = build_pair(mesh, p, q)
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (orc.ndofs, nvec))
    X2 = rng.uniform(-1, 1, (orc.ndofs, nvec))
    Y = gpu_apply(op, X)
    assert colrel(Y, orc.apply(X)) <= TOL
    Y2 = gpu_apply(op, X2)
    Ylin = gpu_apply(op, 2.5 * X - 0.75 * X2)
    assert colrel(Ylin, 2.5 * Y - 0.75 * Y2) <= TOL
    perm = rng.permutation(nvec)
    Yp = gpu_apply(op, X[:, perm])
    assert colrel(Yp, Y[:, perm]) <= TOL


# ------------------------------------------------ partition emulation (eq. AU)
@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0])
@pytest.mark.parametrize("p", [2, 6])
def test_partition_emulation_equals_global_apply(bc, p):
    """The distributed form of eq. AU without a second GPU: the cells split into two
    sub-boxes (each with its own numbering, interface nodes in both), each applied
    locally, the owned and ghost contributions summed on the host through the
    Boolean maps P^(t); constraints applied as C / C^T on the global rows.  Equals
    the global apply."""
    q = p + 1
    mesh = W.BoxMesh(n=(4, 2, 3), lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.5), bc=bc)
    op, orc = build_pair(mesh, p, q)
    N = fo.nodes_per_dir(mesh, p)
    X = np.random.default_rng(p).uniform(-1, 1, (orc.ndofs, 7))
    Xc = np.where(orc.constrained[:, None], 0.0, X)
    Yg = gpu_apply(op, X)
    Ysum = np.zeros_like(X)
    for part, (lo_x, hi_x, g0) in enumerate([(0.0, 1.0, 0), (1.0, 2.0, 2 * p)]):
        sub = W.BoxMesh(n=(2, 2, 3), lo=(lo_x, 0.0, 0.0), hi=(hi_x, 1.0, 1.5), bc=W.BC_NONE)
        sop = mfmv.Operator(sub, p, q, 0.5, vfun(mfmv.quad_points(sub, q)), 0.2)
        Ns = fo.nodes_per_dir(sub, p)
        gz, gy, gx = np.meshgrid(np.arange(Ns[2]), np.arange(Ns[1]), np.arange(Ns[0]),
                                 indexing="ij")
        rows = ((gx.ravel() + g0) + N[0] * (gy.ravel() + N[1] * gz.ravel()))   # P^(t)
        Ysum[rows] += gpu_apply(sop, Xc[rows])
    Ysum[orc.constrained] = 0.0
    assert colrel(Ysum, Yg) <= TOL
