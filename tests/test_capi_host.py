"""Host-side logic of the C ABI (no GPU): the library loads, exports every
declared symbol, and its host setup agrees with the oracle's independent
numbering, quadrature points and 1D tables; argument errors are reported
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fe_oracle as fo
from paper_2208_07129_amd import mfmv
from workloads import BoxMesh, BC_NONE, BC_DIRICHLET0, BC_PERIODIC, config1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = mfmv.lib()
    decl = declared_symbols()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(mfmv.EXPORTS) == decl


SHEAR = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])


@pytest.mark.parametrize("bc", [BC_NONE, BC_DIRICHLET0, BC_PERIODIC])
@pytest.mark.parametrize("p", [1, 2, 5])
def test_numbering_and_points_match_oracle(bc, p):
    mesh = BoxMesh(n=(3, 2, 4), lo=(0.0, -1.0, 0.5), hi=(1.0, 1.0, 2.0), bc=bc, lin=SHEAR)
    orc = fo.Oracle(mesh, p, p + 2, mu=0.5)
    assert mfmv.num_dofs(mesh, p) == orc.ndofs
    assert mfmv.num_cells(mesh) == orc.E
    np.testing.assert_array_equal(mfmv.constrained_mask(mesh, p), orc.constrained)
    np.testing.assert_allclose(mfmv.quad_points(mesh, p + 2), orc.xq, atol=1e-13)


@pytest.mark.parametrize("p", range(1, 11))
def test_basis_tables(p):
    for q in range(p + 1, p + 4):
        b = mfmv.basis_1d(p, q)
        xg, wg = np.polynomial.legendre.leggauss(q)
        np.testing.assert_allclose(b["xq"], xg, atol=1e-14)
        np.testing.assert_allclose(b["wq"], wg, atol=1e-14)
        np.testing.assert_allclose(b["xn"], fo.gll_nodes(p), atol=1e-14)
        np.testing.assert_allclose(b["N"], fo.lagrange_values(b["xn"], xg), atol=1e-13)
        np.testing.assert_allclose(b["D"], fo.lagrange_derivatives(b["xn"], xg), atol=1e-11)
        # eq. DU: D1D = Dt N1D (exact because q >= p+1)
        np.testing.assert_allclose(b["Dt"] @ b["N"], b["D"], atol=1e-11 * max(1, np.abs(b["D"]).max()))
        # Dt differentiates degree <= q-1 polynomials exactly at the Gauss points
        for k in range(q):
            np.testing.assert_allclose(b["Dt"] @ xg ** k, k * xg ** max(k - 1, 0) if k else 0 * xg,
                                       atol=1e-10)


def test_gauss3_collocation_derivative_closed_form():
    """Dt at the 3 Gauss points (-a, 0, a), a = sqrt(3/5): row at -a is (-3/(2a), 2/a, -1/(2a))."""
    a = np.sqrt(0.6)
    Dt = mfmv.basis_1d(1, 3)["Dt"]
    np.testing.assert_allclose(Dt[0], [-3 / (2 * a), 2 / a, -1 / (2 * a)], atol=1e-14)
    np.testing.assert_allclose(Dt.sum(axis=1), 0.0, atol=1e-14)


def test_argument_errors_without_device_work():
    L = mfmv.lib()
    w = config1()
    m = mfmv.mesh_c(w.mesh)
    out = ctypes.c_void_p()
    # unsupported degree / quadrature
    assert L.mf_create_operator(ctypes.byref(m), 0, 2, 0.5, None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_create_operator(ctypes.byref(m), 11, 12, 0.5, None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_create_operator(ctypes.byref(m), 3, 3, 0.5, None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_create_operator(ctypes.byref(m), 3, 7, 0.5, None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_UNSUPPORTED
    assert b"q must be" in L.mf_last_error()
    # invalid meshes
    bad = mfmv.mesh_c(BoxMesh(n=(0, 2, 2)))
    assert L.mf_create_operator(ctypes.byref(bad), 2, 3, 0.5, None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_ARG
    bad = mfmv.mesh_c(BoxMesh(n=(2, 2, 2), lo=(1, 0, 0), hi=(1, 1, 1)))
    assert L.mf_num_dofs(ctypes.byref(bad), 2, ctypes.byref(ctypes.c_int64())) == mfmv.MF_ERR_ARG
    bad = mfmv.mesh_c(BoxMesh(n=(2, 2, 2), lin=np.diag([1.0, -1.0, 1.0])))
    assert L.mf_num_cells(ctypes.byref(bad), ctypes.byref(ctypes.c_int64())) == mfmv.MF_ERR_ARG
    bad = mfmv.mesh_c(BoxMesh(n=(2, 2, 2), bc=7))
    assert L.mf_num_cells(ctypes.byref(bad), ctypes.byref(ctypes.c_int64())) == mfmv.MF_ERR_UNSUPPORTED
    assert L.mf_num_dofs(None, 2, ctypes.byref(ctypes.c_int64())) == mfmv.MF_ERR_ARG
    # the largest mesh: node numbers are int32, so 2^31 nodes or more are refused
    # before anything is allocated (1291^3 = 2^31 + 4,201,523 nodes at p = 1)
    big = mfmv.mesh_c(BoxMesh(n=(1290, 1290, 1290)))
    nd = ctypes.c_int64()
    assert L.mf_num_dofs(ctypes.byref(big), 1, ctypes.byref(nd)) == mfmv.MF_OK
    assert nd.value == 1291 ** 3 and nd.value >= 2 ** 31
    assert L.mf_create_operator(ctypes.byref(big), 1, 2, 0.5, None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_UNSUPPORTED
    assert b"2^31" in L.mf_last_error()
    # NaN parameters and NULL outputs
    assert L.mf_create_operator(ctypes.byref(m), 2, 3, float("nan"), None, 0.0, ctypes.byref(out)) == mfmv.MF_ERR_ARG
    assert L.mf_create_operator(ctypes.byref(m), 2, 3, 0.5, None, 0.0, None) == mfmv.MF_ERR_ARG
    # apply on a NULL operator, zero with bad sizes
    assert L.mf_apply(None, 1, 2, 4, 4, 4, 0, None) == mfmv.MF_ERR_ARG
    assert L.mf_apply_add(None, 1, 2, 4, 4, 4, 0, None) == mfmv.MF_ERR_ARG
    assert L.mf_zero(None, 4, 4, 4, None) == mfmv.MF_ERR_ARG
    assert L.mf_zero(16, 4, 8, 4, None) == mfmv.MF_ERR_ARG
    assert L.mf_zero(16, 0, 4, 4, None) == mfmv.MF_OK  # nothing to do: no device work
    L.mf_destroy_operator(None)  # ignored
