"""GPU test of mf_block_gram_noalloc (the allocation-free Gram block) through the
C ABI: two calls in a row, the second with fewer rows and columns, each equal to
mf_block_gram's result on the same inputs (same kernels and chunking: bitwise),
and the k > 128 refusal."""
import numpy as np
import pytest

from paper_2208_07129_amd import mfmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def gram_noalloc(A, B, C, alpha, beta):
    s = torch.cuda.current_stream().cuda_stream
    k = A.shape[1]
    st = mfmv.lib().mf_block_gram_noalloc(A.shape[0], k, A.data_ptr(), A.stride(0), B.data_ptr(),
                                          B.stride(0), alpha, beta, C.data_ptr(), C.stride(0), s)
    return st


def test_noalloc_gram_matches_gram_on_two_calls():
    rng = np.random.default_rng(21)
    for n, k in ((700003, 128), (12345, 37)):
        A = torch.from_numpy(rng.standard_normal((n, k))).to(dev())
        B = torch.from_numpy(rng.standard_normal((n, k))).to(dev())
        C0 = torch.from_numpy(rng.standard_normal((k, k))).to(dev())
        ref = mfmv.block_gram(A, B, C0.clone(), alpha=0.75, beta=-1.5)
        C = C0.clone()
        assert gram_noalloc(A, B, C, 0.75, -1.5) == 0
        torch.cuda.synchronize()
        assert torch.equal(C, ref), (n, k)
        exact = 0.75 * (A.T @ B) - 1.5 * C0
        assert float((C - exact).abs().max() / exact.abs().max()) <= 1e-12


def test_noalloc_gram_refuses_wide_blocks():
    A = torch.zeros((10, 129), dtype=torch.float64, device=dev())
    C = torch.zeros((129, 129), dtype=torch.float64, device=dev())
    assert gram_noalloc(A, A, C, 1.0, 0.0) == mfmv.MF_ERR_UNSUPPORTED
    assert gram_noalloc(A[:, :64], A[:, :64], A, 1.0, 0.0) == mfmv.MF_ERR_ARG  # C overlaps A
