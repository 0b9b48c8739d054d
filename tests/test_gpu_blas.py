"""GPU parity of the eigensolver's tall-skinny FP64 kernels.  kl_gemm_tall: Out = alpha A S +
beta Out against numpy in FP64, through both forms of the kernel (32-row workgroups with
column groups; for more than 32 columns and at least 16384 rows, 64-row workgroups whose
waves own every column tile), every count of 16-column tiles, more than 128 columns (column
blocks), an empty contraction, padded leading dimensions and beta = 0 (Out not read: it
starts as NaN).  Bar: FP64 products over at most a few hundred terms, relative max error
1e-13 of max |Out|.  kl_gram_tall: C = A^T B over up to 40000 rows (row-range partials added
in order), entrywise within 256 eps of |A|^T |B|, bit-identical on a repeat."""

import numpy as np
import pytest
import torch

import paper_2011_13861_amd as kl
from paper_2011_13861_amd import _binding as B

pytestmark = pytest.mark.gpu

SHAPES = [(300, 7, 5), (1000, 33, 66), (16400, 162, 66), (16400, 130, 100), (16400, 64, 128),
          (16400, 40, 140), (16400, 20, 40), (16384, 250, 33), (17000, 0, 48), (16500, 97, 112),
          (20000, 162, 32), (5000, 64, 90)]


def _padded(a, ld):
    """Column-major device copy of a (rows x cols) with leading dimension ld >= rows."""
    rows, cols = a.shape
    buf = torch.full((max(cols, 1) * ld,), float("nan"), dtype=torch.float64, device="cuda")
    view = buf.as_strided((rows, cols), (1, ld))
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)).cuda())
    return view


@pytest.mark.parametrize("beta", [0.0, -1.3])
@pytest.mark.parametrize("N,m,c", SHAPES, ids=["%dx%dx%d" % s for s in SHAPES])
def test_gemm_tall_matches_numpy(N, m, c, beta):
    rng = np.random.default_rng(N + 7 * m + c)
    A = rng.standard_normal((N, m))
    S = rng.standard_normal((m, c))
    O0 = rng.standard_normal((N, c))
    ref = 0.7 * (A @ S) + beta * O0
    Ad = _padded(A, N + 3) if m else torch.zeros((N, 0), dtype=torch.float64, device="cuda")
    Sd = _padded(S, m + 1) if m else torch.zeros((0, c), dtype=torch.float64, device="cuda")
    Od = _padded(O0, N + 5)
    if beta == 0.0:
        Od.fill_(float("nan"))
    B.gemm_tall(Ad, Sd, Od, alpha=0.7, beta=beta)
    torch.cuda.synchronize()
    got = Od.cpu().numpy()
    scale = max(np.max(np.abs(ref)), 1e-300)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale, (N, m, c, beta)


def test_gemm_tall_stream_order():
    """Queued on a non-default stream after the producer of A, before its consumer."""
    N, m, c = 16500, 70, 70
    rng = np.random.default_rng(3)
    S = rng.standard_normal((m, c))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        Ad = torch.full((m, N), 2.0, dtype=torch.float64, device="cuda").T     # column-major N x m
        Sd = kl.to_device_block(S)
        Od = kl.new_block(N, c)
        B.gemm_tall(Ad, Sd, Od, stream=st)
        tot = Od.sum(dim=0)
    st.synchronize()
    assert np.allclose(tot.cpu().numpy(), N * 2.0 * S.sum(axis=0), rtol=1e-12)


GRAM_SHAPES = [(100, 3, 5), (1000, 64, 32), (17576, 162, 32), (17576, 130, 66), (20000, 200, 140),
               (5000, 65, 128), (333, 97, 17), (129, 1, 1), (40000, 32, 32)]


@pytest.mark.parametrize("N,m,c", GRAM_SHAPES, ids=["%dx%dx%d" % s for s in GRAM_SHAPES])
def test_gram_tall_matches_numpy(N, m, c):
    """C = A^T B against numpy; entrywise error within 256 eps of (|A|^T |B|)_ij (the range
    partials and their ordered sum stay far inside that), and the same bits on a repeat."""
    rng = np.random.default_rng(N + 3 * m + 11 * c)
    A = rng.standard_normal((N, m))
    Bm = rng.standard_normal((N, c))
    Ad, Bd = _padded(A, N + 2), _padded(Bm, N + 7)
    C1 = B.gram_tall(Ad, Bd)
    C2 = B.gram_tall(Ad, Bd)
    torch.cuda.synchronize()
    got = C1.cpu().numpy()
    bound = 256 * np.finfo(np.float64).eps * (np.abs(A).T @ np.abs(Bm))
    assert np.all(np.abs(got - A.T @ Bm) <= bound), (N, m, c)
    assert np.array_equal(got, C2.cpu().numpy())


def test_gram_tall_empty_and_workspace():
    """N = 0 gives C = 0; a workspace smaller than kl_gram_tall_workspace is refused."""
    import ctypes
    C = B.gram_tall(torch.zeros((0, 4), dtype=torch.float64, device="cuda"),
                    torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert C.shape == (4, 3) and np.all(C.cpu().numpy() == 0.0)
    N, m, c = 5000, 40, 20
    A = kl.new_block(N, m)
    Bd = kl.new_block(N, c)
    Cd = kl.new_block(m, c)
    nw = B.lib().kl_gram_tall_workspace(N, m, c)
    assert nw > 0
    work = torch.empty(nw, dtype=torch.float64, device="cuda")
    st = B.lib().kl_gram_tall(N, m, c, ctypes.c_void_p(A.data_ptr()), N, ctypes.c_void_p(Bd.data_ptr()), N,
                              ctypes.c_void_p(Cd.data_ptr()), ctypes.c_void_p(work.data_ptr()), nw - 1, None)
    assert st == -1
