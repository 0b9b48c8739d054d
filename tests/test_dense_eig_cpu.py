"""Host dense symmetric eigensolvers of the library (kl_symeig, kl_symeig_partial, kl_symeig_top), used by
the Rayleigh-Ritz step of the eigensolver, against numpy.linalg.eigh: eigenvalues,
residuals ||A z - w z||, orthonormality, on random matrices, matrices with exactly
repeated eigenvalues (the spectra of symmetric domains), graded spectra and tiny sizes."""

import numpy as np
import pytest

from paper_2011_13861_amd import _binding as B


def _cases():
    rng = np.random.default_rng(0)
    out = []
    for n in (1, 2, 3, 7, 40, 161):
        M = rng.standard_normal((n, n))
        out.append(("random%d" % n, (M + M.T) / 2))
    # exact multiplicities: Q diag(...) Q^T with repeated values
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.concatenate([[3.0, 2.0, 2.0, 2.0, 1.5, 1.5], np.geomspace(1.0, 1e-9, n - 6)])
    out.append(("degenerate", (Q * w) @ Q.T))
    # diagonal (already tridiagonal, zero off-diagonals)
    out.append(("diagonal", np.diag(np.linspace(2.0, -1.0, 25))))
    # graded spectrum as in the Rayleigh-Ritz matrices (eigenvalues over 10 decades)
    Q, _ = np.linalg.qr(rng.standard_normal((120, 120)))
    out.append(("graded", (Q * np.geomspace(1.0, 1e-10, 120)) @ Q.T))
    return out


CASES = _cases()


def _check(A, w, Z, nv):
    n = A.shape[0]
    ref = np.sort(np.linalg.eigvalsh(A))[::-1][:len(w)]
    scale = max(np.max(np.abs(ref)), 1e-300) if len(ref) else 1.0
    assert np.all(np.abs(w - ref) <= 1e-12 * scale * max(1.0, np.sqrt(n)))
    assert np.all(np.diff(w) <= 0)
    if nv:
        R = A @ Z - Z * w[:nv]
        assert np.max(np.linalg.norm(R, axis=0)) <= 1e-11 * scale
        assert np.max(np.abs(Z.T @ Z - np.eye(nv))) <= 1e-11


@pytest.mark.parametrize("name,A", CASES, ids=[c[0] for c in CASES])
def test_symeig_full(name, A):
    w, Z = B.symeig(A)
    _check(A, w, Z, A.shape[0])


@pytest.mark.parametrize("name,A", CASES, ids=[c[0] for c in CASES])
def test_symeig_partial(name, A):
    n = A.shape[0]
    for nv in sorted({0, 1, max(1, n // 3), n}):
        w, Z = B.symeig_partial(A, nv)
        _check(A, w, Z, nv)


@pytest.mark.parametrize("name,A", CASES, ids=[c[0] for c in CASES])
def test_symeig_top(name, A):
    """Only the nv largest pairs (bisection, inverse iteration in cluster groups on host
    threads): the same bars, and the same eigenvectors as the all-eigenvalue path up to sign
    where the eigenvalues are simple."""
    n = A.shape[0]
    for nv in sorted({1, max(1, n // 3), min(n, 66), n}):
        w, Z = B.symeig_top(A, nv)
        assert w.shape == (nv,) and Z.shape == (n, nv)
        _check(A, w, Z, nv)
        wp, Zp = B.symeig_partial(A, nv)
        gaps = np.abs(np.diff(np.sort(np.linalg.eigvalsh(A))[::-1]))
        scale = max(np.max(np.abs(wp)), 1e-300)
        for j in range(nv):
            simple = (j == 0 or gaps[j - 1] > 1e-6 * scale) and (j == n - 1 or gaps[j] > 1e-6 * scale)
            if simple:
                assert abs(abs(Z[:, j] @ Zp[:, j]) - 1.0) <= 1e-9, (name, nv, j)


def test_symeig_top_repeats_and_threads():
    """Repeated calls, and calls from several host threads at once (the thread team serves one
    call at a time, the others run alone), give identical results."""
    import threading
    name, A = CASES[5]
    w0, Z0 = B.symeig_top(A, 40)
    out = [None] * 6

    def run(i):
        out[i] = B.symeig_top(A, 40)

    th = [threading.Thread(target=run, args=(i,)) for i in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for w, Z in out:
        assert np.array_equal(w, w0) and np.array_equal(Z, Z0)


def test_symeig_errors():
    with pytest.raises(B.KLError):
        B.symeig(np.array([[np.nan]]))
    with pytest.raises(B.KLError):
        B.symeig_partial(np.eye(3), 4)
    with pytest.raises(B.KLError):
        B.symeig_top(np.eye(3), 4)
    with pytest.raises(B.KLError):
        B.symeig_top(np.array([[1.0, np.inf], [np.inf, 1.0]]), 1)


def test_gemm_tall_argument_errors():
    """kl_gemm_tall rejects bad sizes, leading dimensions and pointers before any device work
    (so on the host alone), and returns at once for an empty output."""
    import ctypes
    L = B.lib()
    P = ctypes.c_void_p(16)          # never dereferenced: every call below fails its checks first
    assert L.kl_gemm_tall(-1, 2, 2, P, 4, P, 2, 1.0, 0.0, P, 4, None) == -1
    assert L.kl_gemm_tall(4, -2, 2, P, 4, P, 2, 1.0, 0.0, P, 4, None) == -1
    assert L.kl_gemm_tall(4, 2, 2, P, 3, P, 2, 1.0, 0.0, P, 4, None) == -1        # lda < N
    assert L.kl_gemm_tall(4, 2, 2, P, 4, P, 1, 1.0, 0.0, P, 4, None) == -1        # lds < m
    assert L.kl_gemm_tall(4, 2, 2, P, 4, P, 2, 1.0, 0.0, P, 3, None) == -1        # ldo < N
    assert L.kl_gemm_tall(4, 2, 2, None, 4, P, 2, 1.0, 0.0, P, 4, None) == -1     # A NULL
    assert L.kl_gemm_tall(4, 2, 2, P, 4, P, 2, 1.0, 0.0, None, 4, None) == -1     # Out NULL
    assert L.kl_gemm_tall(0, 2, 2, None, 0, None, 2, 1.0, 0.0, None, 0, None) == 0  # nothing to do
    assert L.kl_gemm_tall(4, 2, 0, None, 4, None, 2, 1.0, 0.0, None, 4, None) == 0


def test_gram_tall_argument_errors():
    """kl_gram_tall and its workspace query reject bad arguments on the host alone."""
    import ctypes
    L = B.lib()
    P = ctypes.c_void_p(16)
    assert L.kl_gram_tall_workspace(-1, 2, 2) == 0 and L.kl_gram_tall_workspace(100, 0, 2) == 0
    assert L.kl_gram_tall_workspace(1000, 64, 32) > 0
    assert L.kl_gram_tall(-1, 2, 2, P, 4, P, 4, P, P, 10 ** 6, None) == -1
    assert L.kl_gram_tall(4, 2, 2, P, 3, P, 4, P, P, 10 ** 6, None) == -1        # lda < N
    assert L.kl_gram_tall(4, 2, 2, P, 4, P, 3, P, P, 10 ** 6, None) == -1        # ldb < N
    assert L.kl_gram_tall(4, 2, 2, P, 4, P, 4, None, P, 10 ** 6, None) == -1     # C NULL
    assert L.kl_gram_tall(4, 2, 2, P, 4, P, 4, P, None, 10 ** 6, None) == -1     # no workspace
    assert L.kl_gram_tall(4, 2, 2, P, 4, P, 4, P, P, 1, None) == -1              # workspace too small
    assert L.kl_gram_tall(4, 0, 2, None, 4, None, 4, None, None, 0, None) == 0   # nothing to do
