"""Kernel-level numerics of the HIP library on the GPU: the FP64 MFMA GEMM and
the one-sided Jacobi SVD, against NumPy on the same inputs."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SELFTEST = os.path.join(ROOT, "paper_2506_19339_amd", "libctm_selftest.so")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SELFTEST):
        raise OSError("libctm_selftest.so is not built")
    L = ctypes.CDLL(SELFTEST)
    dp = ctypes.POINTER(ctypes.c_double)
    L.ctm_selftest_gemm.argtypes = [ctypes.c_int] * 6 + [dp, dp, dp]
    L.ctm_selftest_jacobi.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K,batch", [(1, 1, 1, 1), (16, 16, 4, 1), (65, 130, 17, 1),
                                         (200, 37, 300, 3), (5, 64, 1, 2), (1000, 100, 1000, 1)])
def test_gemm_matches_numpy(lib, ta, tb, M, N, K, batch):
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((batch, K, M) if ta else (batch, M, K))
    B = rng.standard_normal((batch, N, K) if tb else (batch, K, N))
    C = np.zeros((batch, M, N))
    assert lib.ctm_selftest_gemm(ta, tb, M, N, K, batch, _p(A), _p(B), _p(C)) == 0
    ref = np.matmul(A.transpose(0, 2, 1) if ta else A, B.transpose(0, 2, 1) if tb else B)
    assert np.max(np.abs(C - ref)) <= 1e-13 * max(1.0, K) * np.max(np.abs(ref)) + 1e-300


@pytest.mark.parametrize("m,n", [(1, 1), (8, 8), (33, 17), (64, 64), (100, 100), (300, 120), (256, 256)])
def test_jacobi_svd_matches_numpy(lib, m, n):
    rng = np.random.default_rng(m + 100 * n)
    X = rng.standard_normal((m, n))
    # graded spectrum down to 1e-10 to exercise relative accuracy
    U0, _, V0 = np.linalg.svd(X, full_matrices=False)
    s0 = np.logspace(0, -10, min(m, n))
    X = (U0 * s0) @ V0
    Xcm = np.asfortranarray(X)
    U = np.zeros((n, m))
    V = np.zeros((n, n))
    S = np.zeros(n)
    assert lib.ctm_selftest_jacobi(m, n, _p(Xcm.ravel(order="F").copy()), _p(U), _p(S), _p(V)) == 0
    U = U.T   # columns
    V = V.T
    k = min(m, n)
    s_ref = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(S[:k] - s_ref)) <= 1e-15 * max(m, n) * s_ref[0]
    assert np.all(np.diff(S[:k]) <= 0)
    assert np.allclose((U[:, :k] * S[:k]) @ V[:, :k].T, X, atol=1e-14)
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)
