"""Kernel-level numerics of the HIP library on the GPU: the FP64 MFMA GEMM
(single pass and split-K), the one-sided Jacobi SVD and the shifted Cholesky QR
factor, against NumPy on the same inputs."""
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
    L.ctm_selftest_gemm.argtypes = [ctypes.c_int] * 6 + [dp, dp, dp, ctypes.c_longlong]
    L.ctm_selftest_gemm_lp.argtypes = [ctypes.c_int] * 7 + [dp, dp, dp, ctypes.c_longlong]
    L.ctm_selftest_permute.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(ctypes.c_int), dp, dp]
    L.ctm_selftest_permute_tiled.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                             ctypes.POINTER(ctypes.c_int)]
    L.ctm_selftest_gemm_splits.argtypes = [ctypes.c_int] * 4 + [ctypes.c_longlong]
    L.ctm_selftest_jacobi.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
    L.ctm_selftest_cholqr.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp]
    L.ctm_selftest_sign_fix.argtypes = [ctypes.c_int] * 3 + [dp, dp]
    ip = ctypes.POINTER(ctypes.c_int)
    L.ctm_selftest_gemm_group.argtypes = [ctypes.c_int] * 3 + [ip, ip, ip, dp, dp, dp, ctypes.c_longlong, ip]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K,batch", [(1, 1, 1, 1), (16, 16, 4, 1), (65, 130, 17, 1),
                                         (200, 37, 300, 3), (5, 64, 1, 2), (1000, 100, 1000, 1)])
def test_gemm_matches_numpy(lib, ta, tb, M, N, K, batch):
    _gemm_case(lib, ta, tb, M, N, K, batch, 0)


@pytest.mark.parametrize("M,N,K", [(65536, 1, 1), (250000, 2, 2), (250000, 4, 1), (65537, 8, 8), (9000, 8, 64),
                                   (1250000, 8, 8), (40000, 25, 50), (70000, 9, 3)])
def test_gemm_skinny_short_k_matches_numpy(lib, M, N, K):
    """Long products with N <= 8, K <= 64 (A, B untransposed, M N >= 65536)
    take the skinny kernel (one thread per row, B in LDS); rows per block that
    do not divide M included, and wider N (tile kernel) beside them."""
    _gemm_case(lib, 0, 0, M, N, K, 1, 0)


def _gemm_case(lib, ta, tb, M, N, K, batch, ws_cap):
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((batch, K, M) if ta else (batch, M, K))
    B = rng.standard_normal((batch, N, K) if tb else (batch, K, N))
    C = np.zeros((batch, M, N))
    assert lib.ctm_selftest_gemm(ta, tb, M, N, K, batch, _p(A), _p(B), _p(C), ws_cap) == 0
    ref = np.matmul(A.transpose(0, 2, 1) if ta else A, B.transpose(0, 2, 1) if tb else B)
    # FP64 dot products of length K: |error| <= K eps sum|a||b| ~ K eps sqrt(K) for N(0,1) data
    assert np.max(np.abs(C - ref)) <= 4e-16 * K * np.sqrt(K) + 1e-300


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("shapes,cap,split", [
    ([(128, 500, 500), (128, 1000, 1000), (100, 1000, 1000)], 1 << 22, True),   # subspace products
    ([(128, 128, 1000), (128, 128, 500), (1, 1, 1)], 1 << 22, True),            # Gram matrices, ragged
    ([(65, 130, 17), (200, 37, 300), (5, 64, 0)], 0, False),                    # no workspace, K = 0
    ([(1000, 1000, 64)] * 3, 1 << 22, False),                                   # enough tiles: no split
    ([(7, 9, 333)] * 16, 1 << 22, True),                                        # the largest group
])
def test_grouped_gemm_matches_numpy(lib, ta, tb, shapes, cap, split):
    rng = np.random.default_rng(len(shapes) + 31 * ta + 7 * tb)
    As, Bs = [], []
    for M, N, K in shapes:
        As.append(rng.standard_normal((K, M) if ta else (M, K)))
        Bs.append(rng.standard_normal((N, K) if tb else (K, N)))
    M = np.array([s[0] for s in shapes], dtype=np.int32)
    N = np.array([s[1] for s in shapes], dtype=np.int32)
    K = np.array([s[2] for s in shapes], dtype=np.int32)
    A = np.concatenate([a.ravel() for a in As])
    B = np.concatenate([b.ravel() for b in Bs])
    C = np.full(int(np.sum(M * N)), np.nan)
    ns = ctypes.c_int(-1)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))  # noqa: E731
    assert lib.ctm_selftest_gemm_group(ta, tb, len(shapes), ip(M), ip(N), ip(K), _p(A), _p(B), _p(C), cap,
                                       ctypes.byref(ns)) == 0
    assert (ns.value > 0) == split
    off = 0
    for (m, n, k), a, b in zip(shapes, As, Bs):
        ref = (a.T if ta else a) @ (b.T if tb else b)
        got = C[off:off + m * n].reshape(m, n)
        off += m * n
        assert np.max(np.abs(got - ref), initial=0.0) <= 4e-16 * k * np.sqrt(k) + 1e-300


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K,batch", [(135, 135, 1000, 1), (135, 1000, 1000, 1), (7, 9, 333, 3),
                                         (64, 64, 4096, 1), (100, 3, 257, 2)])
def test_gemm_split_k_matches_numpy(lib, ta, tb, M, N, K, batch):
    cap = 1 << 22
    assert lib.ctm_selftest_gemm_splits(M, N, K, batch, cap) > 1
    _gemm_case(lib, ta, tb, M, N, K, batch, cap)


@pytest.mark.parametrize("dims,axes", [((7,), (0,)), ((3, 5), (1, 0)), ((2, 3, 4, 5), (3, 1, 0, 2)),
                                       ((5, 2, 100, 2, 5, 2), (4, 0, 5, 2, 1, 3)),
                                       ((100, 5, 5, 2, 2, 5, 5, 2, 2), (0, 2, 4, 6, 8, 1, 3, 5, 7)),
                                       ((1, 1, 3, 1), (3, 2, 1, 0))])
def test_permute_matches_numpy(lib, dims, axes):
    rng = np.random.default_rng(len(dims))
    x = rng.standard_normal(dims)
    out = np.zeros(int(np.prod(dims)))
    d = (ctypes.c_longlong * len(dims))(*dims)
    a = (ctypes.c_int * len(axes))(*axes)
    assert lib.ctm_selftest_permute(len(dims), d, a, _p(np.ascontiguousarray(x)), _p(out)) == 0
    assert np.array_equal(out.reshape([dims[k] for k in axes]), np.transpose(x, axes))


# permutes of the split-CTMRG move (labels of the contraction code, D = 5,
# d = 2; chi = 100, or 60 for the two largest), and random ones
TRACED_PERMUTES = [
    ("vqurkzsbe", "urkzsevqb", (5, 2, 2, 2, 60, 5, 5, 5, 60), 1),
    ("rnqstbfwv", "rnstfvqwb", (5, 5, 2, 2, 2, 5, 60, 5, 60), 1),
    ("rnstfvhe", "rnstfhve", (5, 5, 2, 2, 100, 100, 5, 5), 1),
    ("vadpqurkl", "vdqurkapl", (5, 5, 100, 2, 2, 1, 1, 100, 5), 1),
    ("vdqurkzs", "vqurkzsd", (5, 100, 2, 2, 2, 100, 5, 5), 1),
    ("ibfprnmj", "bfrnjipm", (2, 5, 100, 2, 5, 5, 2, 100), 1),
    ("fblnhqmt", "fblqmhtn", (100, 5, 5, 5, 100, 2, 2, 2), 1),   # output runs of 5, 1e7 elements: tiled
    ("fblnhqmt", "fblqmhtn", (10, 5, 5, 5, 10, 2, 2, 2), 0),     # the same below 1.25e6 elements: element-wise
    ("sonbpmd", "nmdpbos", (5, 2, 100, 100, 2, 5, 5), 1),
]


def _permute_case(lib, dims, axes, seed):
    x = np.random.default_rng(seed).standard_normal(dims)
    out = np.zeros(int(np.prod(dims)))
    d = (ctypes.c_longlong * len(dims))(*dims)
    a = (ctypes.c_int * len(axes))(*axes)
    assert lib.ctm_selftest_permute(len(dims), d, a, _p(np.ascontiguousarray(x)), _p(out)) == 0
    assert np.array_equal(out.reshape([dims[k] for k in axes]), np.transpose(x, axes)), (dims, axes)
    return lib.ctm_selftest_permute_tiled(len(dims), d, a)


@pytest.mark.parametrize("li,lo,dims,tiled", TRACED_PERMUTES)
def test_tiled_permute_of_the_move(lib, li, lo, dims, tiled):
    """The permutes of the contraction code: bit-exact against numpy, in the
    form (LDS-tiled or element-wise) the plan gives them."""
    axes = tuple(li.index(c) for c in lo)
    assert _permute_case(lib, dims, axes, 3) == tiled


def test_tiled_permute_at_the_workload_size(lib):
    """The largest transposition of a D = 5, chi = 100 move (50 M elements,
    400 MB) in the tiled form, bit-exact against numpy."""
    li, lo, dims = "vqurkzsbe", "urkzsevqb", (5, 2, 2, 2, 100, 5, 5, 5, 100)
    axes = tuple(li.index(c) for c in lo)
    assert _permute_case(lib, dims, axes, 5) == 1


def test_random_permutes_tiled_and_elementwise(lib):
    """120 random permutations (rank 1-9, dims from a pool with ragged sizes,
    up to 1.5e6 elements): bit-exact against numpy in both forms; at least a
    quarter of them take the tiled form."""
    rng = np.random.default_rng(17)
    pool = [1, 2, 2, 3, 5, 5, 7, 16, 33, 100, 144]
    tiled = 0
    for case in range(120):
        rank = int(rng.integers(1, 10))
        dims, n = [], 1
        for _ in range(rank):
            v = int(rng.choice(pool))
            if n * v > 1_500_000:
                v = int(rng.integers(1, 4))
            dims.append(v)
            n *= v
        axes = tuple(int(a) for a in rng.permutation(rank))
        tiled += _permute_case(lib, tuple(dims), axes, case)
    assert tiled >= 30, tiled


def _round_bf16(x):
    """float64 -> float32 (nearest even) -> bfloat16 (nearest even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K,batch,cap", [(16, 16, 32, 1, 0), (65, 130, 17, 1, 0), (200, 37, 300, 3, 0),
                                             (135, 1000, 1000, 1, 1 << 22), (1000, 100, 1000, 1, 0)])
def test_gemm_reduced_precision(lib, prec, ta, tb, M, N, K, batch, cap):
    """FP32 / BF16 products with FP32 accumulation: equal to the exact product
    of the rounded operands up to FP32 accumulation error."""
    rng = np.random.default_rng(M + 3 * N + 7 * K + prec)
    A = rng.standard_normal((batch, K, M) if ta else (batch, M, K))
    B = rng.standard_normal((batch, N, K) if tb else (batch, K, N))
    C = np.zeros((batch, M, N))
    assert lib.ctm_selftest_gemm_lp(prec, ta, tb, M, N, K, batch, _p(A), _p(B), _p(C), cap) == 0
    rnd = (lambda x: np.asarray(x, np.float32).astype(np.float64)) if prec == 1 else _round_bf16
    Ar, Br = rnd(A), rnd(B)
    ref = np.matmul(Ar.transpose(0, 2, 1) if ta else Ar, Br.transpose(0, 2, 1) if tb else Br)
    mag = np.matmul(np.abs(Ar.transpose(0, 2, 1) if ta else Ar), np.abs(Br.transpose(0, 2, 1) if tb else Br))
    # FP32 accumulation of K products: |error| <= ~K u32 sum|a||b|, u32 = 2^-24
    assert np.all(np.abs(C - ref) <= 2.0 * K * 2.0 ** -24 * mag + 1e-300)
    # and the rounding of the operands is what separates C from the FP64 product
    exact = np.matmul(A.transpose(0, 2, 1) if ta else A, B.transpose(0, 2, 1) if tb else B)
    u = 2.0 ** -24 if prec == 1 else 2.0 ** -8
    assert np.max(np.abs(C - exact) / (np.abs(exact).max() + 1e-300)) <= 4 * u * np.sqrt(K) + 1e-6 * (prec == 1)


@pytest.mark.parametrize("k,rank", [(1, 1), (9, 9), (16, 16), (63, 63), (65, 65), (100, 100), (127, 127),
                                    (128, 128), (128, 90), (135, 135), (135, 90), (141, 141), (160, 160)])
def test_cholqr_factor(lib, k, rank):
    """T = L^-1 D with L L^T = D G D + shift I, T lower triangular (k <= 128:
    register-resident kernel; 135, 141: LDS; 160: global memory).  Full rank: T matches LAPACK's factor.
    Rank deficient: the factor is as ill-conditioned as 1/shift, so what is
    checked is the property the subspace iteration needs, that two passes
    give orthonormal rows."""
    rng = np.random.default_rng(k + rank)
    Y = rng.standard_normal((k, 3 * k))
    if rank < k:
        Y[rank:] = rng.standard_normal((k - rank, rank)) @ Y[:rank] * 1e-3
    Y *= np.logspace(0, -6, k)[:, None]
    shift = 1e-14

    def factor(Yr):
        G = np.ascontiguousarray(Yr @ Yr.T)
        T = np.zeros((k, k))
        assert lib.ctm_selftest_cholqr(k, _p(G), shift, _p(T)) == 0
        assert np.all(np.triu(T, 1) == 0.0)
        return G, T

    G, T = factor(Y)
    if rank == k:
        d = 1.0 / np.sqrt(np.diag(G))
        L = np.linalg.cholesky(d[:, None] * G * d[None, :] + shift * np.eye(k))
        ref = np.linalg.solve(L, np.diag(d))
        scale = np.abs(ref).max(axis=1, keepdims=True)
        assert np.max(np.abs(T - ref) / scale) <= 1e-12
        Q = T @ Y
        assert np.max(np.abs(Q @ Q.T - np.eye(k))) <= 1e-9
    else:
        Q1 = T @ Y
        _, T2 = factor(Q1)
        Q2 = T2 @ Q1
        assert np.max(np.abs(Q2 @ Q2.T - np.eye(k))) <= 1e-9


@pytest.mark.parametrize("m,n", [(1, 1), (2, 2), (3, 3), (8, 8), (33, 17), (64, 64), (65, 65), (100, 100),
                                 (127, 127), (128, 3), (128, 128), (128, 117), (129, 128), (300, 120), (256, 256)])
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
    sweeps = ctypes.c_int(0)
    assert lib.ctm_selftest_jacobi(m, n, _p(Xcm.ravel(order="F").copy()), _p(U), _p(S), _p(V),
                                   ctypes.byref(sweeps)) == 0
    assert 1 <= sweeps.value < 40, sweeps.value
    U = U.T   # columns
    V = V.T
    k = min(m, n)
    s_ref = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(S[:k] - s_ref)) <= 1e-15 * max(m, n) * s_ref[0]
    assert np.all(np.diff(S[:k]) <= 0)
    assert np.allclose((U[:, :k] * S[:k]) @ V[:, :k].T, X, atol=1e-14)
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("n,off,max_sweeps", [(128, 0.0, 1), (128, 1e-6, 3), (100, 1e-6, 3), (117, 1e-6, 3)])
def test_jacobi_stops_early_on_nearly_diagonal_input(lib, n, off, max_sweeps):
    """The warm Rayleigh-Ritz cores are nearly diagonal.  One-sided Jacobi
    converges quadratically there, and the kernel stops after the first sweep
    whose rotations all had cos^2 < 1e-16 (or that rotated nothing): a
    diagonal input takes one sweep, off-diagonal entries of relative size 1e-6
    at most three; the factorisation still matches numpy."""
    rng = np.random.default_rng(n)
    d = np.logspace(0, -8, n) * rng.choice([-1.0, 1.0], n)
    # off-diagonal entries scaled by the smaller of the two diagonal
    # magnitudes: every pair of columns starts with |cos| ~ 2 off
    X = np.diag(d) + off * rng.standard_normal((n, n)) * np.minimum.outer(np.abs(d), np.abs(d))
    U = np.zeros((n, n))
    V = np.zeros((n, n))
    S = np.zeros(n)
    sweeps = ctypes.c_int(0)
    assert lib.ctm_selftest_jacobi(n, n, _p(np.asfortranarray(X).ravel(order="F").copy()), _p(U), _p(S), _p(V),
                                   ctypes.byref(sweeps)) == 0
    assert 1 <= sweeps.value <= max_sweeps, sweeps.value
    s_ref = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(S - s_ref)) <= 1e-15 * n * s_ref[0]
    assert np.allclose((U.T * S) @ V, X, atol=1e-14)
    assert np.allclose(V @ V.T, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("rows,m,n", [(1, 1, 1), (100, 5000, 1000), (300, 257, 3), (64, 64, 64)])
def test_sign_fix_flips_whole_rows(lib, rows, m, n):
    """Each row pair (u_i, v_i) is negated as a whole exactly when the entry of
    u_i with the largest magnitude (first on ties) is negative; the largest
    entry is placed in the lane that negates first, for every row."""
    rng = np.random.default_rng(rows + m + n)
    U = rng.standard_normal((rows, m))
    V = rng.standard_normal((rows, n))
    for i in range(rows):
        j = (i * 37) % m
        U[i, j] = (-1.0) ** i * (np.max(np.abs(U[i])) + 1.0)
    U0, V0 = U.copy(), V.copy()
    assert lib.ctm_selftest_sign_fix(rows, m, n, _p(U), _p(V)) == 0
    for i in range(rows):
        s = -1.0 if U0[i, np.argmax(np.abs(U0[i]))] < 0 else 1.0
        assert np.array_equal(U[i], s * U0[i]) and np.array_equal(V[i], s * V0[i]), i
