"""Host-side plan of the LDS-tiled permute (no device work): which permutes take
the tiled form, through the self-test library's planner hook."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SELFTEST = os.path.join(ROOT, "paper_2506_19339_amd", "libctm_selftest.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SELFTEST):
        pytest.skip("libctm_selftest.so not built")
    L = ctypes.CDLL(SELFTEST)
    L.ctm_selftest_permute_tiled.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                             ctypes.POINTER(ctypes.c_int)]
    return L


def tiled(lib, dims, axes):
    d = (ctypes.c_longlong * len(dims))(*dims)
    a = (ctypes.c_int * len(axes))(*axes)
    return lib.ctm_selftest_permute_tiled(len(dims), d, a)


@pytest.mark.parametrize("dims,axes,want", [
    ((100, 64), (1, 0), 1),                          # plain transpose
    ((20000, 100), (1, 0), 1),
    ((5, 5, 100, 100, 5, 5), (0, 1, 4, 3, 2, 5), 1),  # shared unit of 5 (the last axis stays last)
    ((100, 100), (0, 1), 0),                         # identity
    ((3, 1000), (0, 1), 0),
    ((8, 64, 64), (1, 0, 2), 0),                     # unit of 64 contiguous in both: element-wise
    ((2, 3), (1, 0), 0),                             # too short for a tile
    ((100, 5, 5, 5, 100, 2, 2, 2), (0, 1, 2, 5, 6, 4, 7, 3), 1),   # output runs of 5, 1e7 elements
    ((10, 5, 5, 5, 10, 2, 2, 2), (0, 1, 2, 5, 6, 4, 7, 3), 0),     # the same below 1.25e6 elements
    ((7,), (0,), 0),
])
def test_plan_choice(lib, dims, axes, want):
    assert tiled(lib, dims, axes) == want


@pytest.fixture(scope="module")
def check(lib):
    lib.ctm_selftest_permute_tile_check.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                                    ctypes.POINTER(ctypes.c_int)]
    return lambda dims, axes: lib.ctm_selftest_permute_tile_check(
        len(dims), (ctypes.c_longlong * len(dims))(*dims), (ctypes.c_int * len(axes))(*axes))


def test_tile_index_arithmetic_on_random_permutes(check):
    """The kernel's tile loop replayed on the host: for 400 random permutations
    (rank 1-9, ragged dims, up to 2e5 elements) every tiled plan writes each
    output element once with the right input element; a quarter or more of
    them take the tiled form."""
    rng = np.random.default_rng(23)
    pool = [1, 2, 2, 3, 5, 5, 7, 16, 33, 60, 100, 144]
    tiled = 0
    for _ in range(400):
        rank = int(rng.integers(1, 10))
        dims, n = [], 1
        for _ in range(rank):
            v = int(rng.choice(pool))
            if n * v > 200_000:
                v = int(rng.integers(1, 4))
            dims.append(v)
            n *= v
        axes = [int(a) for a in rng.permutation(rank)]
        r = check(dims, axes)
        assert r >= 0, (dims, axes, r)
        tiled += r
    assert tiled >= 100, tiled


@pytest.mark.parametrize("li,lo,dims", [
    ("vqurkzsbe", "urkzsevqb", (5, 2, 2, 2, 60, 5, 5, 5, 60)),
    ("rnstfvhe", "rnstfhve", (5, 5, 2, 2, 100, 100, 5, 5)),
    ("vadpqurkl", "vdqurkapl", (5, 5, 100, 2, 2, 1, 1, 100, 5)),
    ("vdqurkzs", "vqurkzsd", (5, 100, 2, 2, 2, 100, 5, 5)),
])
def test_tile_index_arithmetic_on_the_move_permutes(check, li, lo, dims):
    assert check(list(dims), [li.index(c) for c in lo]) == 1
