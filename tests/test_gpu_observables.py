"""Impurity observables in the converged triple-layer environment: the site
magnetisation (ctm_magnetization, split and reduced method) and the in-plane
nearest-neighbour correlation (ctm_bond_correlation, both methods), against
the oracle on the same inputs, the spin-flip symmetry and, for the symmetric
product state, Onsager's nearest-neighbour correlation."""
import numpy as np
import pytest

from oracle import exact, model, split, unsplit
from paper_2506_19339_amd import ctm
from synth_inputs import raw_peps

pytestmark = pytest.mark.gpu

CUT = 1e-8


@pytest.fixture(autouse=True)
def oracle_cutoff(monkeypatch):
    monkeypatch.setattr(unsplit, "EIG_CUTOFF", CUT)


def gpu_m(beta, A, chi, n, method):
    with ctm.SplitCTM(beta, A, chi, svd_cutoff=CUT, method=method) as c:
        assert c.iterate(n)[0] == n
        return c.magnetization()


def oracle_m(beta, A, chi, n, method):
    As = model.d4_symmetrize(A)
    O = model.pepo_O(beta)
    if method == "split":
        env, _, _, _ = split.run(As, O, chi, n, cutoff=CUT)
        return split.magnetization(env, As, beta)
    D = As.shape[1]
    C, T, _, _ = unsplit.run(model.fuse_triple(As, O), (D, 2, D), chi, n)
    return unsplit.magnetization(C, T, As, beta)


@pytest.mark.parametrize("method", ["split", "reduced"])
@pytest.mark.parametrize("beta,D,chi,n,seed", [(0.2, 2, 12, 20, 1), (0.22, 3, 20, 15, 2)])
def test_magnetisation_vs_oracle(method, beta, D, chi, n, seed):
    A = raw_peps(D, seed)
    m, mo = gpu_m(beta, A, chi, n, method), oracle_m(beta, A, chi, n, method)
    assert abs(mo) > 1e-3
    assert abs(m - mo) <= 1e-10, (m, mo)


@pytest.mark.parametrize("method", ["split", "reduced"])
def test_magnetisation_spin_flip_and_symmetric_state(method):
    beta, chi, n = 0.2, 12, 20
    A = raw_peps(2, 1)
    m = gpu_m(beta, A, chi, n, method)
    mf = gpu_m(beta, A[::-1].copy(), chi, n, method)
    assert abs(m + mf) <= 1e-10 * max(1.0, abs(m)), (m, mf)
    assert abs(gpu_m(beta, model.embed_product_state(2, +1), chi, n, method)) <= 1e-12


def test_magnetisation_before_iterating_is_a_state_error():
    with ctm.SplitCTM(0.2, raw_peps(2, 0), 8) as c:
        with pytest.raises(ctm.CtmError) as e:
            c.magnetization()
        assert e.value.status == ctm.CTM_ESTATE


@pytest.mark.parametrize("method", ["split", "reduced"])
@pytest.mark.parametrize("beta,D,chi,n,seed", [(0.2, 2, 12, 20, 1), (0.22, 3, 20, 15, 2)])
def test_bond_correlation_vs_oracle(method, beta, D, chi, n, seed):
    A = raw_peps(D, seed)
    with ctm.SplitCTM(beta, A, chi, svd_cutoff=CUT, method=method) as c:
        assert c.iterate(n)[0] == n
        zz = c.bond_correlation()
    As = model.d4_symmetrize(A)
    O = model.pepo_O(beta)
    if method == "split":
        env, _, _, _ = split.run(As, O, chi, n, cutoff=CUT)
        zo = split.bond_correlation(env, As, beta)
    else:
        C, T, _, _ = unsplit.run(model.fuse_triple(As, O), (D, 2, D), chi, n)
        zo = unsplit.bond_correlation(C, T, As, beta)
    assert abs(zz - zo) <= 1e-10, (zz, zo)


@pytest.mark.parametrize("method,chi,tol", [("split", 16, 1e-9), ("reduced", 24, 1e-10)])
def test_bond_correlation_of_the_product_state_is_onsagers(method, chi, tol):
    """A = (1, 1)/sqrt(2): the triple-layer network is the 2D Ising network up to
    a constant per site, so <sigma sigma'> is the 2D nearest-neighbour value.
    The split environment at chi = 16 with the 1e-8 relative cutoff is within
    ~4e-10 of it (the oracle's split at the same chi without that cutoff: 7e-13)."""
    beta = 0.2
    with ctm.SplitCTM(beta, model.embed_product_state(2, +1), chi, max_iter=400, tol=1e-13, svd_cutoff=CUT,
                      method=method) as c:
        assert c.iterate(0)[2]
        zz = c.bond_correlation()
    assert abs(zz - exact.onsager_nn_correlation(beta)) <= tol, (zz, exact.onsager_nn_correlation(beta))


def test_bond_correlation_before_iterating_is_a_state_error():
    with ctm.SplitCTM(0.2, raw_peps(2, 0), 8) as c:
        with pytest.raises(ctm.CtmError) as e:
            c.bond_correlation()
        assert e.value.status == ctm.CTM_ESTATE
