"""Site magnetisation from the impurity PEPO in the converged triple-layer
environment (ctm_magnetization), split and reduced method, against the oracle
(oracle.split.magnetization / oracle.unsplit.magnetization) on the same inputs,
and against the spin-flip symmetry."""
import numpy as np
import pytest

from oracle import model, split, unsplit
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
