"""L-BFGS minimisation of f(beta, A) on the HIP library (paper_2506_19339_amd.
optimize): the product-state optimum in the disordered phase against its closed
form, and descent of a random D = 2 tensor below the best product state."""
import numpy as np
import pytest

from oracle import exact, model
from paper_2506_19339_amd import optimize
from synth_inputs import raw_peps

pytestmark = pytest.mark.gpu


def test_product_state_optimum_is_the_closed_form():
    """D = 1, beta = 0.2 (below the 3D transition): the best product state is
    A+ = (1, 1)/sqrt(2), whose f has a closed form (2D Ising per-site value of
    the PEPO's row sums).  L-BFGS from (cos 0.3, sin 0.3) reaches ||g||_inf < 1e-7
    there.  The evaluations use the reduced method, whose chi = 16 environment
    of a product state reproduces the closed form to ~1e-12 (split-CTMRG at
    chi = 16 is within ~1e-8 of it)."""
    beta = 0.2
    A = np.zeros((2, 1, 1, 1, 1))
    A[0], A[1] = np.cos(0.3), np.sin(0.3)
    r = optimize.minimize(beta, A, 16, max_steps=60, gtol=1e-7, method="reduced")
    assert r.converged, r.history[-3:]
    assert abs(r.f - exact.product_state_f(beta, 1)) <= 1e-9 * abs(r.f), (r.f, exact.product_state_f(beta, 1))
    a = r.A.ravel() / np.linalg.norm(r.A)
    assert np.allclose(np.abs(a), 1 / np.sqrt(2), atol=1e-6)


def test_random_d2_descends_below_the_product_state():
    """D = 2 from a random D4-symmetric tensor: f never increases, the D = 2
    ansatz goes below the best product state, and the warm-started evaluations
    take fewer moves than the cold first one."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 0))
    r = optimize.minimize(beta, A, 12, max_steps=10, gtol=1e-9)
    fs = [h[1] for h in r.history]
    assert all(b <= a + 1e-12 for a, b in zip(fs, fs[1:])), fs
    assert r.f < exact.product_state_f(beta, 1) - 1e-3, (r.f, fs)
    cold = r.history[0][3]
    warm = [h[3] for h in r.history[1:]]
    assert np.median(warm) < cold, (cold, warm)
