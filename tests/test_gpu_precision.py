"""Reduced-precision forms of the bulk contractions (FP32 / BF16 products with
FP32 accumulation) against the FP64 oracle.

Bars (relative error of f against the FP64 oracle): FP32 <= 1e-6, BF16 with FP64
refinement <= 1e-5; the gradient is checked at 1e-4 (FP32) and 1e-4 (BF16 +
refinement) in relative l2 norm.  The projector factorisations, the corner
spectrum, the normalisations and f / g are FP64 in every form, so the errors
come from the rounding of the absorption products only.
"""
import os

import numpy as np
import pytest

from oracle import model, split
from paper_2506_19339_amd import ctm
from synth_inputs import WORKLOADS, raw_peps, workload_peps

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CUT = 1e-8


def oracle_run(beta, A, chi, n_iter, tol=0.0, with_logs=False):
    As = model.d4_symmetrize(A)
    O3, O2 = model.pepo_O(beta), model.identity_pepo()
    e3, _, _, _ = split.run(As, O3, chi, n_iter, tol=tol, cutoff=CUT)
    e2, _, _, _ = split.run(As, O2, chi, n_iter, tol=tol, cutoff=CUT)
    l3, _ = split.log_kappa(e3, As, O3)
    l2, _ = split.log_kappa(e2, As, O2)
    g = split.gradient(beta, As, dict(env3=e3, env2=e2))
    if with_logs:
        return -(l3 - l2) / beta, g, l3, l2
    return -(l3 - l2) / beta, g


def rel(a, b):
    return abs(a - b) / abs(b)


def test_fp32_form_fixed_iterations_vs_oracle():
    """D = 3, chi = 30, beta = 0.2216, 40 moves: FP32 products vs FP64 oracle.
    Here f (~0.15) is a small difference of the two per-site logs (~2.7 each),
    so the FP32 bar is put on what each network's contraction yields, ln kappa
    (relative 1e-6), and on f relative to the scale of those logs; the bar on f
    itself is checked at the FP32 workload below, where |f| ~ 6.6."""
    beta, D, chi, n = 0.2216, 3, 30, 40
    A = raw_peps(D, 0)
    fo, go, l3o, l2o = oracle_run(beta, A, chi, n, with_logs=True)
    with ctm.SplitCTM(beta, A, chi, precision=ctm.CTM_FP32, svd_cutoff=CUT) as c:
        assert c.iterate(n)[0] == n
        f, l3, l2 = c.free_energy()
        g = c.grad()
    assert rel(l3, l3o) <= 1e-6 and rel(l2, l2o) <= 1e-6, (l3, l3o, l2, l2o)
    assert abs(f - fo) <= 1e-6 * (abs(l3o) + abs(l2o)) / beta, (f, fo)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_bf16_form_with_fp64_refinement_vs_oracle():
    """D = 3, chi = 30: BF16 products until the spectrum change is below 1e-2,
    then FP64 moves to 1e-10; the oracle converged to 1e-10."""
    beta, D, chi = 0.2216, 3, 30
    A = raw_peps(D, 0)
    fo, go = oracle_run(beta, A, chi, 300, tol=1e-10)
    with ctm.SplitCTM(beta, A, chi, max_iter=300, tol=1e-10, precision=ctm.CTM_BF16,
                      svd_cutoff=CUT, refine=True) as c:
        done, delta, conv = c.iterate(0)
        assert conv, delta
        f, _, _ = c.free_energy()
        g = c.grad()
    assert rel(f, fo) <= 1e-5, (f, fo)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_bf16_phase_alone_is_within_its_own_precision():
    """Without refinement the BF16 phase (here run until its spectrum change is
    below 1e-3) stops at its own floor; f is then accurate to the BF16 level
    only (documented, not a parity claim)."""
    beta, D, chi = 0.2216, 3, 30
    A = raw_peps(D, 0)
    fo, _ = oracle_run(beta, A, chi, 300, tol=1e-10)
    with ctm.SplitCTM(beta, A, chi, max_iter=300, tol=1e-10, precision=ctm.CTM_BF16,
                      svd_cutoff=CUT, lp_tol=1e-3) as c:
        done, delta, conv = c.iterate(0)
        assert conv and delta < 1e-3
        f, _, _ = c.free_energy()
    assert rel(f, fo) <= 1e-2, (f, fo)


def test_fp32_form_d4_chi64_vs_stored_oracle():
    """The FP32 workload (beta = 0.2216, D = 4, chi = 64) run until its FP32
    phase ends (spectrum change below 1e-6, no FP64 refinement), against the
    FP64 oracle converged to tol 1e-9, stored by tests/golden/make_reference.py
    (d4_chi64_conv.npz).  Bar: f relative 5e-6, the sum of two parts.  The
    phase stops one move after the spectrum changes by less than 1e-6; the
    FP64 run contracts by about 0.45 per move here (25 moves to 1e-9), so the
    environment is left about 1e-6 from its fixed point and f, first order in
    it, as far.  FP32 rounding in a contraction over K = chi D^2 = 1024 terms
    adds about sqrt(K) 2^-24 = 2e-6.  (The gradient of an environment converged
    only to the FP32 floor is checked after the refinement, below.)"""
    path = os.path.join(GOLDEN, "d4_chi64_conv.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle reference not generated")
    ref = np.load(path)
    w = WORKLOADS["d4_chi64"]
    A = workload_peps("d4_chi64")
    with ctm.SplitCTM(w["beta"], A, w["chi"], max_iter=w["max_iter"], tol=w["tol"], precision=ctm.CTM_FP32,
                      svd_cutoff=float(ref["svd_cutoff"])) as c:
        done, delta, conv = c.iterate(0)
        assert conv, (done, delta)
        f, _, _ = c.free_energy()
    assert rel(f, float(ref["f"])) <= 5e-6, (f, float(ref["f"]))


def test_fp32_form_with_refinement_d4_chi64_vs_stored_oracle():
    """The same workload with the FP64 refinement after the FP32 phase, to
    tol 1e-9: f relative 1e-9 and g relative l2 1e-6 against the converged
    FP64 oracle."""
    path = os.path.join(GOLDEN, "d4_chi64_conv.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle reference not generated")
    ref = np.load(path)
    w = WORKLOADS["d4_chi64"]
    with ctm.SplitCTM(w["beta"], workload_peps("d4_chi64"), w["chi"], max_iter=w["max_iter"], tol=w["tol"],
                      precision=ctm.CTM_FP32, refine=True, svd_cutoff=float(ref["svd_cutoff"])) as c:
        done, delta, conv = c.iterate(0)
        assert conv, (done, delta)
        f, _, _ = c.free_energy()
        g = c.grad()
    assert rel(f, float(ref["f"])) <= 1e-9, (f, float(ref["f"]))
    assert np.linalg.norm(g - ref["g"]) <= 1e-6 * np.linalg.norm(ref["g"])


def test_reduced_precision_context_reports_fp32_gemm_class():
    """Profile mode attributes the bulk GEMMs of an FP32 context to the
    reduced-precision class and the factorisation GEMMs to the FP64 class."""
    A = raw_peps(2, 0)
    with ctm.SplitCTM(0.2, A, 16, precision=ctm.CTM_FP32, profile=True) as c:
        c.iterate(5)
        n64, _, _, _ = c.kernel_stats(0)
        n32, _, fl32, by32 = c.kernel_stats(3)
    assert n32 > 0 and fl32 > 0 and by32 > 0


def test_factorisation_gemms_are_a_subset_of_the_fp64_class():
    """Class 5 counts the FP64 GEMMs issued by the factorisations: a part of
    class 0, non-empty once a move truncates, with its own event times."""
    A = raw_peps(3, 0)
    with ctm.SplitCTM(0.2, A, 20, profile=True) as c:
        c.iterate(6)
        n0, ms0, fl0, by0 = c.kernel_stats(0)
        n5, ms5, fl5, by5 = c.kernel_stats(5)
        with pytest.raises(ctm.CtmError):
            c.kernel_stats(6)
    assert 0 < n5 < n0 and 0 < fl5 < fl0 and 0 < by5 < by0
    assert 0 < ms5 < ms0


def test_bf16_refinement_large_cores_vs_stored_oracle():
    """BF16 + FP64 refinement at D = 4, chi = 128 (beta = 0.2216): the
    Rayleigh-Ritz cores are 144 wide, above the 128 of the register kernels,
    as in the BF16 workload at D = 6, chi = 144 (block Gram-Schmidt bases,
    LDS Jacobi, the thin power schedule), at a size whose converged oracle run
    is stored (d4_chi128_conv.npz, tests/golden/make_reference.py).  Bar:
    1e-5 relative on f and on the l2 norm of g, the BF16 form's tolerance."""
    path = os.path.join(GOLDEN, "d4_chi128_conv.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle reference not generated")
    ref = np.load(path)
    w = WORKLOADS["d4_chi128"]
    with ctm.SplitCTM(w["beta"], workload_peps("d4_chi128"), w["chi"], max_iter=w["max_iter"], tol=w["tol"],
                      precision=ctm.CTM_BF16, refine=True, svd_cutoff=float(ref["svd_cutoff"])) as c:
        done, delta, conv = c.iterate(0)
        assert conv, (done, delta)
        f, _, _ = c.free_energy()
        g = c.grad()
    assert rel(f, float(ref["f"])) <= 1e-5, (f, float(ref["f"]))
    assert np.linalg.norm(g - ref["g"]) <= 1e-5 * np.linalg.norm(ref["g"])
