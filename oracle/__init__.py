"""FP64 CPU oracle for the split-CTMRG free energy and gradient.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
HIP product path never imports, links or calls it, and it imports nothing from
the product package: the only code both sides share is the seeded input
generator in ``synth_inputs.py``, which holds none of the method's arithmetic.

Modules
  model    -- Ising Boltzmann weight W, sqrt(W), the PEPO tensor O, the D4
              projection of the PEPS tensor, fused (reduced) site tensors.
  unsplit  -- the reduced method: C4v-symmetric CTMRG on the fused triple- and
              double-layer tensors, kappa estimator, f and environment gradient.
  split    -- the split-CTMRG scheme written as plain einsum steps, with the six
              projector pairs built from rho_T / rho_B and the D2 relations.
  exact    -- closed forms and brute force used to pin the two above: Onsager's
              2D Ising free energy, product-state reductions, finite-patch
              contraction, central finite differences.

Every function is FP64 NumPy/SciPy and deliberately unoptimised.
"""
