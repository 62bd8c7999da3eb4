"""Write stored oracle references for GPU parity at sizes the oracle needs
minutes for.  Calls only oracle/ (and the seeded input generator).

Usage: python tests/golden/make_reference.py d5_chi100 30 [reduced]
       python tests/golden/make_reference.py d5_chi100 conv
Output: tests/golden/<workload>_it<n>.npz with f, ln kappa3, ln kappa2, g and
the two corner spectra after n split-CTMRG iterations (the first one
untruncated), FP64, with the workload's relative pseudo-inverse cutoff;
"conv": tests/golden/<workload>_conv.npz, both networks moved together until
the spectrum change of each is below the workload's tol (at most its
max_iter moves), with the move count stored; with
"reduced": tests/golden/<workload>_reduced_it<n>.npz with f, ln kappa3,
ln kappa2 and the corner spectra after n steps of the oracle's reduced method
(eigenvalue cutoff set to the same relative cutoff).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import model, split, unsplit  # noqa: E402
from synth_inputs import WORKLOADS, workload_peps  # noqa: E402


def main(name, n_iter):
    """n_iter > 0: exactly that many moves; n_iter == 0: both networks move
    together until the spectrum change of each is below the workload's tol
    (at most its max_iter moves), as the library iterates them."""
    w = WORKLOADS[name]
    beta, chi = w["beta"], w["chi"]
    A = model.d4_symmetrize(workload_peps(name))
    t0 = time.time()
    nets = {"3": model.pepo_O(beta), "2": model.identity_pepo()}
    env = {k: split.init_env(A.shape[1], O.shape[2]) for k, O in nets.items()}
    s_old = {k: split.corner_spectrum(e) for k, e in env.items()}
    cap = n_iter if n_iter > 0 else w["max_iter"]
    for it in range(1, cap + 1):
        delta = {}
        for k, O in nets.items():
            env[k], _ = split.step(env[k], A, O, chi if it > 1 else split.GROW_CHI, w["svd_cutoff"])
            s = split.corner_spectrum(env[k])
            delta[k] = split.spectrum_delta(s, s_old[k])
            s_old[k] = s
        print("iteration %d  delta3 %.3e  delta2 %.3e  %.0f s" % (it, delta["3"], delta["2"], time.time() - t0),
              flush=True)
        if n_iter == 0 and it > 1 and max(delta.values()) < w["tol"]:
            break
    out = {"iters": it}
    for k, O in nets.items():
        out["log_kappa" + k] = split.log_kappa(env[k], A, O)[0]
        out["spectrum" + k] = split.corner_spectrum(env[k])
    g = split.gradient(beta, A, dict(env3=env["3"], env2=env["2"]))
    f = -(out["log_kappa3"] - out["log_kappa2"]) / beta
    tag = "conv" if n_iter == 0 else "it%d" % n_iter
    path = os.path.join(HERE, "%s_%s.npz" % (name, tag))
    np.savez(path, f=f, log_kappa3=out["log_kappa3"], log_kappa2=out["log_kappa2"], g=g,
             spectrum3=out["spectrum3"], spectrum2=out["spectrum2"], beta=beta, chi=chi,
             n_iter=n_iter, iters=out["iters"], svd_cutoff=w["svd_cutoff"], tol=w["tol"])
    print("wrote", path, "f =", repr(f))


def main_reduced(name, n_iter):
    w = WORKLOADS[name]
    beta, chi = w["beta"], w["chi"]
    unsplit.EIG_CUTOFF = w["svd_cutoff"]
    A = model.d4_symmetrize(workload_peps(name))
    D = A.shape[1]
    O = model.pepo_O(beta)
    t0 = time.time()
    out = {}
    for tag, a, dims in (("3", model.fuse_triple(A, O), (D, O.shape[2], D)), ("2", model.fuse_double(A), (D, D))):
        C, T, _, _ = unsplit.run(a, dims, chi, n_iter)
        print("network %s: %d steps  %.0f s" % (tag, n_iter, time.time() - t0), flush=True)
        out["log_kappa" + tag] = unsplit.log_kappa(C, T, a)[0]
        out["spectrum" + tag] = unsplit.corner_spectrum(C)
    f = -(out["log_kappa3"] - out["log_kappa2"]) / beta
    path = os.path.join(HERE, "%s_reduced_it%d.npz" % (name, n_iter))
    np.savez(path, f=f, log_kappa3=out["log_kappa3"], log_kappa2=out["log_kappa2"],
             spectrum3=out["spectrum3"], spectrum2=out["spectrum2"], beta=beta, chi=chi,
             n_iter=n_iter, eig_cutoff=w["svd_cutoff"])
    print("wrote", path, "f =", repr(f))


if __name__ == "__main__":
    if len(sys.argv) > 3 and sys.argv[3] == "reduced":
        main_reduced(sys.argv[1], int(sys.argv[2]))
    else:
        main(sys.argv[1], 0 if sys.argv[2] == "conv" else int(sys.argv[2]))
