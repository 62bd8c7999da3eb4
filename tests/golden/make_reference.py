"""Write stored oracle references for GPU parity at sizes the oracle needs
minutes for.  Calls only oracle/ (and the seeded input generator).

Usage: python tests/golden/make_reference.py d5_chi100 30 [reduced]
Output: tests/golden/<workload>_it<n>.npz with f, ln kappa3, ln kappa2, g and
the two corner spectra after n split-CTMRG iterations (the first one
untruncated), FP64, with the workload's relative pseudo-inverse cutoff; with
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
    w = WORKLOADS[name]
    beta, chi = w["beta"], w["chi"]
    A = model.d4_symmetrize(workload_peps(name))
    t0 = time.time()
    out = {}
    for tag, O in (("3", model.pepo_O(beta)), ("2", model.identity_pepo())):
        env = split.init_env(A.shape[1], O.shape[2])
        for it in range(1, n_iter + 1):
            env, _ = split.step(env, A, O, chi if it > 1 else split.GROW_CHI, w["svd_cutoff"])
            print("network %s iteration %d  %.0f s" % (tag, it, time.time() - t0), flush=True)
        lk, _ = split.log_kappa(env, A, O)
        out["log_kappa" + tag] = lk
        out["spectrum" + tag] = split.corner_spectrum(env)
        out["env" + tag] = env
    g = split.gradient(beta, A, dict(env3=out["env3"], env2=out["env2"]))
    f = -(out["log_kappa3"] - out["log_kappa2"]) / beta
    path = os.path.join(HERE, "%s_it%d.npz" % (name, n_iter))
    np.savez(path, f=f, log_kappa3=out["log_kappa3"], log_kappa2=out["log_kappa2"], g=g,
             spectrum3=out["spectrum3"], spectrum2=out["spectrum2"], beta=beta, chi=chi,
             n_iter=n_iter, svd_cutoff=w["svd_cutoff"])
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
        main(sys.argv[1], int(sys.argv[2]))
