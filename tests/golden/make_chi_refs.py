"""Write the reduced-method references of the split-vs-reduced chi pins.

Calls only oracle/ (and the seeded input generator).  For every seed of the
list it converges the oracle's reduced method (C4v CTMRG on the fused site
tensors) at a large chi and stores ln kappa3 and ln kappa2, and whether the
network is period-2 ordered: the two largest |eigenvalues| of the converged
corner agree to 1e-4 relative (a degenerate +-lambda pair of the transfer
matrix), see oracle.unsplit.leading_pair_degenerate.

Usage: python tests/golden/make_chi_refs.py
Output: tests/golden/chi_refs.json
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

BETA = 0.2
SETS = {2: (list(range(20)), 64), 3: (list(range(16)), 81)}


def one(args):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return one_1(args)


def one_1(args):
    D, seed, chi_ref = args
    import numpy as np
    from oracle import model, unsplit
    from synth_inputs import raw_peps
    A = model.d4_symmetrize(raw_peps(D, seed))
    A /= np.linalg.norm(A)
    _, info = unsplit.free_energy(BETA, A, chi_ref, 800, tol=1e-12)
    return dict(D=D, seed=seed, chi_ref=chi_ref, beta=BETA,
                log_kappa3=info["log_kappa3"], log_kappa2=info["log_kappa2"],
                iters=list(info["iters"]),
                period2=[bool(unsplit.leading_pair_degenerate(info["env3"][0])),
                         bool(unsplit.leading_pair_degenerate(info["env2"][0]))])


def main():
    jobs = [(D, s, chi) for D, (seeds, chi) in SETS.items() for s in seeds]
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        out = list(ex.map(one, jobs))
    path = os.path.join(HERE, "chi_refs.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
