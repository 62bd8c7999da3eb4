"""Split-CTMRG reaches the reduced method's value as chi grows (Sec. IV A), on
many seeded random D4-symmetric tensors: a pin of the oracle's reading of the
six-projector scheme that does not come from the split oracle itself.

References: tests/golden/chi_refs.json, written by tests/golden/make_chi_refs.py
(oracle reduced method converged to 1e-12 at chi 64 (D = 2) / 81 (D = 3)).

Domain.  A seed takes part when neither of its networks is period-2 ordered
(oracle.unsplit.leading_pair_degenerate: the converged reduced corner has a
degenerate +-lambda leading pair).  For such staggered networks a one-site
environment can only hold a mixture of the two ordered boundaries; the
reduced method's single symmetric corner fixes that mixture, the D2 split
environment does not (its fixed point then depends on the start), so the
split value need not approach the reduced one.  The exclusion is by that
computed property, recorded in the reference file and rechecked here.

The relative pseudo-inverse cutoff is 1e-10: below the GPU's 1e-8, whose
floor would hide the convergence below ~1e-8, and above the ~1e-12 at which
S^-1/2 amplifies rounding enough to unsettle the iteration (seed 16's norm
network at chi = 32).
"""
import json
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

REFS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chi_refs.json")
CHIS = {2: (8, 16, 32), 3: (9, 18)}
# bound on the gap at the largest chi (D = 3 at chi = 2 D^2 converges more slowly)
LAST = {2: 1e-6, 3: 3e-4}
# D = 3: the regular seeds whose split iteration settles within 200 moves at
# these chi (seed 9 converges too slowly for this suite; seed 8 is covered at
# chi = 27 separately, where the half projector 4 does not settle)
SEEDS3 = (0, 2, 3, 6, 7, 10, 12, 13)


def _load():
    with open(REFS) as fh:
        return json.load(fh)


def _split_errors(args):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return _split_errors_1(args)


def _split_errors_1(args):
    D, seed, beta, lk3, lk2, chis = args
    from oracle import model, split
    from synth_inputs import raw_peps
    A = model.d4_symmetrize(raw_peps(D, seed))
    A /= np.linalg.norm(A)
    out = []
    for chi in chis:
        row = []
        for O, ref in ((model.pepo_O(beta), lk3), (model.identity_pepo(), lk2)):
            env, it, _, _ = split.run(A, O, chi, 200, 1e-10, 1e-10)
            row.append(abs(split.log_kappa(env, A, O)[0] - ref))
        out.append(row)
    return seed, np.array(out)


@pytest.mark.parametrize("D", [2, 3])
def test_split_converges_to_reduced_value_on_regular_seeds(D):
    refs = [r for r in _load() if r["D"] == D and not any(r["period2"])]
    if D == 3:
        refs = [r for r in refs if r["seed"] in SEEDS3]
    assert len(refs) >= (12 if D == 2 else 8)
    jobs = [(D, r["seed"], r["beta"], r["log_kappa3"], r["log_kappa2"], CHIS[D]) for r in refs]
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(_split_errors, jobs))
    bad = []
    for seed, e in res:
        first, last = e[0], e[-1]
        # converged at the largest chi, and the gap falls with chi unless it
        # already sits at the reference's own level (~1e-8)
        ok = np.all(last < LAST[D]) and np.all(last <= np.maximum(0.3 * first, 1e-7))
        if not ok:
            bad.append((seed, e.tolist()))
    assert not bad, bad


def test_period2_exclusions_are_recomputed():
    """The seeds left out above are period-2 by a fresh oracle run."""
    from oracle import model, unsplit
    from synth_inputs import raw_peps
    for r in _load():
        if r["D"] != 2 or not any(r["period2"]):
            continue
        A = model.d4_symmetrize(raw_peps(2, r["seed"]))
        A /= np.linalg.norm(A)
        net = 0 if r["period2"][0] else 1
        a = model.fuse_triple(A, model.pepo_O(r["beta"])) if net == 0 else model.fuse_double(A)
        dims = (2, 2, 2) if net == 0 else (2, 2)
        C, _, _, _ = unsplit.run(a, dims, 24, 400, 1e-12)
        assert unsplit.leading_pair_degenerate(C), r["seed"]


def test_full_projector4_converges_to_reduced_value():
    """The full projector 4 (Appendix, Fig. Projector4(a)) reaches the reduced
    method's value as chi grows on the same kind of seeds (its
    rho_B rho_T is a four-corner product whose spectrum decays as the square of
    the half one's; with the 1e-10 cutoff it keeps enough directions here)."""
    from oracle import model, split
    from synth_inputs import raw_peps
    refs = {r["seed"]: r for r in _load() if r["D"] == 2}
    for seed in (9, 11):
        r = refs[seed]
        A = model.d4_symmetrize(raw_peps(2, seed))
        A /= np.linalg.norm(A)
        errs = []
        for chi in (8, 16):
            row = []
            for O, ref in ((model.pepo_O(r["beta"]), r["log_kappa3"]), (model.identity_pepo(), r["log_kappa2"])):
                env, _, _, _ = split.run(A, O, chi, 200, 1e-10, 1e-10, p4="full")
                row.append(abs(split.log_kappa(env, A, O)[0] - ref))
            errs.append(row)
        e = np.array(errs)
        assert np.all(e[-1] < 1e-5) and np.all(e[-1] <= np.maximum(0.3 * e[0], 1e-7)), (seed, e)
