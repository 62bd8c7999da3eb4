"""Host logic of the L-BFGS minimiser (paper_2506_19339_amd.optimize.lbfgs) on
scale-invariant test functions with known minima, on the CPU."""
import numpy as np

from paper_2506_19339_amd.optimize import lbfgs


def rayleigh(Hm):
    """f(x) = x.H.x / x.x: scale invariant, minimum = smallest eigenvalue at its
    eigenvector; gradient 2 (H x - f x) / x.x."""
    def fg(x):
        n2 = np.sum(x * x)
        f = float(x @ Hm @ x / n2)
        return f, 2.0 * (Hm @ x - f * x) / n2, 1
    return fg


def test_rayleigh_quotient_minimum():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    ev = np.linspace(1.0, 30.0, 40)
    Hm = (Q * ev) @ Q.T
    r = lbfgs(rayleigh(Hm), rng.standard_normal(40), max_steps=500, gtol=1e-7)
    assert r.converged
    assert abs(r.f - 1.0) < 1e-12
    assert abs(abs(r.A @ Q[:, 0]) - 1.0) < 1e-8
    fs = [h[1] for h in r.history]
    assert all(b <= a + 1e-15 for a, b in zip(fs, fs[1:]))


def test_undefined_trial_points_are_backtracked():
    """Points where the objective is undefined (f = +inf, no gradient) shrink
    the step; the iteration still reaches the minimum."""
    Hm = np.diag([1.0, 2.0, 5.0])
    base = rayleigh(Hm)

    def fg(x):
        if abs(x[2]) / np.linalg.norm(x) > 0.8:
            return np.inf, None, 0
        return base(x)
    r = lbfgs(fg, np.array([0.3, 0.5, 0.7]), max_steps=200, gtol=1e-7)
    assert r.converged and abs(r.f - 1.0) < 1e-12
