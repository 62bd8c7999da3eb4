"""Variational optimisation of the PEPS tensor: minimise f(beta, A) over the
D4-symmetric A with L-BFGS (Sec. II: the free energy is minimised with a
quasi-Newton method fed by the gradient g = 2 d f / d conj(A); for real A the
factor 2 and the conjugate combine into d f / d A).

Every evaluation runs on the HIP library: one context holds both converged
environments, and each new A restarts from them (``ctm_reset_tensor``), so an
evaluation near the previous point needs only a few moves.  This module only
keeps the L-BFGS history (a few vectors of 2 D^4 numbers) and the line search.

L-BFGS: two-loop recursion over the last ``history`` curvature pairs,
backtracking line search with the Armijo condition, pairs with s.y <= 0
skipped.  f is invariant under A -> c A and <A, g> = 0, so the iterates stay
in the D4 subspace of the start (g is D4-projected) and their norm changes
only at second order; A is rescaled to unit norm after every step (f does not
change) and the history is kept in the rescaled frame.  Stops when
||g||_inf < gtol (the paper's criterion) or after max_steps.
"""
from dataclasses import dataclass, field

import numpy as np

from . import ctm


@dataclass
class OptResult:
    A: np.ndarray
    f: float
    g_inf: float
    steps: int
    evaluations: int
    moves: int
    converged: bool
    history: list = field(default_factory=list)   # (step, f, ||g||_inf, moves of that step)


class Optimizer:
    def __init__(self, beta, A0, chi, env_tol=1e-10, env_max_iter=300, history=10, method="split",
                 svd_cutoff=0.0, lib=None):
        self.beta = float(beta)
        A = np.asarray(A0, dtype=np.float64)
        self.A = A / np.linalg.norm(A)
        self.m = int(history)
        self._kw = dict(max_iter=env_max_iter, tol=env_tol, svd_cutoff=svd_cutoff, lib=lib, method=method)
        self.chi = int(chi)
        self._ctx = ctm.SplitCTM(self.beta, self.A, self.chi, **self._kw)
        self._first = True
        self.evaluations = 0
        self.moves = 0

    def close(self):
        self._ctx.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def f_and_grad(self, A):
        """(f, g, moves) at A, warm-started from the last converged environments;
        after a failed evaluation (no positive network value, non-finite
        spectrum) the environments start cold once more, and f = +inf if that
        fails too."""
        for attempt in range(2):
            try:
                c = self._ctx
                if not self._first:
                    c.reset_tensor(self.beta, A)
                self._first = False
                done, _, _ = c.iterate(0)
                self.evaluations += 1
                self.moves += done
                f = c.free_energy()[0]
                g = c.grad()
                return f, g, done
            except ctm.CtmError:
                self._ctx.close()
                self._ctx = ctm.SplitCTM(self.beta, A, self.chi, **self._kw)
                self._first = True
        return np.inf, None, 0

    def run(self, max_steps=100, gtol=1e-7, c1=1e-4, callback=None):
        r = lbfgs(self.f_and_grad, self.A, max_steps=max_steps, gtol=gtol, history=self.m, c1=c1,
                  callback=callback)
        self.A = r.A
        r.evaluations, r.moves = self.evaluations, self.moves
        return r



def lbfgs(fg, x0, max_steps=100, gtol=1e-7, history=10, c1=1e-4, first_step=1e-2, callback=None):
    """Minimise a scale-invariant function with L-BFGS.

    fg(x) -> (f, g, cost) with g the gradient (None and f = +inf where f is not
    defined); f(c x) = f(x) is assumed, so every accepted point is rescaled to
    unit norm (and g by the norm).  The first step has length first_step.
    Returns an OptResult (evaluations and moves are filled in by the caller)."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    f, g, cost = fg(x)
    if g is None:
        raise ctm.CtmError(ctm.CTM_ENUMERIC, "the objective is not defined at the start")
    S, Y = [], []
    hist = [(0, f, float(np.max(np.abs(g))), cost)]
    step = 0
    while step < max_steps and np.max(np.abs(g)) >= gtol:
        # two-loop recursion: d = -H g
        q = g.copy()
        al = []
        for s, y in zip(reversed(S), reversed(Y)):
            rho = 1.0 / np.sum(y * s)
            a = rho * np.sum(s * q)
            q -= a * y
            al.append((rho, a, s, y))
        if S:
            q *= np.sum(S[-1] * Y[-1]) / np.sum(Y[-1] * Y[-1])
        else:
            q *= first_step / max(np.linalg.norm(g), 1e-300)
        for rho, a, s, y in reversed(al):
            b = rho * np.sum(y * q)
            q += (a - b) * s
        d = -q
        slope = np.sum(g * d)
        if slope >= 0.0:           # not a descent direction: restart from steepest descent
            S, Y = [], []
            d = -g * (first_step / max(np.linalg.norm(g), 1e-300))
            slope = np.sum(g * d)
        t = 1.0
        while True:
            xn = x + t * d
            fn, gn, cost = fg(xn)
            if gn is not None and fn <= f + c1 * t * slope:
                break
            t *= 0.5
            if t < 1e-10:
                return OptResult(A=x, f=f, g_inf=float(np.max(np.abs(g))), steps=step, evaluations=0,
                                 moves=0, converged=False, history=hist)
        # rescale to unit norm (f and the direction of g are unchanged; g
        # scales with 1 / |x|)
        nrm = np.linalg.norm(xn)
        xn = xn / nrm
        gn = gn * nrm
        s, y = xn - x, gn - g
        if np.sum(s * y) > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > history:
                S.pop(0)
                Y.pop(0)
        x, f, g = xn, fn, gn
        step += 1
        hist.append((step, f, float(np.max(np.abs(g))), cost))
        if callback:
            callback(step, f, g)
    return OptResult(A=x, f=f, g_inf=float(np.max(np.abs(g))), steps=step, evaluations=0, moves=0,
                     converged=bool(np.max(np.abs(g)) < gtol), history=hist)


def minimize(beta, A0, chi, max_steps=100, gtol=1e-7, **kw):
    """Convenience wrapper: run the optimiser and release the device context."""
    with Optimizer(beta, A0, chi, **kw) as opt:
        return opt.run(max_steps=max_steps, gtol=gtol)
