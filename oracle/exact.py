"""Closed forms and brute force that pin the oracle (FP64, CPU).

Test infrastructure only.  Nothing here is a step of the method; these are the
independent facts the CTMRG oracles are checked against.

  * Onsager's free energy of the square-lattice Ising model, in two independent
    forms (single quadrature with the elliptic modulus, and the double integral
    over the Brillouin zone).
  * Product-state reductions: for A = |+> or |-> on the physical leg with trivial
    virtual legs, the triple-layer network is the 2D Ising network times
    cosh(beta) (resp. sinh(beta)) per site and the norm network is trivial, so
    f = -(ln cosh(beta) + ln kappa_2D)/beta (resp. sinh).
  * Finite-patch contraction: the Lx x Ly patch of fused site tensors with
    product boundary vectors on every dangling leg, contracted site by site.
  * Central finite differences of a scalar function along given directions.
"""
import numpy as np
from scipy import integrate, special


def onsager_log_kappa(beta):
    """ln kappa of the 2D square-lattice Ising model (J = 1), single-integral form:
    ln(2 cosh 2b) + (1/pi) int_0^{pi/2} ln[(1 + sqrt(1 - k^2 sin^2 t))/2] dt,
    k = 2 sinh 2b / cosh^2 2b."""
    k = 2.0 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    I, _ = integrate.quad(
        lambda t: np.log((1.0 + np.sqrt(1.0 - (k * np.sin(t)) ** 2)) / 2.0),
        0.0, np.pi / 2, epsabs=1e-15, epsrel=1e-15, limit=200)
    return float(np.log(2.0 * np.cosh(2 * beta)) + I / np.pi)


def onsager_log_kappa_double(beta):
    """Same quantity from the double integral
    ln 2 + (1/(8 pi^2)) int int ln[cosh^2 2b - sinh 2b (cos t1 + cos t2)] dt1 dt2
    over [0, 2pi]^2 (evaluated on [0, pi]^2 by symmetry)."""
    c2, s2 = np.cosh(2 * beta) ** 2, np.sinh(2 * beta)
    I, _ = integrate.dblquad(
        lambda t2, t1: np.log(c2 - s2 * (np.cos(t1) + np.cos(t2))),
        0.0, np.pi, 0.0, np.pi, epsabs=1e-13, epsrel=1e-13)
    return float(np.log(2.0) + 4.0 * I / (8.0 * np.pi ** 2))


def onsager_nn_correlation(beta):
    """Nearest-neighbour <s s'> of the 2D square-lattice Ising model (J = 1):
    (1/2) coth(2b) [1 + (2/pi)(2 tanh^2(2b) - 1) K(k)], k = 2 sinh 2b / cosh^2 2b,
    K the complete elliptic integral of the first kind (Onsager's internal
    energy per site, -2 <s s'>)."""
    k = 2.0 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    K = special.ellipk(k * k)
    return float(0.5 / np.tanh(2 * beta) * (1.0 + (2.0 / np.pi) * (2.0 * np.tanh(2 * beta) ** 2 - 1.0) * K))


def product_state_f(beta, sign=+1):
    """f for A = |+> (sign=+1) or |-> (sign=-1): -(ln cosh|sinh + ln kappa_2D)/beta."""
    h = np.cosh(beta) if sign > 0 else np.sinh(beta)
    return -(np.log(h) + onsager_log_kappa(beta)) / beta


def product_state_energy(beta, sign=+1):
    """Internal energy per site U = d(beta f)/d beta of the product state
    A = |+> (sign=+1) or |-> (sign=-1): beta f = -(ln cosh|sinh + ln kappa_2D),
    and d ln kappa_2D / d beta is twice Onsager's nearest-neighbour correlation
    (two links per site of the square lattice).  The first term is the link to
    the layer whose spin the state leaves free (tanh beta for |+>)."""
    h = np.tanh(beta) if sign > 0 else 1.0 / np.tanh(beta)
    return -h - 2.0 * onsager_nn_correlation(beta)


def patch_value(a, boundary, Lx, Ly):
    """Contract the Lx x Ly patch of site tensors a[l,u,r,d] whose dangling legs
    all carry the boundary vector.  Row by row, site by site; the state holds the
    Lx downward legs of the rows above plus the horizontal bond being swept."""
    Df = a.shape[0]
    e = boundary
    # state indexed by the Lx vertical legs (left to right); start: top boundary
    state = np.ones(1)
    for _ in range(Lx):
        state = np.kron(state, e)
    state = state.reshape((Df,) * Lx)
    for _ in range(Ly):
        # horizontal bond entering from the left boundary
        cur = np.einsum("...,h->...h", state, e)           # legs (v_0..v_{Lx-1}, h)
        for x in range(Lx):
            # contract vertical leg x (as site 'u') and the horizontal leg (site 'l')
            cur = np.moveaxis(cur, x, -2)                   # (..., u, h)
            cur = np.einsum("...uh,hurd->...dr", cur, a)    # new (d, r)
            cur = np.moveaxis(cur, -2, x)                   # put d back at slot x
        state = np.einsum("...h,h->...", cur, e)            # right boundary
    for _ in range(Lx):
        state = np.tensordot(state, e, axes=([0], [0]))
    return float(state)


def central_fd(fun, x0, directions, h):
    """(fun(x0 + h v) - fun(x0 - h v)) / (2h) for each direction v."""
    return np.array([(fun(x0 + h * v) - fun(x0 - h * v)) / (2 * h) for v in directions])
