"""Model and ansatz pieces of the oracle (FP64, CPU).  Test infrastructure only.

Paper passages followed:
  * Sec. II, Eq. (SVD) and the delta-tensor definition: the partition function is
    a network of delta tensors on sites and Boltzmann matrices W on links; each W
    is split in two factors and the six factors around a site are grouped with
    the delta into the uniform PEPO tensor O.
  * Sec. IV (3D Ising benchmark): W = [[e^b, e^-b], [e^-b, e^b]] is symmetric
    positive definite, so the split is the matrix square root W = sqrt(W) sqrt(W)
    obtained from the eigendecomposition W = U lambda U^T.
  * Sec. III B (symmetric scheme): A is real and its virtual legs are projected
    onto the D4-invariant subspace.
  * Sec. II (reduced method, Fig. "reduced method review"): contracting the
    physical legs of A, O and conj(A) gives the single-layer site tensor a3 of
    bond D^2 d; without O one gets the norm-network tensor a2 of bond D^2.

Index conventions (used by every oracle module):
  A[p, l, u, r, d]           ket PEPS tensor, p physical (dim 2), virtual dim D
  O[p, q, l, u, r, d]        PEPO; p meets the ket layer, q the bra layer
  a3[L, U, R, D]             fused leg = (ket, int, bra) in that order
"""
import numpy as np


def ein(spec, *ops):
    """np.einsum with the pairwise BLAS path (the value is the plain sum)."""
    return np.einsum(spec, *ops, optimize=True)

PHYS = 2  # Ising spin: physical dimension of A and of every PEPO leg


def boltzmann_W(beta):
    """Link weight W(s, s') = exp(beta s s') for s, s' in {+1, -1} (Sec. IV)."""
    eb, emb = np.exp(beta), np.exp(-beta)
    return np.array([[eb, emb], [emb, eb]], dtype=np.float64)


def sqrt_W(beta):
    """Matrix square root of W via its eigendecomposition (Sec. IV)."""
    lam, U = np.linalg.eigh(boltzmann_W(beta))
    if np.any(lam <= 0):
        raise ValueError("W must be positive definite (beta > 0)")
    return (U * np.sqrt(lam)) @ U.T


def pepo_O(beta):
    """O[p,q,l,u,r,d] = sum_s sW[s,p] sW[s,q] sW[s,l] sW[s,u] sW[s,r] sW[s,d].

    The delta tensor forces all six legs of W around a site to the same spin s;
    grouping it with one sqrt(W) factor per link gives O (Sec. II, Fig. "tensor
    network representation", panel c)."""
    s = sqrt_W(beta)
    return ein("sp,sq,sl,su,sr,sd->pqlurd", s, s, s, s, s, s)


def pepo_Oz(beta):
    """Impurity PEPO of the spin at a site: O with the spin's value under the
    sum, Oz[p,q,l,u,r,d] = sum_s sigma(s) sW[s,p] sW[s,q] sW[s,l] sW[s,u]
    sW[s,r] sW[s,d] with sigma = +1 for s = 0 and -1 for s = 1 (the local
    observable of Sec. IV B as an impurity tensor).  In the converged
    triple-layer environment <sigma> = n1(Oz) / n1(O)."""
    s = sqrt_W(beta)
    sig = np.array([1.0, -1.0])
    return ein("s,sp,sq,sl,su,sr,sd->pqlurd", sig, s, s, s, s, s, s)


def sqrt_W_dbeta(beta):
    """d sqrt(W) / d beta.  W has the beta-independent eigenvectors (1, 1)/sqrt2
    and (1, -1)/sqrt2 with eigenvalues 2 cosh(beta) and 2 sinh(beta), so only
    the square roots of the eigenvalues move: d sqrt(2 cosh b) = sinh b /
    sqrt(2 cosh b) and d sqrt(2 sinh b) = cosh b / sqrt(2 sinh b)."""
    if beta <= 0:
        raise ValueError("W must be positive definite (beta > 0)")
    Pp = np.array([[0.5, 0.5], [0.5, 0.5]])
    Pm = np.array([[0.5, -0.5], [-0.5, 0.5]])
    return (np.sinh(beta) / np.sqrt(2 * np.cosh(beta))) * Pp + (np.cosh(beta) / np.sqrt(2 * np.sinh(beta))) * Pm


def pepo_dO(beta):
    """d O / d beta: the product rule over the six sqrt(W) factors of O.

    Each link's W = sqrt(W) sqrt(W) is split over its two end sites, so the sum
    over one site's six legs of the single-leg derivatives, in a translation
    invariant environment, counts every link of the site's three once:
    -n1(dO) / n1(O) is the internal energy per site (Sec. IV B, U computed with
    an impurity tensor)."""
    s, ds = sqrt_W(beta), sqrt_W_dbeta(beta)
    out = np.zeros((PHYS,) * 6)
    for k in range(6):
        mats = [ds if j == k else s for j in range(6)]
        out += ein("sp,sq,sl,su,sr,sd->pqlurd", *mats)
    return out


def identity_pepo():
    """PEPO of the norm network <psi|psi>: delta_{pq} with in-plane legs of size 1.

    Inserting it in the triple-layer network turns <psi|T|psi> into <psi|psi>;
    the split scheme then contracts the norm network with the same code."""
    O = np.zeros((PHYS, PHYS, 1, 1, 1, 1))
    for p in range(PHYS):
        O[p, p, 0, 0, 0, 0] = 1.0
    return O


# The eight elements of D4 acting on the cyclic leg order (l, u, r, d):
# identity, rotations by one, two and three quarter turns, and four reflections.
D4_LEG_PERMS = (
    (0, 1, 2, 3),
    (1, 2, 3, 0),
    (2, 3, 0, 1),
    (3, 0, 1, 2),
    (0, 3, 2, 1),  # u <-> d
    (2, 1, 0, 3),  # l <-> r
    (1, 0, 3, 2),  # l <-> u, r <-> d
    (3, 2, 1, 0),  # l <-> d, u <-> r
)


def d4_symmetrize(A):
    """Projection of A[p,l,u,r,d] onto the D4-invariant subspace (Sec. III B):
    the average over the eight permutations of the four virtual legs."""
    out = np.zeros_like(A)
    for perm in D4_LEG_PERMS:
        out += np.transpose(A, (0,) + tuple(1 + k for k in perm))
    return out / len(D4_LEG_PERMS)


def fuse_triple(A, O):
    """Reduced-method site tensor a3 = sum_{p,q} A[p] O[p,q] A[q] (Sec. II).

    Fused leg order (ket, int, bra); bond dimension D^2 d."""
    D = A.shape[1]
    dd = O.shape[2]
    a3 = ein("pabcd,pqefgh,qijkl->aeibfjcgkdhl", A, O, A)
    Df = D * dd * D
    return a3.reshape(Df, Df, Df, Df)


def fuse_double(A):
    """Norm-network site tensor a2 = sum_p A[p] A[p]; fused leg (ket, bra)."""
    D = A.shape[1]
    a2 = ein("pabcd,pijkl->aibjckdl", A, A)
    return a2.reshape(D * D, D * D, D * D, D * D)


def ising_2d_site_z(beta):
    """The 2D site tensor with the spin's value (+1 / -1 for s = 0 / 1) under the
    sum: the impurity of the 2D pins."""
    s = sqrt_W(beta)
    return ein("s,sl,su,sr,sd->lurd", np.array([1.0, -1.0]), s, s, s, s)


def ising_2d_site(beta):
    """Square-lattice 2D Ising site tensor a[l,u,r,d] = sum_s prod_4 sqrt(W)[s,.]
    (the 2D analogue of O, used only to pin the CTMRG core against Onsager)."""
    s = sqrt_W(beta)
    return ein("sl,su,sr,sd->lurd", s, s, s, s)


def embed_product_state(D, sign=+1):
    """A = |+> (sign=+1) or |-> (sign=-1) on the physical leg, with every virtual
    leg fixed to index 0; embedded at virtual dimension D."""
    A = np.zeros((PHYS, D, D, D, D))
    A[0, 0, 0, 0, 0] = 1.0 / np.sqrt(2.0)
    A[1, 0, 0, 0, 0] = sign / np.sqrt(2.0)
    return A
