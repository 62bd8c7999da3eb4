"""Reduced method: C4v-symmetric CTMRG on the fused site tensor (FP64, CPU).

Test infrastructure only.  Follows Sec. II (reduced method; environment of
corner C and edge T tensors with boundary bond chi, grown by absorbing local
tensors and truncated with projectors) in the C4v-symmetric form that the
symmetric PEPO and D4-symmetric A allow (Sec. III B): one corner C and one
edge T describe all four directions.

Conventions
  C[x, y]        symmetric chi x chi corner matrix
  T[a, m, b]     edge tensor, symmetric in its two chi legs a, b; m meets the site
  a[l, u, r, d]  fused site tensor (C4v symmetric)

Convergence follows Sec. III D: the singular values S of
rho_eff = C^4 / Tr C^4 (here the |eigenvalues|^4 of C, normalised) are compared
between successive steps in the l2 norm, zero-padded to a common length.

The per-site value is the single-site CTM estimator
kappa = n1 * n0 / n2^2 with n1 the 3x3 patch, n2 the 3x2 strip and n0 = Tr C^4
(free-energy expression, Sec. II).  f = -(ln kappa3 - ln kappa2) / beta.
The gradient is the environment of the conjugate tensor in the 3x3 patch,
g = -(2/beta)(E3/n1_3 - E2/n1_2), projected onto the D4 subspace (gradient
expression, Sec. II; projection, Sec. III B).
"""
import numpy as np


def ein(spec, *ops):
    """np.einsum with the pairwise BLAS path (the value is the plain sum)."""
    return np.einsum(spec, *ops, optimize=True)

from . import model

EIG_CUTOFF = 1e-14


def boundary_vector(dims):
    """Product boundary: the normalised all-ones vector on every layer leg."""
    v = np.ones(1)
    for n in dims:
        v = np.kron(v, np.ones(n) / np.sqrt(n))
    return v


def init_env(dims):
    """chi0 = 1 initial environment: C = [[1]], T[0, m, 0] = e(m)."""
    e = boundary_vector(dims)
    C = np.ones((1, 1))
    T = e.reshape(1, -1, 1).copy()
    return C, T


def enlarged_corner(C, T, a):
    """M[(b1, d), (b2, r)] = sum C[a1, a2] T[a1, m1, b1] T[a2, m2, b2] a[m1, m2, r, d].

    Corner C touches the left edge with leg a1 and the top edge with leg a2; the
    site's left leg meets the left edge, its up leg the top edge."""
    X = ein("xy,xmb->ymb", C, T)          # left edge attached
    X = ein("ymb,ync->mbnc", X, T)        # top edge attached
    M = ein("mbnc,mnrd->bdcr", X, a)
    chi, Df = T.shape[2], a.shape[3]
    return M.reshape(chi * Df, chi * Df)


def step(C, T, a, chi):
    """One C4v CTMRG step: grow the corner by one site and each edge by one column,
    then truncate with the eigenvectors of the symmetric enlarged corner."""
    M = enlarged_corner(C, T, a)
    M = 0.5 * (M + M.T)
    lam, V = np.linalg.eigh(M)
    order = np.lexsort((np.arange(lam.size), -np.abs(lam)))
    lam, V = lam[order], V[:, order]
    keep = int(np.sum(np.abs(lam) > EIG_CUTOFF * np.abs(lam[0])))
    keep = max(1, min(chi, keep))
    P = V[:, :keep]
    chi_old, Df = T.shape[0], a.shape[0]
    Cn = P.T @ M @ P
    Ten = ein("amb,murd->aurbd", T, a)     # edge absorbs one site column
    Ten = Ten.reshape(chi_old * Df, Df, chi_old * Df)
    Tn = ein("xa,xmy,yb->amb", P, Ten, P)
    Cn = 0.5 * (Cn + Cn.T)
    Tn = 0.5 * (Tn + Tn.transpose(2, 1, 0))
    Cn /= np.linalg.norm(Cn)
    Tn /= np.linalg.norm(Tn)
    return Cn, Tn


def corner_spectrum(C):
    """Singular values of rho_eff = C^4 / Tr C^4, descending (Sec. III D)."""
    ev = np.linalg.eigvalsh(0.5 * (C + C.T))
    s = np.sort(ev ** 4)[::-1]
    return s / np.sum(s)


def leading_pair_degenerate(C, rel=1e-4):
    """True when the two largest |eigenvalues| of the converged symmetric corner
    agree to rel: the network's transfer matrix then has a (near-)degenerate
    leading pair +-lambda, i.e. the network is period-2 ordered (a staggered
    fixed point that a one-site environment represents only as a mixture of
    the two ordered boundaries)."""
    ev = np.linalg.eigvalsh(0.5 * (C + C.T))
    ev = np.sort(np.abs(ev))[::-1]
    return ev.size > 1 and ev[0] - ev[1] <= rel * ev[0]


def spectrum_delta(s_new, s_old):
    n = max(s_new.size, s_old.size)
    a = np.zeros(n)
    b = np.zeros(n)
    a[: s_new.size] = s_new
    b[: s_old.size] = s_old
    return float(np.linalg.norm(a - b))


def run(a, dims, chi, max_iter, tol=0.0, min_iter=1):
    """Iterate from the product boundary; stop after max_iter steps or when the
    corner spectrum changes by less than tol (if tol > 0)."""
    C, T = init_env(dims)
    s_old = corner_spectrum(C)
    it, delta = 0, np.inf
    for it in range(1, max_iter + 1):
        C, T = step(C, T, a, chi)
        s = corner_spectrum(C)
        delta = spectrum_delta(s, s_old)
        s_old = s
        if tol > 0 and it >= min_iter and delta < tol:
            break
    return C, T, it, delta


def patch_values(C, T, a):
    """n1 (3x3 patch), n2 (3x2 strip), n0 (2x2 corners) for a C4v environment."""
    CTC = ein("xa,amb,by->xmy", C, T, C)             # corner-edge-corner row
    n2 = ein("xmy,xmy->", CTC, CTC)
    n0 = np.trace(C @ C @ C @ C)
    env = site_environment(C, T)
    n1 = ein("lurd,lurd->", env, a)
    return n1, n2, n0


def site_environment(C, T):
    """Environment of the centre site in the 3x3 patch: d n1 / d a[l,u,r,d]."""
    CTC = ein("xa,amb,by->xmy", C, T, C)             # top row (and bottom)
    # top row + left and right edges hanging down from its two corners
    X = ein("xuy,xlc->luyc", CTC, T)                  # left edge under C(tl)
    X = ein("luyc,yre->lurce", X, T)                  # right edge under C(tr)
    return ein("lurce,cde->lurd", X, CTC)             # bottom row closes


def magnetization(C, T, A, beta):
    """<sigma> at a site: the fused site tensor built with the impurity PEPO,
    over the one built with O, in the 3x3 patch of the converged triple-layer
    environment (C, T)."""
    env = site_environment(C, T)
    nz = ein("lurd,lurd->", env, model.fuse_triple(A, model.pepo_Oz(beta)))
    n1 = ein("lurd,lurd->", env, model.fuse_triple(A, model.pepo_O(beta)))
    return float(nz / n1)


def energy(C, T, A, beta):
    """Internal energy per site U = -n1(dO/dbeta) / n1(O): the fused site built
    with dO/dbeta over the one built with O, in the 3x3 patch of the converged
    triple-layer environment (C, T)."""
    env = site_environment(C, T)
    nd = ein("lurd,lurd->", env, model.fuse_triple(A, model.pepo_dO(beta)))
    n1 = ein("lurd,lurd->", env, model.fuse_triple(A, model.pepo_O(beta)))
    return float(-nd / n1)


def two_site_value(C, T, a1, a2):
    """The 3 x 4 patch: corners and edges around two horizontally adjacent sites
    a1 (left) and a2 (right), sharing the bond k (a1's right leg, a2's left leg):
      C[x,a] T[a,m,b] T[b,n,c] C[c,y]          (top row)
      T[x,l,p] a1[l,m,k,d] a2[k,n,r,e] T[y,r,q] (middle row)
      C[p,z] T[z,d,g] T[g,e,h] C[h,q]          (bottom row)
    summed as the left half L[b,k,g] times the right half R[b,k,g]."""
    L = ein("xa,amb->xmb", C, T)
    L = ein("xmb,xlp->mblp", L, T)
    L = ein("mblp,lmkd->bpkd", L, a1)
    L = ein("bpkd,pz->bkdz", L, C)
    L = ein("bkdz,zdg->bkg", L, T)
    R = ein("bnc,cy->bny", T, C)
    R = ein("bny,yrq->bnrq", R, T)
    R = ein("bnrq,knre->bkqe", R, a2)
    R = ein("bkqe,hq->bkeh", R, C)
    R = ein("bkeh,geh->bkg", R, T)
    return float(ein("bkg,bkg->", L, R))


def nn_correlation(C, T, a, az):
    """<s s'> of two horizontally adjacent spins carried by the site tensors:
    the two-site patch with both impurity tensors az over the one with a."""
    return two_site_value(C, T, az, az) / two_site_value(C, T, a, a)


def bond_correlation(C, T, A, beta):
    """In-plane nearest-neighbour <sigma sigma'> of the PEPO layer in the
    converged triple-layer environment (C, T)."""
    a = model.fuse_triple(A, model.pepo_O(beta))
    az = model.fuse_triple(A, model.pepo_Oz(beta))
    return nn_correlation(C, T, a, az)


def log_kappa(C, T, a):
    n1, n2, n0 = patch_values(C, T, a)
    kap = n1 * n0 / (n2 * n2)
    if not kap > 0:
        raise FloatingPointError("non-positive kappa estimate %r" % kap)
    return float(np.log(kap)), n1


def free_energy(beta, A, chi, max_iter, tol=0.0):
    """f(beta, A) by the reduced method; returns (f, info dict)."""
    O = model.pepo_O(beta)
    D = A.shape[1]
    a3 = model.fuse_triple(A, O)
    a2 = model.fuse_double(A)
    d = O.shape[2]
    C3, T3, it3, dl3 = run(a3, (D, d, D), chi, max_iter, tol)
    C2, T2, it2, dl2 = run(a2, (D, D), chi, max_iter, tol)
    lk3, n13 = log_kappa(C3, T3, a3)
    lk2, n12 = log_kappa(C2, T2, a2)
    f = -(lk3 - lk2) / beta
    info = dict(env3=(C3, T3), env2=(C2, T2), iters=(it3, it2), deltas=(dl3, dl2),
                log_kappa3=lk3, log_kappa2=lk2, spectrum3=corner_spectrum(C3))
    return f, info


def gradient(beta, A, info):
    """g = -(2/beta) (E3/n1_3 - E2/n1_2), D4-projected (gradient expression)."""
    O = model.pepo_O(beta)
    D = A.shape[1]
    d = O.shape[2]
    C3, T3 = info["env3"]
    C2, T2 = info["env2"]
    env3 = site_environment(C3, T3).reshape((D, d, D) * 4)
    env2 = site_environment(C2, T2).reshape((D, D) * 4)
    # legs of env3: (lk,li,lb, uk,ui,ub, rk,ri,rb, dk,di,db)
    X = ein("aeibfjcgkdhl,pabcd->peifjgkhl", env3, A)
    E3 = ein("peifjgkhl,pqefgh->qijkl", X, O)
    n13 = ein("qijkl,qijkl->", E3, A)
    E2 = ein("aibjckdl,pabcd->pijkl", env2, A)
    n12 = ein("qijkl,qijkl->", E2, A)
    g = -(2.0 / beta) * (E3 / n13 - E2 / n12)
    return model.d4_symmetrize(g)


def f_and_grad(beta, A, chi, max_iter, tol=0.0):
    f, info = free_energy(beta, A, chi, max_iter, tol)
    return f, gradient(beta, A, info), info
