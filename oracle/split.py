"""Split-CTMRG for the triple-layer network, written as plain einsum steps.

Test infrastructure only (FP64, CPU).  Follows Sec. III of the paper:
  * Sec. III A: split-CTM environment {C_i, T_i^ket, T_i^int, T_i^bra}; the norm
    network uses the same construction (here: the PEPO replaced by delta_{pq}
    with in-plane legs of size one, see model.identity_pepo).
  * Sec. III B: a move inserts one column of {T1, T3, A, O, conj(A)}, absorbs it
    row-wise into the edge and corner tensors, and truncates every new vertical
    bond with two projector pairs -- one for the bra-related legs (P1, P2, P3),
    then one for the ket-related legs (P4, P5, P6), with P_aT P_aB = I.
  * Eq. (Symmetry constraints): with the O_h-symmetric PEPO and D4-symmetric A
    the environment obeys D2 relations, so C1 (= C3), C4 (= C2) and the left
    edge chain T^ket, T^int, T^bra determine everything and a single set of
    projectors updates all directions; corners grow diagonally.
  * Sec. III C, Eqs. (projector construction, ... 2): rho_B rho_T = U S V,
    keep chi, P_B = rho_T V^+ (S^1/2)^+, P_T = (S^1/2)^+ U^+ rho_B.
  * Appendix, six-projector scheme: P2, P3 from a 1x1 unit cell with its full
    environment; P1 from a one-column, two-row strip; P4 from the enlarged
    corners with their bra legs pre-renormalised by P1: by default the half
    construction of the main text (the two left corners of a 2x1 block,
    Fig. Projector4(b), horizontal legs renormalised by the up / down images
    of P1), optionally the full one (2x2 block, Fig. Projector4(a): vertical
    legs renormalised by P1 and its right-move image P1^R = (P1B, P1T),
    horizontal legs whole); P5, P6 from a two-column, one-row block
    pre-renormalised by P2, P2^R (resp. P3, P3^R).  In the D2 scheme
    P2^R_T = P3_B, P2^R_B = P3_T, P3^R_T = P2_B, P3^R_B = P2_T, and the up / down
    images of P1 are its transposes.  The full P4's rho_B rho_T is a product
    of four enlarged corners: its spectrum decays as the square of the half
    one's, so the same relative cutoff truncates it to fewer directions (with
    1e-12 it reaches the reduced value on tensors where the half construction
    does not settle, e.g. the norm network of D = 3, seed 8 at chi = 27).
  * Sec. III C, environment selection: the rank of rho_B rho_T is bounded by
    the corner matrices of its patch.  During the growth phase (the corner
    bond still below chi after the product boundary) a rank-deficient
    rho_B rho_T would cut a bond below chi for want of environment, not of
    weight; such a pair is replaced by the orthogonal projector onto the
    leading eigenvectors of the truncated legs' Gram matrix (projector_pair).
  * Sec. III D: convergence from the singular values of
    rho_eff = C1 C2 C3 C4 / Tr(C1 C2 C3 C4).

Domain of this reading: networks whose transfer matrix has a unique leading
eigenvalue.  On period-2 ordered networks (a degenerate +-lambda leading
pair, oracle.unsplit.leading_pair_degenerate) a one-site environment can
only hold a mixture of the two ordered boundaries; the D2 split iteration
then has several fixed points and, from the product boundary, may settle on
one whose kappa is not the reduced method's.

The figures that fix the wiring are not part of the text; the wiring below is
one reading of them, stated here in full ("nested" placement of A, O, conj(A)
along the anti-diagonal of the unit cell).  In that placement the bonds of the
left edge chain carry, besides the environment bond chi,
    bk (T^bra -> next T^ket, also every corner leg):  A.d, O.d, B.d
    ki (T^ket -> T^int):                               A.d, p,  O.d', B.d'
    ib (T^int -> T^bra):                               A.d, O.d, q,   B.d'
(B = conj(A); primes mark the lines of the row above passing by).  Projector
trunc-slot orders: P1 (chi,B)  P2 (chi,O,B)  P3 (chi,B,q)  P4 (c,A,O)
P5 (c,A,p)  P6 (c,A,O).

Tensor conventions
  C1[x, y]   top-left corner;    x -> top edge, y -> left edge.   C3 = C1
  C4[x, y]   bottom-left corner; x -> left edge, y -> bottom edge. C2 = C4
  Tk, Ti, Tb [a, m, b]  left edge chain (a up, m into the bulk, b down)
  top edge    T1x = Tx                  (a left, m down, b right)
  right edge  T2x[a, m, b] = Tx'[b, m, a],  x' = bra/int/ket for x = ket/int/bra
  bottom edge T3x = T2x as arrays       (a left, m up, b right)
  A[p,l,u,r,d] ket, O[p,q,l,u,r,d], B[q,l,u,r,d] = A (real) bra.
"""
import numpy as np


def ein(spec, *ops):
    """np.einsum with the pairwise BLAS path (the value is the plain sum)."""
    return np.einsum(spec, *ops, optimize=True)

from . import model

SVD_CUTOFF = 1e-12
GROW_CHI = 1 << 30   # "no truncation" for the first move
LAST_STAGE2_ENVS = {}  # rho_T / rho_B of P5 and P6 from the last stage2 call


# ----------------------------------------------------------------------------
# environment state
# ----------------------------------------------------------------------------

def init_env(D, d):
    """Product boundary, chi0 = 1: every layer leg sees the normalised all-ones
    vector; corners are [[1]]."""
    return dict(
        C1=np.ones((1, 1)), C4=np.ones((1, 1)),
        Tk=np.ones((1, D, 1)) / np.sqrt(D),
        Ti=np.ones((1, d, 1)) / np.sqrt(d),
        Tb=np.ones((1, D, 1)) / np.sqrt(D),
    )


def right_edge(env):
    """(Rk, Ri, Rb): right and bottom edge tensors from the D2 relations."""
    return (env["Tb"].transpose(2, 1, 0), env["Ti"].transpose(2, 1, 0),
            env["Tk"].transpose(2, 1, 0))


# ----------------------------------------------------------------------------
# projector construction (Eqs. projector construction / ... 2)
# ----------------------------------------------------------------------------

def projector_pair(rhoB, rhoT, chi, cutoff=SVD_CUTOFF, fill=False):
    """rhoT: (trunc x remT) matrix, rhoB: (remB x trunc) matrix.
    Returns (PT [k x trunc], PB [trunc x k], kept singular values).

    A bond whose untruncated dimension does not exceed chi is not truncated:
    both projectors are the identity.  Otherwise rho_B rho_T = U S V, the
    chi leading triplets above the relative cutoff are kept and
    PB = rhoT V^T S^-1/2, PT = S^-1/2 U^T rhoB (Eqs. projector construction).

    fill (growth phase, Sec. III C environment-selection principle): the
    number of non-zero singular values of rho_B rho_T is bounded by the rank
    of the corner matrices of the patch.  While the environment's corner bond
    is still below chi (the first truncated moves after the product
    boundary), that bound reflects the small environment, not the network.
    If rho_B rho_T then has fewer than k = min(chi, trunc) singular values
    above the cutoff, the pair is the orthogonal projector onto the leading
    left singular vectors of Z = [rhoT / |rhoT|, rhoB^T / |rhoB|] (the
    eigenvectors of the truncated legs' Gram matrix
    G = rhoT rhoT^T / |rhoT|^2 + rhoB^T rhoB / |rhoB|^2): at most k of them,
    those whose singular value is above the same relative cutoff.  So no bond
    is cut below chi on the strength of a rank-deficient environment, and
    directions that neither half reaches are dropped.  Returned singular
    values are then empty."""
    ntr = rhoT.shape[0]
    if ntr <= chi:
        eye = np.eye(ntr)
        return eye, eye, np.zeros(0)
    M = rhoB @ rhoT
    U, S, Vh = np.linalg.svd(M, full_matrices=False)
    if S.size == 0 or S[0] <= 0:
        raise FloatingPointError("zero rho_B rho_T")
    keep = int(np.sum(S > cutoff * S[0]))
    k = min(chi, ntr)
    if fill and keep < k:
        Z = np.concatenate([rhoT / np.linalg.norm(rhoT), rhoB.T / np.linalg.norm(rhoB)], axis=1)
        Uz, sz, _ = np.linalg.svd(Z, full_matrices=False)
        kf = max(1, min(k, int(np.sum(sz > cutoff * sz[0]))))
        Q = Uz[:, :kf]
        return Q.T.copy(), Q.copy(), np.zeros(0)
    keep = max(1, min(chi, keep))
    sinv = 1.0 / np.sqrt(S[:keep])
    PB = (rhoT @ Vh[:keep].T) * sinv[None, :]
    PT = sinv[:, None] * (U[:, :keep].T @ rhoB)
    return PT, PB, S[:keep]


def _mat(X, nrow):
    shp = X.shape
    return X.reshape(int(np.prod(shp[:nrow])), int(np.prod(shp[nrow:])))


# ----------------------------------------------------------------------------
# the half-infinite pieces every construction is made of
# ----------------------------------------------------------------------------

def top_row(env):
    """C1 - T1(ket,int,bra) - C2.  Legs [y1 (down, left), Au, Ou, Bu, y2 (down, right)]."""
    C1, C4, Tk, Ti, Tb = env["C1"], env["C4"], env["Tk"], env["Ti"], env["Tb"]
    X = ein("xy,xas->yas", C1, Tk)
    X = ein("yas,sot->yaot", X, Ti)
    X = ein("yaot,tbu->yaobu", X, Tb)
    return ein("yaobu,uz->yaobz", X, C4)


def bottom_row(env):
    """C4 - T3(ket,int,bra) - C3.  Legs [x4 (up, left), Ad, Od, Bd, x3 (up, right)]."""
    Rk, Ri, Rb = right_edge(env)
    C1, C4 = env["C1"], env["C4"]
    X = ein("xy,yas->xas", C4, Rk)
    X = ein("xas,sot->xaot", X, Ri)
    X = ein("xaot,tbu->xaobu", X, Rb)
    return ein("xaobu,zu->xaobz", X, C1)


def upper_sequence(env, A, O):
    """Top row with the left/right edge cells and one site absorbed layer by layer.

    Returns the upper halves cut at ki (rho_T of P2), at ib (rho_T of P3) and at
    the next bk bond (rho_T of P1):
      up_ki [tkb, p, Ad, Ou, Bu, rkb]
      up_ib [tib, q, Od, Ad, Bu, rib]
      up_bk [tbb, Bd, Od, Ad, rbb]
    """
    Tk, Ti, Tb = env["Tk"], env["Ti"], env["Tb"]
    Rk, Ri, Rb = right_edge(env)
    X = top_row(env)                                            # y1 Au Ou Bu y2
    X = ein("yaobz,ylc->claobz", X, Tk)                   # c=Tk.b, l=Al
    X = ein("claobz,plarg->cpgrobz", X, A)                # g=Ad, r=Ar
    up_ki = ein("cpgrobz,zrh->cpgobh", X, Rk)             # [tkb,p,Ad,Ou,Bu,rkb]
    X = ein("cpgobh,cmj->jmpgobh", up_ki, Ti)             # j=Ti.b, m=Ol
    X = ein("jmpgobh,pqmost->jqtsgbh", X, O)              # s=Or, t=Od
    up_ib = ein("jqtsgbh,hsk->jqtgbk", X, Ri)             # [tib,q,Od,Ad,Bu,rib]
    X = ein("jqtgbk,jnw->wnqtgbk", up_ib, Tb)             # w=Tb.b, n=Bl
    X = ein("wnqtgbk,qnbve->wvetgk", X, B_of(A))          # v=Br, e=Bd
    up_bk = ein("wvetgk,kvz->wetgz", X, Rb)               # [tbb,Bd,Od,Ad,rbb]
    return up_ki, up_ib, up_bk


def lower_sequence(env, A, O):
    """Bottom row with the left/right edge cells and one site, bra layer first.

      lo_ib [tba, q, Bu, Ad, Od, rba]   (rho_B of P3)
      lo_ki [tia, p, Ou, Bu, Ad, ria]   (rho_B of P2)
      lo_bk [tka, Au, Ou, Bu, rka]      (rho_B of P1)
    """
    Tk, Ti, Tb = env["Tk"], env["Ti"], env["Tb"]
    Rk, Ri, Rb = right_edge(env)
    B = B_of(A)
    Y = bottom_row(env)                                         # x4 Ad Od Bd x3
    Y = ein("xaobz,cnx->cnaobz", Y, Tb)                   # c=Tb.a, n=Bl
    Y = ein("cnaobz,qnuvb->cquvaoz", Y, B)                # u=Bu, v=Br
    lo_ib = ein("cquvaoz,hvz->cquaoh", Y, Rb)             # [tba,q,Bu,Ad,Od,rba]
    Y = ein("cquaoh,jmc->jmquaoh", lo_ib, Ti)             # j=Ti.a, m=Ol
    Y = ein("jmquaoh,pqmsto->jpsutah", Y, O)              # s=Ou, t=Or
    lo_ki = ein("jpsutah,kth->jpsuak", Y, Ri)             # [tia,p,Ou,Bu,Ad,ria]
    Y = ein("jpsuak,ilj->ilpsuak", lo_ki, Tk)             # i=Tk.a, l=Al
    Y = ein("ilpsuak,plwra->iwrsuk", Y, A)                # w=Au, r=Ar
    lo_bk = ein("iwrsuk,zrk->iwsuz", Y, Rk)               # [tka,Au,Ou,Bu,rka]
    return lo_ki, lo_ib, lo_bk


def B_of(A):
    """Bra tensor: conj(A) = A for the real ansatz (Sec. III B)."""
    return A


# ----------------------------------------------------------------------------
# stage 1: P1, P2, P3
# ----------------------------------------------------------------------------

def stage1(env, A, O, chi, cutoff=SVD_CUTOFF, fill=False):
    up_ki, up_ib, up_bk = upper_sequence(env, A, O)
    lo_ki, lo_ib, lo_bk = lower_sequence(env, A, O)
    # P1: trunc (chi, B) ; rem (A, O, chiR)
    rT = _mat(up_bk.transpose(0, 1, 3, 2, 4), 2)                # (tbb,Bd) x (Ad,Od,rbb)
    rB = _mat(lo_bk.transpose(1, 2, 4, 0, 3), 3)                # (Au,Ou,rka) x (tka,Bu)
    P1 = projector_pair(rB, rT, chi, cutoff, fill)
    # P2: trunc (chi, O, B) ; rem (A, p, chiR)
    rT = _mat(up_ki.transpose(0, 3, 4, 2, 1, 5), 3)             # (tkb,Ou,Bu) x (Ad,p,rkb)
    rB = _mat(lo_ki.transpose(4, 1, 5, 0, 2, 3), 3)             # (Ad,p,ria) x (tia,Ou,Bu)
    P2 = projector_pair(rB, rT, chi, cutoff, fill)
    # P3: trunc (chi, B, q) ; rem (A, O, chiR)
    rT = _mat(up_ib.transpose(0, 4, 1, 3, 2, 5), 3)             # (tib,Bu,q) x (Ad,Od,rib)
    rB = _mat(lo_ib.transpose(3, 4, 5, 0, 2, 1), 3)             # (Ad,Od,rba) x (tba,Bu,q)
    P3 = projector_pair(rB, rT, chi, cutoff, fill)
    return P1, P2, P3


def bond_dims(env):
    """(chi_bk, chi_ki, chi_ib): the three bonds of the left edge chain."""
    return env["Tk"].shape[0], env["Tk"].shape[2], env["Ti"].shape[2]


def stage1_tensors(env, A, O, P1, P2, P3):
    """Stage-1 projector matrices reshaped to their trunc-slot legs."""
    D, d, P = A.shape[1], O.shape[2], A.shape[0]
    xbk, xki, xib = bond_dims(env)
    return (_as_tensor_T(P1[0], (xbk, D)), _as_tensor_B(P1[1], (xbk, D)),
            _as_tensor_T(P2[0], (xki, d, D)), _as_tensor_B(P2[1], (xki, d, D)),
            _as_tensor_T(P3[0], (xib, D, P)), _as_tensor_B(P3[1], (xib, D, P)))


def _as_tensor_T(PT, dims):
    """PT [k x trunc] -> [k, *dims]"""
    return PT.reshape((PT.shape[0],) + tuple(dims))


def _as_tensor_B(PB, dims):
    """PB [trunc x k] -> [*dims, k]"""
    return PB.reshape(tuple(dims) + (PB.shape[1],))


# ----------------------------------------------------------------------------
# enlarged corners (Fig. "D2 symmetric CTMRG": diagonal corner growth)
# ----------------------------------------------------------------------------

def enlarged_C1(env, A, O):
    """C1 + top cell + left cell + site.  [s3 (chi right), a3 (chi down), Ar, Ad, Or, Od, Br, Bd]"""
    C1, Tk, Ti, Tb = env["C1"], env["Tk"], env["Ti"], env["Tb"]
    B = B_of(A)
    X = ein("xy,xus,yla->usla", C1, Tk, Tk)               # top Tk and left Tk
    X = ein("usla,plurd->saprd", X, A)
    X = ein("saprd,sot->toaprd", X, Ti)                   # top Ti
    X = ein("toaprd,amc->tomcprd", X, Ti)                 # left Ti
    X = ein("tomcprd,pqmoef->tcqrdef", X, O)              # e=Or, f=Od
    X = ein("tcqrdef,tbu->ubcqrdef", X, Tb)               # top Tb
    X = ein("ubcqrdef,cnw->ubnwqrdef", X, Tb)             # left Tb
    return ein("ubnwqrdef,qnbvg->uwrdefvg", X, B)         # v=Br, g=Bd


def enlarged_C4(env, A, O):
    """C4 + left cell + bottom cell + site.  [a0 (chi up), s3 (chi right), Au, Ar, Ou, Or, Bu, Br]"""
    C4, Tk, Ti, Tb = env["C4"], env["Tk"], env["Ti"], env["Tb"]
    Rk, Ri, Rb = right_edge(env)
    B = B_of(A)
    X = ein("xy,cnx,yas->cnas", C4, Tb, Rk)               # left Tb, bottom T3k
    X = ein("cnas,jmc->jmnas", X, Ti)                     # left Ti
    X = ein("jmnas,sot->jmnaot", X, Ri)                   # bottom T3i
    X = ein("jmnaot,pqmhio->jnatpqhi", X, O)              # h=Ou, i=Or
    X = ein("jnatpqhi,klj->klnatpqhi", X, Tk)             # left Tk
    X = ein("klnatpqhi,plwra->knwrtqhi", X, A)            # w=Au, r=Ar
    X = ein("knwrtqhi,tbv->knwrbvqhi", X, Rb)             # bottom T3b
    return ein("knwrbvqhi,qnuyb->kvwrhiuy", X, B)         # u=Bu, y=Br


# ----------------------------------------------------------------------------
# stage 2: P4 (half), P5, P6
# ----------------------------------------------------------------------------

def stage2(env, A, O, chi, P1, P2, P3, cutoff=SVD_CUTOFF, fill=False, p4="half"):
    D, d, P = A.shape[1], O.shape[2], A.shape[0]
    Tk, Ti, Tb = env["Tk"], env["Ti"], env["Tb"]
    Rk, Ri, Rb = right_edge(env)
    C1, C4 = env["C1"], env["C4"]
    B = B_of(A)
    P1T, P1B, P2T, P2B, P3T, P3B = stage1_tensors(env, A, O, P1, P2, P3)

    # ---- half projector 4: enlarged corners with bra legs pre-renormalised
    K1 = enlarged_C1(env, A, O)                                 # s3 a3 Ar Ad Or Od Br Bd
    K1 = ein("uwrdefvg,cwg->ucrdefv", K1, P1T)            # down leg (a3,Bd) -> c
    C1p = ein("ucrdefv,Xuv->cdfXre", K1, P1T)             # right leg (s3,Br) -> X
    # C1p [c_d, Ad, Od, c_r, Ar, Or]
    K4 = enlarged_C4(env, A, O)                                 # a0 s3 Au Ar Ou Or Bu Br
    K4 = ein("kvwrhiuy,kuc->cvwrhiy", K4, P1B)            # up leg (a0,Bu) -> c
    C4p = ein("cvwrhiy,vrX->cwhXyi", K4, P1B)             # right (s3, Ar) -> X
    # C4p [c_u, Au, Ou, c_r', Br, Or]
    nT = C1p.shape[0] * D * d
    if p4 == "full":
        # full projector 4 (Appendix, Fig. Projector4(a)): the 2x2 block of
        # enlarged corners, vertical legs after P1 (left bond) and its
        # right-move image P1^R = (P1B, P1T) (right bond), horizontal legs whole.
        # K1 (P1T on the down leg): [u=chi right, c, r=Ar, d=Ad, e=Or, f=Od, v=Br]
        # K4 (P1B on the up leg):   [c, s=chi right, a=Au, r=Ar, h=Ou, o=Or, y=Br]
        # upper right corner: the diagonal-reflection image of the enlarged C4,
        # [a0 -> left chi, s3 -> down chi, Au, Ar, Ou, Or, Bu, Br -> A.l, A.d,
        # O.l, O.d, B.l, B.d], with P1^R_T = P1B on its down leg's (chi, A.d)
        C2e = ein("kvwrhiuy,vrX->kwhuXiy", enlarged_C4(env, A, O), P1B)   # [chi, Al, Ol, Bl, X, Od, Bd]
        rhoT4 = ein("ucrdefv,urevXiy->cdfXiy", K1, C2e)                 # [c, Ad, Od | X, Od2, Bd2]
        # lower right corner: the 180-degree image of the enlarged C1 with
        # P1^R_B = P1T on its up leg's (chi, A.u): the arrays of K1 with legs
        # [chi left, c', B.l, B.u, O.l, O.u, A.l]
        rhoB4 = ein("csarhoy,sCyBoOr->cahCBO", K4, K1)                  # [c, Au, Ou | C, Bu2, Ou2]
        n4 = rhoT4.shape[0] * rhoT4.shape[1] * rhoT4.shape[2]
        P4 = projector_pair(rhoB4.reshape(n4, -1).T, rhoT4.reshape(n4, -1), chi, cutoff, fill)
    else:
        rT = C1p.reshape(nT, -1)                                # (c_d,Ad,Od) x (c_r,Ar,Or)
        rB = C4p.reshape(nT, -1).T                              # (c_r',Br,Or) x (c_u,Au,Ou)
        P4 = projector_pair(rB, rT, chi, cutoff, fill)

    # ---- P5 (ki bond, stage 2): two-column block cut at ki
    X = ein("xy,xus,sot,tbw->yuobw", C1, Tk, Ti, Tb)      # C1 + top cell 1
    X = ein("yuobw,ylc->uobwlc", X, Tk)                   # left Tk
    UL = ein("uobwlc,plurg->wobcpgr", X, A)               # [s3,Ou1,Bu1,tkb,p1,Ad1,Ar1]
    UL = ein("wobcpgr,ecob->wepgr", UL, P2T)              # -> [s3,c2L,p1,Ad1,Ar1]
    X = ein("wus,sot,tbv,vz->wuobz", Tk, Ti, Tb, C4)      # top cell 2 + C2 (= C4)
    X = ein("wuobz,zrh->wuobrh", X, Rk)                   # right Tk'
    UR = ein("wuobrh,plurg->wlgpobh", X, A)               # [s3,Al2,Ad2,p2,Ou2,Bu2,rkb]
    # P2^R_T[c,(chi,a,p)] = P3B[(chi,a,p),c]
    UR = ein("wlgpobh,hgpe->wlobe", UR, P3B)              # [s3,Al2,Ou2,Bu2,c2R]
    rhoT5 = ein("wepgr,wrobf->egpobf", UL, UR)            # [c2L,Ad1,p1,Ou2,Bu2,c2R]

    Y = ein("xy,yas,sot,tbv->xaobv", C4, Rk, Ri, Rb)      # C4 + bottom cell 1
    Y = ein("xaobv,cnx->cnaobv", Y, Tb)                   # left Tb
    Y = ein("cnaobv,qnuyb->cquyaov", Y, B)                # u=Bu1, y=Br1
    Y = ein("cquyaov,jmc->jmquyaov", Y, Ti)               # left Ti
    LL = ein("jmquyaov,pqmsto->jpsutyav", Y, O)           # [tia,p1,Ou1,Bu1,Or1,Br1,Ad1,v3]
    LL = ein("jpsutyav,jsue->epatyv", LL, P2B)            # [c2L,p1,Ad1,Or1,Br1,v3]
    Y = ein("zy,vas,sot,tby->zvaob", C1, Rk, Ri, Rb)      # C3 (= C1) + bottom cell 2
    Y = ein("zvaob,kyz->kyvaob", Y, Rb)                   # right Tb'
    Y = ein("kyvaob,qnuyb->kqnuvao", Y, B)                # n=Bl2, u=Bu2
    Y = ein("kqnuvao,hik->hiqnuvao", Y, Ri)               # right Ti'
    LR = ein("hiqnuvao,pqmsio->hpmsnuva", Y, O)           # [ria,p2,Ol2,Ou2,Bl2,Bu2,v3,Ad2]
    # P2^R_B[(chi,a,p),c] = P3T[c,(chi,a,p)]
    LR = ein("hpmsnuva,ehap->emsnuv", LR, P3T)            # [c2R,Ol2,Ou2,Bl2,Bu2,v3]
    rhoB5 = ein("epatyv,ftsyuv->eapsuf", LL, LR)          # [c2L,Ad1,p1,Ou2,Bu2,c2R]
    n5 = rhoT5.shape[0] * D * P
    P5 = projector_pair(rhoB5.reshape(n5, -1).T, rhoT5.reshape(n5, -1), chi, cutoff, fill)

    # ---- P6 (ib bond, stage 2): same block cut at ib
    X = ein("xy,xus,sot,tbw->yuobw", C1, Tk, Ti, Tb)
    X = ein("yuobw,ylc->uobwlc", X, Tk)
    X = ein("uobwlc,plurg->wobcpgr", X, A)                # [s3,Ou1,Bu1,tkb,p1,Ad1,Ar1]
    X = ein("wobcpgr,cmj->wobjpgrm", X, Ti)               # left Ti
    UL6 = ein("wobjpgrm,pqmoef->wbjqgref", X, O)          # [s3,Bu1,tib,q1,Ad1,Ar1,Or1,Od1]
    UL6 = ein("wbjqgref,cjbq->wcgref", UL6, P3T)          # [s3,c3L,Ad1,Ar1,Or1,Od1]
    X = ein("wus,sot,tbv,vz->wuobz", Tk, Ti, Tb, C4)
    X = ein("wuobz,zrh->wuobrh", X, Rk)
    X = ein("wuobrh,plurg->wlgpobh", X, A)                # [s3,Al2,Ad2,p2,Ou2,Bu2,rkb]
    X = ein("wlgpobh,hsk->wlgpobsk", X, Ri)               # right Ti', s=Or2
    UR6 = ein("wlgpobsk,pqmost->wlgbkqmt", X, O)          # [s3,Al2,Ad2,Bu2,rib,q2,Ol2,Od2]
    # P3^R_T[c,(chi,o,a)] = P2B[(chi,o,a),c]
    UR6 = ein("wlgbkqmt,ktge->wlbqme", UR6, P2B)          # [s3,Al2,Bu2,q2,Ol2,c3R]
    rhoT6 = ein("wcgref,wrbqeh->cgfbqh", UL6, UR6)        # [c3L,Ad1,Od1,Bu2,q2,c3R]

    Y = ein("xy,yas,sot,tbv->xaobv", C4, Rk, Ri, Rb)
    Y = ein("xaobv,cnx->cnaobv", Y, Tb)
    LL6 = ein("cnaobv,qnuyb->cquyaov", Y, B)              # [tba,q1,Bu1,Br1,Ad1,Od1,v3]
    LL6 = ein("cquyaov,cuqe->eyaov", LL6, P3B)            # [c3L,Br1,Ad1,Od1,v3]
    Y = ein("zy,vas,sot,tby->zvaob", C1, Rk, Ri, Rb)
    Y = ein("zvaob,kyz->kyvaob", Y, Rb)
    LR6 = ein("kyvaob,qnuyb->kqnuvao", Y, B)              # [rba,q2,Bl2,Bu2,v3,Ad2,Od2]
    # P3^R_B[(chi,o,a),c] = P2T[c,(chi,o,a)]
    LR6 = ein("kqnuvao,ekoa->eqnuv", LR6, P2T)            # [c3R,q2,Bl2,Bu2,v3]
    rhoB6 = ein("eyaov,fqyuv->eaouqf", LL6, LR6)          # [c3L,Ad1,Od1,Bu2,q2,c3R]
    n6 = rhoT6.shape[0] * D * d
    P6 = projector_pair(rhoB6.reshape(n6, -1).T, rhoT6.reshape(n6, -1), chi, cutoff, fill)
    LAST_STAGE2_ENVS.clear()
    LAST_STAGE2_ENVS.update(rhoT5=rhoT5, rhoB5=rhoB5, rhoT6=rhoT6, rhoB6=rhoB6)
    return P4, P5, P6, C1p, C4p


# ----------------------------------------------------------------------------
# one symmetric split-CTMRG step
# ----------------------------------------------------------------------------

def growing(env, chi):
    """Growth phase: the corner bond has not yet reached chi since the
    product boundary (the environment-selection principle of Sec. III C
    cannot hold yet)."""
    return (not env.get("grown", False)) and env["C1"].shape[0] < chi


def step(env, A, O, chi, cutoff=SVD_CUTOFF, p4="half"):
    """One symmetric split-CTMRG move.  p4: "half" (the main-text choice,
    Fig. Projector4(b)) or "full" (Fig. Projector4(a))."""
    D, d, P = A.shape[1], O.shape[2], A.shape[0]
    B = B_of(A)
    fill = growing(env, chi)
    P1, P2, P3 = stage1(env, A, O, chi, cutoff, fill)
    P4, P5, P6, C1p, C4p = stage2(env, A, O, chi, P1, P2, P3, cutoff, fill, p4)
    c1, c2, c3 = P1[0].shape[0], P2[0].shape[0], P3[0].shape[0]
    P1T, P1B, P2T, P2B, P3T, P3B = stage1_tensors(env, A, O, P1, P2, P3)
    P4T = _as_tensor_T(P4[0], (c1, D, d))
    P4B = _as_tensor_B(P4[1], (c1, D, d))
    P5T = _as_tensor_T(P5[0], (c2, D, P))
    P5B = _as_tensor_B(P5[1], (c2, D, P))
    P6T = _as_tensor_T(P6[0], (c3, D, d))
    P6B = _as_tensor_B(P6[1], (c3, D, d))
    # combined two-stage projectors on each bond of the left edge
    PbkT = ein("nxao,xcb->ncaob", P4T, P1T)        # [n, chi, A, O, B]
    PbkB = ein("cbx,xaon->caobn", P1B, P4B)        # [chi, A, O, B, n]
    PkiT = ein("nxap,xcob->ncapob", P5T, P2T)      # [n, chi, A, p, O, B]
    PkiB = ein("cobx,xapn->capobn", P2B, P5B)      # [chi, A, p, O, B, n]
    PibT = ein("nxao,xcbq->ncaoqb", P6T, P3T)      # [n, chi, A, O, q, B]
    PibB = ein("cbqx,xaon->caoqbn", P3B, P6B)      # [chi, A, O, q, B, n]
    Tk, Ti, Tb = env["Tk"], env["Ti"], env["Tb"]
    # edge renormalisation (row-wise absorption, then the projectors of the
    # bond above (P_B side) and of the bond below (P_T side))
    X = ein("cuosn,clb->nuoslb", PbkB, Tk)
    X = ein("nuoslb,plumd->nosbpmd", X, A)
    Tk_n = ein("nosbpmd,kbdpos->nmk", X, PkiT)
    X = ein("capusn,clb->napuslb", PkiB, Ti)
    X = ein("napuslb,pqlumt->nasbmtq", X, O)
    Ti_n = ein("nasbmtq,kbatqs->nmk", X, PibT)
    X = ein("caoqun,clb->naoqulb", PibB, Tb)
    X = ein("naoqulb,qlumt->naobmt", X, B)
    Tb_n = ein("naobmt,kbaot->nmk", X, PbkT)
    # corners: second-stage projectors on the stage-1 renormalised enlarged corners
    C1_n = ein("Xqre,cdfqre->cdfX", P4T, C1p)           # right leg -> X
    C1_n = ein("cdfX,Ycdf->XY", C1_n, P4T)              # down leg -> Y
    C4_n = ein("cwhXyi,cwhx->xXyi", C4p, P4B)           # up leg -> x
    C4_n = ein("xXyi,Xyiz->xz", C4_n, P4B)              # right leg -> z
    C1_n = 0.5 * (C1_n + C1_n.T)
    C4_n = 0.5 * (C4_n + C4_n.T)
    new = dict(C1=C1_n, C4=C4_n, Tk=Tk_n, Ti=Ti_n, Tb=Tb_n)
    for k in new:
        new[k] = new[k] / np.linalg.norm(new[k])
    new["grown"] = bool(env.get("grown", False) or C1_n.shape[0] >= chi)
    projs = dict(P1=P1, P2=P2, P3=P3, P4=P4, P5=P5, P6=P6)
    return new, projs


# ----------------------------------------------------------------------------
# convergence, values, gradient
# ----------------------------------------------------------------------------

def rho_eff(env):
    C1, C4 = env["C1"], env["C4"]
    return C1 @ C4 @ C1 @ C4


def corner_spectrum(env):
    """Singular values of rho_eff = C1 C2 C3 C4 / Tr(C1 C2 C3 C4) (Sec. III D)."""
    r = rho_eff(env)
    s = np.linalg.svd(r, compute_uv=False)
    return s / abs(np.trace(r))


def spectrum_delta(s_new, s_old):
    n = max(s_new.size, s_old.size)
    a = np.zeros(n)
    b = np.zeros(n)
    a[: s_new.size] = s_new
    b[: s_old.size] = s_old
    return float(np.linalg.norm(a - b))


def run(A, O, chi, max_iter, tol=0.0, cutoff=SVD_CUTOFF, env=None, p4="half"):
    D, d = A.shape[1], O.shape[2]
    if env is None:
        env = init_env(D, d)
    s_old = corner_spectrum(env)
    it, delta = 0, np.inf
    history = []
    for it in range(1, max_iter + 1):
        # the first move from the product boundary never truncates: its
        # projector environments would see the boundary vectors only and would
        # cap the rank of every bond that carries lines of the row above
        env, _ = step(env, A, O, chi if it > 1 else GROW_CHI, cutoff, p4)
        s = corner_spectrum(env)
        delta = spectrum_delta(s, s_old)
        history.append(delta)
        s_old = s
        if tol > 0 and delta < tol:
            break
    return env, it, delta, history


def patch_values(env, A, O):
    """n1 (3x3), n2h (3 wide x 2 high), n2v (2 wide x 3 high), n0 (corners)."""
    Tk, Ti, Tb = env["Tk"], env["Ti"], env["Tb"]
    Rk, Ri, Rb = right_edge(env)
    C1, C4 = env["C1"], env["C4"]
    top = top_row(env)
    bot = bottom_row(env)
    _, _, up_bk = upper_sequence(env, A, O)                     # [tbb,Bd,Od,Ad,rbb]
    n1 = ein("wetgz,wgtez->", up_bk, bot)
    n2h = ein("yaobz,yaobz->", top, bot)
    # vertical strip: C1 C2 / left chain . right chain / C4 C3
    X = ein("xy,xz->yz", C1, C4)                          # C1 - C2 (top)
    X = ein("yz,yma,zmb->ab", X, Tk, Rk)
    X = ein("ab,amc,bmd->cd", X, Ti, Ri)
    X = ein("cd,cme,dmf->ef", X, Tb, Rb)
    # bottom: C4[e, g] (x = up) and C3 = C1[f, h] (x = up), joined by g - h
    n2v = ein("ef,eg,fg->", X, C4, C1)
    n0 = np.trace(rho_eff(env))
    return n1, n2h, n2v, n0


def log_kappa(env, A, O):
    n1, n2h, n2v, n0 = patch_values(env, A, O)
    kap = n1 * n0 / (n2h * n2v)
    if not kap > 0:
        raise FloatingPointError("non-positive kappa estimate %r" % kap)
    return float(np.log(kap)), n1


def magnetization(env, A, beta):
    """<sigma> at a site of the PEPO layer: the 3x3 patch with the impurity
    PEPO at its centre over the same patch with O, both in the converged
    triple-layer environment env."""
    bot = bottom_row(env)
    vals = []
    for O in (model.pepo_Oz(beta), model.pepo_O(beta)):
        _, _, up_bk = upper_sequence(env, A, O)
        vals.append(ein("wetgz,wgtez->", up_bk, bot))
    return float(vals[0] / vals[1])


def energy(env, A, beta):
    """Internal energy per site U = -n1(dO/dbeta) / n1(O) in the converged
    triple-layer environment env: minus the beta derivative of ln kappa3 at
    fixed A and environment, which at the optimum of A (f stationary in A) is
    d(beta f)/d beta (Sec. IV B)."""
    bot = bottom_row(env)
    vals = []
    for O in (model.pepo_dO(beta), model.pepo_O(beta)):
        _, _, up_bk = upper_sequence(env, A, O)
        vals.append(ein("wetgz,wgtez->", up_bk, bot))
    return float(-vals[0] / vals[1])


def two_site_value(env, A, O1, O2):
    """The 3 x 4 patch around two horizontally adjacent sites with the PEPOs O1
    (left) and O2 (right): the two-column top row, then the ket, PEPO and bra
    layers of both sites absorbed layer by layer between the left edge chain
    and its D2 image on the right, closed by the two-column bottom row."""
    C1, C4, Tk, Ti, Tb = env["C1"], env["C4"], env["Tk"], env["Ti"], env["Tb"]
    Rk, Ri, Rb = right_edge(env)
    B = B_of(A)
    # top row C1 - (Tk Ti Tb) - (Tk Ti Tb) - C2: [y, a o b (site 1 up), c p d (site 2 up), z]
    X = ein("xy,xas->yas", C1, Tk)
    X = ein("yas,sot->yaot", X, Ti)
    X = ein("yaot,tbu->yaobu", X, Tb)
    X = ein("yaobu,ucv->yaobcv", X, Tk)
    X = ein("yaobcv,vpw->yaobcpw", X, Ti)
    X = ein("yaobcpw,wdz->yaobcpdz", X, Tb)
    X = ein("yaobcpdz,zq->yaobcpdq", X, C4)
    # ket layer: left edge, A (site 1), A (site 2), right edge
    X = ein("yaobcpdz,ylg->glaobcpdz", X, Tk)
    X = ein("glaobcpdz,slare->gserobcpdz", X, A)
    X = ein("gserobcpdz,trcvf->gseobtfvpdz", X, A)
    X = ein("gseobtfvpdz,zvh->gseobtfpdh", X, Rk)
    # PEPO layer
    X = ein("gseobtfpdh,gmj->jmseobtfpdh", X, Ti)
    X = ein("jmseobtfpdh,sqmonk->jqknebtfpdh", X, O1)
    X = ein("jqknebtfpdh,twnpxu->jqkebwuxfdh", X, O2)
    X = ein("jqkebwuxfdh,hxi->jqkebwufdi", X, Ri)
    # bra layer
    X = ein("jqkebwufdi,jLJ->JLqkebwufdi", X, Tb)
    X = ein("JLqkebwufdi,qLbRE->JERkewufdi", X, B)
    X = ein("JERkewufdi,wRdVF->JEkeFVufi", X, B)
    up2 = ein("JEkeFVufi,iVH->JEkeFufH", X, Rb)               # [tbb, Bd1, Od1, Ad1, Bd2, Od2, Ad2, rbb]
    # bottom row C4 - (Rk Ri Rb) - (Rk Ri Rb) - C3: [x4, Ad1 Od1 Bd1, Ad2 Od2 Bd2, x3]
    Y = ein("xy,yas->xas", C4, Rk)
    Y = ein("xas,sot->xaot", Y, Ri)
    Y = ein("xaot,tbu->xaobu", Y, Rb)
    Y = ein("xaobu,ucv->xaobcv", Y, Rk)
    Y = ein("xaobcv,vpw->xaobcpw", Y, Ri)
    Y = ein("xaobcpw,wdz->xaobcpdz", Y, Rb)
    bot2 = ein("xaobcpdz,qz->xaobcpdq", Y, C1)
    return float(ein("JEkeFufH,JekEfuFH->", up2, bot2))


def bond_correlation(env, A, beta):
    """In-plane nearest-neighbour <sigma sigma'> of the PEPO layer: the two-site
    patch with both impurity PEPOs over the one with O, in the converged
    triple-layer environment."""
    O, Oz = model.pepo_O(beta), model.pepo_Oz(beta)
    return two_site_value(env, A, Oz, Oz) / two_site_value(env, A, O, O)


def bra_environment(env, A, O):
    """d n1 / d B[q, l, u, r, d]: the 3x3 patch with the bra tensor removed."""
    _, up_ib, _ = upper_sequence(env, A, O)                     # [tib,q,Od,Ad,Bu,rib]
    Tb = env["Tb"]
    _, _, Rb = right_edge(env)
    bot = bottom_row(env)                                       # [x4,Ad,Od,Bd,x3]
    X = ein("jqtgbk,jnw->qtgbnwk", up_ib, Tb)
    X = ein("qtgbnwk,kvz->qtgbnwvz", X, Rb)
    return ein("qtgbnwvz,wgtez->qnbve", X, bot)


def free_energy(beta, A, chi, max_iter, tol=0.0, cutoff=SVD_CUTOFF, p4="half"):
    O3 = model.pepo_O(beta)
    O2 = model.identity_pepo()
    env3, it3, dl3, h3 = run(A, O3, chi, max_iter, tol, cutoff, p4=p4)
    env2, it2, dl2, h2 = run(A, O2, chi, max_iter, tol, cutoff, p4=p4)
    lk3, _ = log_kappa(env3, A, O3)
    lk2, _ = log_kappa(env2, A, O2)
    f = -(lk3 - lk2) / beta
    info = dict(env3=env3, env2=env2, iters=(it3, it2), deltas=(dl3, dl2),
                log_kappa3=lk3, log_kappa2=lk2, spectrum3=corner_spectrum(env3),
                spectrum2=corner_spectrum(env2), history3=h3, history2=h2)
    return f, info


def gradient(beta, A, info):
    O3 = model.pepo_O(beta)
    O2 = model.identity_pepo()
    E3 = bra_environment(info["env3"], A, O3)
    E2 = bra_environment(info["env2"], A, O2)
    n13 = ein("qlurd,qlurd->", E3, A)
    n12 = ein("qlurd,qlurd->", E2, A)
    g = -(2.0 / beta) * (E3 / n13 - E2 / n12)
    return model.d4_symmetrize(g)


def f_and_grad(beta, A, chi, max_iter, tol=0.0, cutoff=SVD_CUTOFF, p4="half"):
    f, info = free_energy(beta, A, chi, max_iter, tol, cutoff, p4)
    return f, gradient(beta, A, info), info
