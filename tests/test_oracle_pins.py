"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Each test names the fact it checks.  Together they are chosen so that a
plausible slip in the oracle (a dropped factor in O, a wrong D4 permutation, a
transposed edge tensor, a mis-wired projector, a wrong gradient normalisation)
fails at least one of them.
"""
import itertools
import warnings

import numpy as np
import pytest

from oracle import exact, model, split, unsplit
from synth_inputs import raw_peps, random_directions

warnings.simplefilter("ignore")


# ---------------------------------------------------------------- model pieces

@pytest.mark.parametrize("beta", [0.05, 0.2, 0.7])
def test_sqrtW_squares_to_W(beta):
    s = model.sqrt_W(beta)
    assert np.allclose(s @ s, model.boltzmann_W(beta), rtol=1e-14, atol=0)
    # eigenvalues 2cosh(b), 2sinh(b) with eigenvectors (1,1), (1,-1)
    assert np.isclose(s.sum(axis=1)[0] ** 2, 2 * np.cosh(beta), rtol=1e-14)


@pytest.mark.parametrize("beta", [0.1, 0.22, 0.4])
def test_pepo_single_site_torus(beta):
    """A 1x1x1 periodic cube: the six legs of one O traced pairwise give
    Z = sum_s W[s,s]^3 = 2 e^{3 beta}."""
    O = model.pepo_O(beta)
    Z = np.einsum("ppllkk->", O.transpose(0, 1, 2, 4, 3, 5))
    assert np.isclose(Z, 2 * np.exp(3 * beta), rtol=1e-13)


def test_pepo_fully_symmetric():
    """O_h symmetry of the PEPO (Sec. IV): invariant under any leg permutation."""
    O = model.pepo_O(0.3)
    for perm in [(1, 0, 2, 3, 4, 5), (0, 1, 3, 2, 4, 5), (5, 4, 3, 2, 1, 0), (2, 3, 4, 5, 0, 1)]:
        assert np.allclose(O.transpose(perm), O, rtol=0, atol=1e-15)


@pytest.mark.parametrize("beta", [0.1, 0.25])
def test_pepo_two_site_torus(beta):
    """Two sites stacked along z with periods (1, 1, 2): each site has one x link
    and one y link to itself and the two sites share two z links, so
    Z = sum_{s0,s1} W[s0,s0]^2 W[s1,s1]^2 W[s0,s1]^2 = e^{4b} (2 e^{2b} + 2 e^{-2b})."""
    O = model.pepo_O(beta)
    Z = np.einsum("pqlulu,qpmvmv->", O, O)
    assert np.isclose(Z, np.exp(4 * beta) * (2 * np.exp(2 * beta) + 2 * np.exp(-2 * beta)), rtol=1e-13)


# ------------------------------------------------------------------- D4 ansatz

@pytest.mark.parametrize("D", [2, 3, 4])
def test_d4_projection_rank_and_idempotence(D):
    """Burnside: the D4-invariant subspace of C^2 (x) (C^D)^(x4) under leg
    permutations has dimension 2 (D^4 + 2 D^3 + 3 D^2 + 2 D) / 8."""
    n = 2 * D ** 4
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = model.d4_symmetrize(e.reshape(2, D, D, D, D)).ravel()
    assert np.allclose(M @ M, M, atol=1e-14)
    assert np.allclose(M, M.T, atol=1e-14)
    rank = int(round(np.trace(M)))
    assert rank == 2 * (D ** 4 + 2 * D ** 3 + 3 * D ** 2 + 2 * D) // 8


def test_d4_symmetric_tensor_invariant_under_every_group_element():
    A = model.d4_symmetrize(raw_peps(3, 5))
    # generators of D4 acting on (l,u,r,d): quarter turn and one reflection
    rot = A.transpose(0, 2, 3, 4, 1)
    ref = A.transpose(0, 3, 2, 1, 4)
    assert np.allclose(rot, A, atol=1e-15) and np.allclose(ref, A, atol=1e-15)


# -------------------------------------------------------------- Onsager (2D)

@pytest.mark.parametrize("beta", [0.18, 0.2, 0.26])
def test_onsager_two_forms_agree(beta):
    assert abs(exact.onsager_log_kappa(beta) - exact.onsager_log_kappa_double(beta)) < 1e-12


@pytest.mark.parametrize("beta", [0.18, 0.2, 0.26])
def test_ctm_core_reproduces_onsager(beta):
    a = model.ising_2d_site(beta)
    C, T, it, dl = unsplit.run(a, (2,), 32, 400, tol=1e-14)
    lk, _ = unsplit.log_kappa(C, T, a)
    assert abs(lk - exact.onsager_log_kappa(beta)) < 1e-12


@pytest.mark.parametrize("beta", [0.2, 0.3, 0.6])
def test_onsager_nn_correlation_is_the_energy_derivative(beta):
    """<s s'> = (1/2) d ln kappa_2D / d beta (two bonds per site): the elliptic
    closed form against central differences of the quadrature form."""
    h = 1e-5
    fd = (exact.onsager_log_kappa(beta + h) - exact.onsager_log_kappa(beta - h)) / (4 * h)
    assert abs(exact.onsager_nn_correlation(beta) - fd) < 1e-8


@pytest.mark.parametrize("beta", [0.2, 0.3])
def test_ctm_core_reproduces_onsager_nn_correlation(beta):
    """The two-site impurity patch in the converged 2D environment gives the
    exact nearest-neighbour correlation."""
    a, az = model.ising_2d_site(beta), model.ising_2d_site_z(beta)
    C, T, _, _ = unsplit.run(a, (2,), 32, 400, tol=1e-14)
    assert abs(unsplit.nn_correlation(C, T, a, az) - exact.onsager_nn_correlation(beta)) < 1e-11


def test_product_state_bond_correlation_is_the_2d_one():
    """For A = (1, 1)/sqrt(2) the triple-layer network is cosh(beta) times the 2D
    Ising network per site, with or without the impurity PEPOs, so the in-plane
    <sigma sigma'> is the 2D nearest-neighbour correlation."""
    beta = 0.2
    A = model.embed_product_state(2, +1)
    O = model.pepo_O(beta)
    C, T, _, _ = unsplit.run(model.fuse_triple(A, O), (2, 2, 2), 24, 400, tol=1e-14)
    assert abs(unsplit.bond_correlation(C, T, A, beta) - exact.onsager_nn_correlation(beta)) < 1e-11


@pytest.mark.parametrize("beta", [0.05, 0.2, 0.7])
def test_pepo_beta_derivative_is_the_finite_difference(beta):
    """d sqrt(W)/d beta (closed form in the eigenbasis of W) against central
    differences of the eigh-based sqrt(W), and dO/d beta (product rule over the
    six legs) against central differences of O."""
    h = 1e-6
    fd = (model.sqrt_W(beta + h) - model.sqrt_W(beta - h)) / (2 * h)
    assert np.max(np.abs(model.sqrt_W_dbeta(beta) - fd)) < 1e-8
    fdO = (model.pepo_O(beta + h) - model.pepo_O(beta - h)) / (2 * h)
    assert np.max(np.abs(model.pepo_dO(beta) - fdO)) < 1e-8 * max(1.0, np.max(np.abs(fdO)))


@pytest.mark.parametrize("sign", [+1, -1])
@pytest.mark.parametrize("beta", [0.2, 0.3])
def test_product_state_energy_is_the_beta_derivative(sign, beta):
    """The closed-form U of the product states against central differences of
    beta f(beta), whose 2D part is the quadrature form of ln kappa_2D."""
    h = 1e-5
    bf = lambda b: b * exact.product_state_f(b, sign)
    fd = (bf(beta + h) - bf(beta - h)) / (2 * h)
    assert abs(exact.product_state_energy(beta, sign) - fd) < 1e-8


@pytest.mark.parametrize("sign", [+1, -1])
def test_unsplit_product_state_energy_is_the_closed_form(sign):
    """For A = (1, +-1)/sqrt(2) the energy impurity gives the 2D Ising energy
    plus the link to the free neighbouring layer."""
    beta = 0.2
    A = model.embed_product_state(2, sign)
    O = model.pepo_O(beta)
    C, T, _, _ = unsplit.run(model.fuse_triple(A, O), (2, 2, 2), 24, 400, tol=1e-14)
    assert abs(unsplit.energy(C, T, A, beta) - exact.product_state_energy(beta, sign)) < 1e-10


def test_energy_is_the_beta_derivative_at_fixed_A():
    """U = -d ln kappa3 / d beta at fixed A: the impurity value in the converged
    environment against central differences of the re-converged reduced-method
    ln kappa3 (beta f = -(ln kappa3 - ln kappa2); kappa2 does not depend on
    beta).  A random D = 2 tensor, chi = 16."""
    beta, chi, h = 0.2, 16, 1e-5
    A = model.d4_symmetrize(raw_peps(2, 0))
    D = A.shape[1]

    def env_and_lk3(b):
        a3 = model.fuse_triple(A, model.pepo_O(b))
        C, T, _, _ = unsplit.run(a3, (D, 2, D), chi, 400, tol=1e-13)
        return C, T, unsplit.log_kappa(C, T, a3)[0]

    C, T, _ = env_and_lk3(beta)
    U = unsplit.energy(C, T, A, beta)
    fd = -(env_and_lk3(beta + h)[2] - env_and_lk3(beta - h)[2]) / (2 * h)
    assert abs(U - fd) < 1e-6 * abs(U), (U, fd)


def test_split_energy_is_the_beta_derivative_at_fixed_A():
    """The same fact for the split environment (D = 2, chi = 16)."""
    beta, chi, h = 0.2, 16, 1e-5
    A = model.d4_symmetrize(raw_peps(2, 0))

    def env_and_lk3(b):
        O = model.pepo_O(b)
        env, _, _, _ = split.run(A, O, chi, 300, tol=1e-13)
        return env, split.log_kappa(env, A, O)[0]

    env, _ = env_and_lk3(beta)
    U = split.energy(env, A, beta)
    fd = -(env_and_lk3(beta + h)[1] - env_and_lk3(beta - h)[1]) / (2 * h)
    assert abs(U - fd) < 1e-6 * abs(U), (U, fd)


# ------------------------------------------------------ reduced (unsplit) CTM

@pytest.mark.parametrize("n", [1, 2])
def test_magnetization_untruncated_split_equals_unsplit(n):
    """The impurity contraction of the split patch and of the fused-site patch
    are independent codes for the same finite network when nothing is
    truncated: the two magnetisations agree."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 1))
    O = model.pepo_O(beta)
    env, _, _, _ = split.run(A, O, 10 ** 9, n)
    C, T, _, _ = unsplit.run(model.fuse_triple(A, O), (2, 2, 2), 10 ** 9, n)
    ms, mu = split.magnetization(env, A, beta), unsplit.magnetization(C, T, A, beta)
    assert abs(ms) > 1e-3
    assert abs(ms - mu) < 1e-12


@pytest.mark.parametrize("n", [1, 2])
def test_bond_correlation_untruncated_split_equals_unsplit(n):
    """The split two-site patch (two columns absorbed layer by layer) and the
    fused-site two-site patch are independent codes for the same finite network
    when nothing is truncated."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 1))
    O = model.pepo_O(beta)
    env, _, _, _ = split.run(A, O, 10 ** 9, n)
    C, T, _, _ = unsplit.run(model.fuse_triple(A, O), (2, 2, 2), 10 ** 9, n)
    assert abs(split.bond_correlation(env, A, beta) - unsplit.bond_correlation(C, T, A, beta)) < 1e-12


@pytest.mark.parametrize("n", [1, 2])
def test_energy_untruncated_split_equals_unsplit(n):
    """The energy impurity in the split patch and in the fused-site patch:
    independent codes for the same finite network when nothing is truncated."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 1))
    O = model.pepo_O(beta)
    env, _, _, _ = split.run(A, O, 10 ** 9, n)
    C, T, _, _ = unsplit.run(model.fuse_triple(A, O), (2, 2, 2), 10 ** 9, n)
    assert abs(split.energy(env, A, beta) - unsplit.energy(C, T, A, beta)) < 1e-12


def test_split_product_state_energy_is_the_closed_form():
    beta = 0.2
    P = model.embed_product_state(2, +1)
    env, _, _, _ = split.run(P, model.pepo_O(beta), 16, 300, tol=1e-13)
    assert abs(split.energy(env, P, beta) - exact.product_state_energy(beta, +1)) < 1e-10


def test_split_product_state_bond_correlation_is_onsagers():
    beta = 0.2
    P = model.embed_product_state(2, +1)
    env, _, _, _ = split.run(P, model.pepo_O(beta), 16, 300, tol=1e-13)
    assert abs(split.bond_correlation(env, P, beta) - exact.onsager_nn_correlation(beta)) < 1e-10


def test_magnetization_spin_flip_and_symmetric_state():
    """Z2: flipping the physical index of A (A[p] -> A[1 - p]) maps the network
    with O to itself and Oz to -Oz, so m changes sign; the flip-symmetric product
    state (1, 1)/sqrt(2) has m = 0; |m| <= 1."""
    beta, chi = 0.2, 12
    A = model.d4_symmetrize(raw_peps(2, 1))
    O = model.pepo_O(beta)
    for B, want in ((A, None), (A[::-1].copy(), "flip")):
        env, _, _, _ = split.run(B, O, chi, 40)
        C, T, _, _ = unsplit.run(model.fuse_triple(B, O), (2, 2, 2), chi, 40)
        m = (split.magnetization(env, B, beta), unsplit.magnetization(C, T, B, beta))
        if want is None:
            m0 = m
        else:
            assert abs(m[0] + m0[0]) < 1e-10 and abs(m[1] + m0[1]) < 1e-10
    assert 1e-3 < abs(m0[1]) <= 1.0
    P = model.embed_product_state(2, +1)
    env, _, _, _ = split.run(P, O, chi, 20)
    assert abs(split.magnetization(env, P, beta)) < 1e-13


@pytest.mark.parametrize("sign", [+1, -1])
@pytest.mark.parametrize("D", [2, 3])
def test_unsplit_product_state_closed_form(sign, D):
    beta = 0.2
    f, _ = unsplit.free_energy(beta, model.embed_product_state(D, sign), 24, 100)
    assert abs(f - exact.product_state_f(beta, sign)) < 1e-10


@pytest.mark.parametrize("n", [1, 2])
def test_unsplit_equals_brute_force_patches(n):
    """n untruncated steps from the product boundary represent the finite patches
    exactly: kappa = Z(2n+1,2n+1) Z(2n,2n) / (Z(2n+1,2n) Z(2n,2n+1))."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 0))
    a3 = model.fuse_triple(A, model.pepo_O(beta))
    e = unsplit.boundary_vector((2, 2, 2))
    C, T, _, _ = unsplit.run(a3, (2, 2, 2), 10 ** 6, n)
    n1, n2, n0 = unsplit.patch_values(C, T, a3)
    Z = lambda x, y: exact.patch_value(a3, e, x, y)  # noqa: E731
    kb = Z(2 * n + 1, 2 * n + 1) * Z(2 * n, 2 * n) / (Z(2 * n + 1, 2 * n) * Z(2 * n, 2 * n + 1))
    assert abs(n1 * n0 / n2 ** 2 / kb - 1) < 1e-12


# --------------------------------------------------------------- split CTMRG

@pytest.mark.parametrize("n", [1, 2])
def test_split_untruncated_equals_unsplit(n):
    """Without truncation the split environment reproduces the reduced one: same
    per-site kappa and the same corner eigenvalues (the spectrum of rho_eff up to
    the bond gauge)."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 0))
    O = model.pepo_O(beta)
    a3 = model.fuse_triple(A, O)
    env, _, _, _ = split.run(A, O, 10 ** 9, n)
    n1, n2h, n2v, n0 = split.patch_values(env, A, O)
    C, T, _, _ = unsplit.run(a3, (2, 2, 2), 10 ** 9, n)
    m1, m2, m0 = unsplit.patch_values(C, T, a3)
    assert abs(n1 * n0 / (n2h * n2v) / (m1 * m0 / m2 ** 2) - 1) < 1e-12
    ev_s = np.sort(np.abs(np.linalg.eigvals(split.rho_eff(env))))[::-1]
    ev_u = np.sort(np.abs(np.linalg.eigvalsh(C)) ** 4)[::-1]
    k = min(ev_s.size, ev_u.size)
    ev_s, ev_u = ev_s[:k] / ev_s.sum(), ev_u[:k] / ev_u.sum()
    big = ev_u > 1e-10
    assert np.allclose(ev_s[big], ev_u[big], rtol=1e-8)


@pytest.mark.parametrize("sign", [+1, -1])
def test_split_product_state_closed_form(sign):
    beta = 0.2
    f, _ = split.free_energy(beta, model.embed_product_state(2, sign), 16, 300, tol=1e-13)
    assert abs(f - exact.product_state_f(beta, sign)) < 1e-8


def test_split_converges_to_reduced_method():
    """Sec. IV A: the split scheme reaches the reduced-method value as chi grows."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 0))
    f_ref, _ = unsplit.free_energy(beta, A, 48, 100)
    errs = []
    for chi in (8, 16, 32):
        f, _ = split.free_energy(beta, A, chi, 100)
        errs.append(abs(f - f_ref))
    assert errs[-1] < 1e-10
    assert errs[0] > errs[1] > errs[2]


def test_growth_phase_projectors_do_not_cut_below_chi():
    """Sec. III C, environment selection: the rank of rho_B rho_T is bounded by
    the corner matrices of its patch.  On the first truncated move after the
    product boundary the corner bond is still below chi, so that bound reflects
    the small environment; the pair is then the orthogonal projector onto the
    leading eigenvectors of the truncated legs' Gram matrix and no bond is cut
    below min(chi, n).  For the norm network of this tensor the rank-limited
    projectors cut two bonds to 8 of chi = 16 at move 2 and the iteration never
    settled; with the rule it converges to the reduced method's value."""
    A = model.d4_symmetrize(raw_peps(2, 15))
    A /= np.linalg.norm(A)
    O = model.identity_pepo()
    env = split.init_env(2, 1)
    env, _ = split.step(env, A, O, split.GROW_CHI)
    assert split.growing(env, 16)
    env, projs = split.step(env, A, O, 16)
    assert split.bond_dims(env) == (16, 16, 16) and not split.growing(env, 16)
    filled = [name for name, (PT, PB, S) in projs.items() if S.size == 0 and PT.shape[0] < PT.shape[1]]
    assert filled
    for name in filled:
        PT, PB, _ = projs[name]
        assert np.allclose(PT @ PB, np.eye(PT.shape[0]), atol=1e-12) and np.allclose(PT, PB.T), name
    env, it, _, _ = split.run(A, O, 16, 300, 1e-9, 1e-12)
    a = model.fuse_double(A)
    C, T, _, _ = unsplit.run(a, (2, 2), 48, 300, 1e-12)
    assert it < 300
    assert abs(split.log_kappa(env, A, O)[0] - unsplit.log_kappa(C, T, a)[0]) < 1e-7


def test_split_double_layer_matches_reduced_norm():
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 3))
    _, info_s = split.free_energy(beta, A, 32, 100)
    _, info_u = unsplit.free_energy(beta, A, 48, 100)
    assert abs(info_s["log_kappa2"] - info_u["log_kappa2"]) < 1e-10


def test_split_d2_relation_and_projector_identity():
    """n2 strips agree in both orientations (D2 relations) and every projector
    pair satisfies P_T P_B = I (Sec. III B)."""
    beta = 0.22
    A = model.d4_symmetrize(raw_peps(2, 1))
    O = model.pepo_O(beta)
    env, _, _, _ = split.run(A, O, 12, 8)
    n1, n2h, n2v, n0 = split.patch_values(env, A, O)
    assert abs(n2h / n2v - 1) < 1e-12
    assert np.allclose(env["C1"], env["C1"].T) and np.allclose(env["C4"], env["C4"].T)
    _, projs = split.step(env, A, O, 12)
    for name, (PT, PB, S) in projs.items():
        assert np.allclose(PT @ PB, np.eye(PT.shape[0]), atol=1e-9), name


def test_split_invariants():
    """f(cA) = f(A); f is invariant under the spin flip of the physical leg
    (Ising Z2); <A, g> = 0 (g is the log-derivative difference)."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 4))
    f, g, _ = split.f_and_grad(beta, A, 12, 60)
    f2, _ = split.free_energy(beta, 3.7 * A, 12, 60)
    f3, _ = split.free_energy(beta, A[::-1].copy(), 12, 60)
    assert abs(f2 - f) < 1e-11 and abs(f3 - f) < 1e-11
    assert abs(np.sum(A * g)) < 1e-12 * np.linalg.norm(A) * np.linalg.norm(g) * 100


def test_split_gradient_central_differences():
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 0))
    f, g, _ = split.f_and_grad(beta, A, 16, 300, tol=1e-13)
    h = 1e-5
    for v in random_directions(A.shape, 2, 11):
        v = model.d4_symmetrize(v)
        v /= np.linalg.norm(v)
        fp, _ = split.free_energy(beta, A + h * v, 16, 300, tol=1e-13)
        fm, _ = split.free_energy(beta, A - h * v, 16, 300, tol=1e-13)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - np.sum(g * v)) < 1e-5 * abs(fd)


def test_split_gradient_matches_reduced_gradient():
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(2, 0))
    _, g_s, _ = split.f_and_grad(beta, A, 32, 100)
    _, g_u, _ = unsplit.f_and_grad(beta, A, 48, 100)
    assert np.linalg.norm(g_s - g_u) < 1e-8 * np.linalg.norm(g_u)


def test_split_halves_are_related_by_the_180_degree_rotation():
    """Eq. (Symmetry constraints): the 180-degree rotation about the PEPO site
    swaps ket and bra, left and right, up and down.  It maps every upper half
    used for a projector onto the matching lower half, so these pairs must be
    index permutations of each other."""
    beta = 0.2
    A = model.d4_symmetrize(raw_peps(3, 0))
    O = model.pepo_O(beta)
    env, _, _, _ = split.run(A, O, 20, 4)
    up_ki, up_ib, up_bk = split.upper_sequence(env, A, O)
    lo_ki, lo_ib, lo_bk = split.lower_sequence(env, A, O)
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)  # noqa: E731
    assert rel(lo_bk, up_bk.transpose(4, 1, 2, 3, 0)) < 1e-13
    assert rel(lo_ib, np.einsum("fqbeca->aqbcef", up_ki)) < 1e-13
    assert rel(lo_ki, np.einsum("fpobca->apobcf", up_ib)) < 1e-13
    P1, P2, P3 = split.stage1(env, A, O, 20)
    split.stage2(env, A, O, 20, P1, P2, P3)
    E = split.LAST_STAGE2_ENVS
    assert rel(E["rhoB5"], np.einsum("gfebca->abcefg", E["rhoT6"])) < 1e-13
    assert rel(E["rhoB6"], np.einsum("gefcba->abcefg", E["rhoT5"])) < 1e-13


# ---------------------------------------------------------------- beta -> 0

@pytest.mark.parametrize("method", ["unsplit", "split"])
def test_beta_to_zero_product_state(method):
    """beta f(A+) -> -ln 2 for the |+> product state.  At small beta the 2D
    high-temperature expansion gives ln kappa_2D = ln 2 + 2 ln cosh b + O(b^4),
    so beta f + ln 2 = -(ln cosh b + ln kappa_2D - ln 2) = -3/2 b^2 + O(b^4):
    the CTMRG value approaches -ln 2 quadratically with that coefficient."""
    mod = unsplit if method == "unsplit" else split
    A = model.embed_product_state(2, +1)
    e = []
    for beta in (0.05, 0.01):
        f, _ = mod.free_energy(beta, A, 8, 400, tol=1e-13)
        e.append((beta * f + np.log(2.0)) / beta ** 2)
    assert abs(e[1] + 1.5) < 2e-3
    assert abs(e[1] + 1.5) < abs(e[0] + 1.5)


@pytest.mark.parametrize("method", ["unsplit", "split"])
def test_beta_to_zero_random_tensor(method):
    """At beta = 0 every entry of sqrt(W) is 1/sqrt2, so O is the constant 1/4:
    each in-plane PEPO bond sums to 2 (two per site), and the PEPO layer
    reduces to 2 |+><+| between the ket and the bra.  Hence
    -beta f -> ln 2 + ln kappa2(A+) - ln kappa2(A) with A+ = sum_p A_p / sqrt2,
    a value that needs only norm networks.  sqrt(W) = sqrt(2 cosh b) |+><+| +
    sqrt(2 sinh b) |-><-| and only even powers of the second term survive the
    spin sum in O, so the approach is linear in beta.

    The split iteration runs at chi = 24.  At chi = 16 and beta = 8e-3 (or
    1e-3) it settles, from the product boundary, on a second attractor whose
    ln kappa3 is 0.1198 below the reduced value for this tensor (a 1e-3
    perturbation of the starting environment reaches the right one): at small
    beta the PEPO's in-plane legs are nearly rank one and a subleading pair of
    the corner spectrum is nearly degenerate."""
    mod = unsplit if method == "unsplit" else split
    D = 2
    A = model.d4_symmetrize(raw_peps(D, 4))
    A /= np.linalg.norm(A)
    Ap = (A.sum(axis=0) / np.sqrt(2.0))[None]
    lk2 = []
    for X in (A, Ap):
        a = model.fuse_double(X)
        C, T, _, _ = unsplit.run(a, (D, D), 16, 400, 1e-13)
        lk2.append(unsplit.log_kappa(C, T, a)[0])
    limit = np.log(2.0) + lk2[1] - lk2[0]
    err = []
    chi = 16 if method == "unsplit" else 24
    for beta in (8e-3, 2e-3):
        f, _ = mod.free_energy(beta, A, chi, 400, tol=1e-13)
        err.append(-beta * f - limit)
    assert 0.1 < err[0] / 8e-3 < 0.4 and 0.1 < err[1] / 2e-3 < 0.4
    assert abs(err[1] / err[0] - 0.25) < 0.05
