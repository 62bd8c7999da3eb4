/*
 * ctm.h -- C ABI of the split-CTMRG library (libctm.so, HIP / gfx950).
 *
 * The library contracts the two infinite networks of the variational iPEPS
 * method for 3D classical models -- the triple-layer <psi(A)|T|psi(A)> with the
 * 3D Ising PEPO T, and the double-layer norm <psi(A)|psi(A)> -- with the split
 * corner-transfer-matrix renormalisation group, and returns the free-energy
 * density f(beta, A) of Eq. (free energy expression) and its gradient g of
 * Eq. (gradient expression).
 *
 *   environment    Sec. III A: corners C_i and one edge tensor per layer
 *                  (T^ket, T^int, T^bra); the D2 relations of Eq. (Symmetry
 *                  constraints) leave C1 (= C3), C4 (= C2) and the left-edge
 *                  chain as the stored state.
 *   one iteration  Sec. III B: absorption of one column into all four
 *                  directions at once, two-stage truncation of every bond with
 *                  six projector pairs (P1..P3 bra-related, P4..P6 ket-related),
 *                  built as in Sec. III C and the Appendix (six-projector scheme).
 *   convergence    Sec. III D: l2 change of the singular values of
 *                  C1 C2 C3 C4 / Tr(C1 C2 C3 C4).
 *
 * Layouts.  The PEPS tensor A and the gradient g are dense float64 arrays of
 * 2 * D^4 entries, row-major over [p][l][u][r][d] (p physical, then the four
 * virtual legs left, up, right, down).  A is copied at init; the caller keeps
 * ownership of every pointer it passes.  Pointers are host pointers unless
 * cfg->flags has CTM_FLAG_DEVICE_PTRS set, in which case A and g are device
 * pointers on the current HIP device.
 *
 * Streams.  The work of every call is ordered after the work already
 * enqueued on the hip_stream given at init (NULL = the legacy default stream),
 * and work enqueued on that stream after the call returns is ordered after
 * it.  Inside a call the two networks run concurrently on two streams the
 * context owns (default priority), each driven by its own host thread.  Calls
 * that return host values (ctm_iterate's delta, ctm_free_energy, ctm_grad
 * with host g, spectra) synchronise.  A context must be used by one host
 * thread at a time; distinct contexts are independent.
 *
 * Errors.  Every call returns a ctm_status; nothing is thrown across the ABI.
 * ctm_last_error() gives a message for the last failing call on a context.
 */
#ifndef CTM_H
#define CTM_H

#ifdef __cplusplus
extern "C" {
#endif

#define CTM_ABI_VERSION 5

typedef struct ctm_ctx ctm_ctx;

typedef enum {
    CTM_OK = 0,
    CTM_EINVAL = 1,     /* bad argument: beta <= 0, D < 1, chi < 1, NULL ... */
    CTM_ENOMEM = 2,     /* device memory: allocation failed, or the temporaries */
                        /* exceed the fixed scratch of ctm_free_energy_noalloc */
    CTM_EDEVICE = 3,    /* a HIP call failed                                  */
    CTM_ENOCONV = 4,    /* max_iter reached before tol; results stay readable */
    CTM_ENUMERIC = 5,   /* NaN/Inf or a non-positive network value            */
    CTM_ESTATE = 6      /* call out of order (e.g. f before any iteration)    */
} ctm_status;

typedef enum {
    CTM_FP64 = 0,       /* every contraction in float64                          */
    CTM_FP32 = 1,       /* bulk contractions float32 products / float32 accumulate */
    CTM_BF16 = 2        /* bulk contractions bfloat16 products / float32 accumulate */
} ctm_precision;
/* In the reduced-precision forms the bulk contractions of a move of the
 * triple-layer network (the layer-by-layer absorption that builds the
 * corners, edges and the projector environments rho_T, rho_B, and the
 * renormalisation with the projectors) run on the FP32 or BF16 matrix cores
 * with FP32 accumulation; the double-layer (norm) network, the cheaper one
 * and the one whose environment is the more sensitive to rounding, stays
 * FP64.  The projector
 * construction -- the product rho_B rho_T, its factorisation and the
 * application of V S^-1/2 and S^-1/2 U^T -- the corner spectrum, the
 * normalisations and f and g stay FP64.  Tensors are stored in FP64
 * throughout (operands are rounded when they are staged for the matrix
 * cores).  During the reduced-precision phase the relative pseudo-inverse
 * cutoff is raised to the rounding level of the products (1e-7 FP32, 1e-3
 * BF16).  The phase ends when the spectrum change drops below
 * max(tol, lp_tol); with refine = 1 the iteration then continues in FP64
 * (with svd_cutoff) until the change is below tol, and the phase also ends
 * once a quarter of max_iter is spent. */

#define CTM_FLAG_DEVICE_PTRS 1
#define CTM_FLAG_PROFILE 2      /* record HIP events around GEMM / Jacobi launches */
/* CTM_FLAG_REDUCED: contract both networks with the reduced method instead of
 * split-CTMRG (Sec. II; the comparison method of Sec. IV): the ket, PEPO and
 * bra layers of a site are fused into one tensor a with bond D^2 d (norm
 * network: D^2), and a C4v-symmetric CTMRG with one corner C (chi x chi) and
 * one edge T (chi x D^2 d x chi) truncates the enlarged corner to the chi
 * eigenvectors of largest |eigenvalue| (svd_cutoff relative to the largest).
 * Convergence uses the singular values of C^4 / Tr C^4 (Sec. III D); f and g
 * use the same estimators as the split path.  CTM_FP64 only (CTM_EINVAL
 * otherwise).  Device memory grows as chi^2 (D^2 d)^2 for the enlarged
 * corner and (D^2 d)^4 for a. */
#define CTM_FLAG_REDUCED 4
/* CTM_FLAG_FULL_P4: build the second-stage projector of the cell-boundary bond
 * (projector 4) from the full 2x2 block of enlarged corners, vertical legs
 * renormalised by projector 1 and its right-move image, horizontal legs whole
 * (Appendix, Fig. Projector4(a); O(chi^3 D^4 d^3)).  Default: the half
 * construction of the main text from the two left enlarged corners, their
 * horizontal legs renormalised by the up / down images of projector 1
 * (Fig. Projector4(b); O(chi^3 D^3 d^3)).  The full construction's
 * rho_B rho_T is a product of four corners, whose spectrum decays as the
 * square of the half one's: the same svd_cutoff keeps fewer directions.
 * Split-CTMRG only. */
#define CTM_FLAG_FULL_P4 8

typedef struct {
    int D;              /* PEPS virtual bond dimension, 1 <= D <= 8               */
    int chi;            /* environment bond dimension, 1 <= chi <= 512            */
    int max_iter;       /* cap used by ctm_iterate(n_iter <= 0)                   */
    double tol;         /* convergence threshold on the spectrum change (>= 0)    */
    int precision;      /* ctm_precision of the bulk contractions                 */
    int flags;          /* CTM_FLAG_* bits                                        */
    int power_iters;    /* subspace iterations of the projector SVD (0: default)  */
    double svd_cutoff;  /* relative singular-value cutoff (0: default 1e-8)       */
    double lp_tol;      /* end of the reduced-precision phase (0: 1e-6 FP32,      */
                        /* 1e-2 BF16); ignored for CTM_FP64                       */
    int refine;         /* 1: continue in FP64 to tol after that phase            */
} ctm_config;

/* Build a context: the PEPO O of the 3D Ising model at inverse temperature
 * beta (Sec. IV: O = delta grouped with six sqrt(W) factors), the D4 projection
 * of A (Sec. III B), and the product-boundary initial environments of both
 * networks.  beta must be > 0.  On success *out owns all device memory it
 * allocates; release it with ctm_destroy.  On failure *out is NULL. */
ctm_status ctm_init(const ctm_config* cfg, double beta, const double* A,
                    void* hip_stream, ctm_ctx** out);

/* Run split-CTMRG iterations on both networks.  n_iter > 0: exactly n_iter
 * moves.  n_iter == 0: until the spectrum change of both networks is below
 * cfg->tol, or max_iter moves since init or the last ctm_reset_tensor (then
 * CTM_ENOCONV).  n_iter < 0: the same stopping rule for at most -n_iter moves
 * (a slice; CTM_ENOCONV only when max_iter is reached).  iters_done (may be
 * NULL) receives the moves done by this call and last_delta (may be NULL) the
 * larger of the two spectrum changes of the last move. */
ctm_status ctm_iterate(ctm_ctx* c, int n_iter, int* iters_done, double* last_delta);

/* Continuous-batching form of ctm_iterate for n (1..64) distinct contexts
 * (serving: independent f-and-gradient requests, any shapes).  In every move
 * the two networks of every still-active context step concurrently, each on
 * its own stream and host thread; each context applies the stopping rule of
 * ctm_iterate for the given n_iter and leaves the batch when it is done, so a
 * scheduler can call it with n_iter < 0 in slices and add or retire contexts
 * between calls.  The results of a context do not depend on the other members
 * of the batch.  iters_done, last_delta, converged (1 when the stopping rule
 * was met) and status (each may be NULL) receive one entry per context; the
 * return value is the first non-OK status (CTM_EINVAL for a NULL or repeated
 * context or n out of range). */
ctm_status ctm_iterate_batch(ctm_ctx** cs, int n, int n_iter, int* iters_done, double* last_delta,
                             int* converged, int* status);

/* f = -(ln kappa3 - ln kappa2) / beta with the per-site values kappa of the
 * triple- and double-layer networks estimated as n1 n0 / (n2h n2v) from the
 * current environments (Eq. free energy expression).  Any output pointer may be
 * NULL.  CTM_ESTATE before the first iteration. */
ctm_status ctm_free_energy(ctm_ctx* c, double* f, double* log_kappa3, double* log_kappa2);

/* The same result as ctm_free_energy for callers that cannot allocate device
 * memory (code that must not call hipMalloc, e.g. between graph captures or in
 * tight serving loops): the contraction temporaries of both networks come from
 * a fixed 128 MiB device array inside the library (64 MiB per network), one
 * per GPU, held until the process ends; the call makes no hipMalloc or
 * hipFree.  Returns CTM_ENOMEM (message in ctm_last_error) when the
 * temporaries do not fit (e.g. D = 5, chi = 100); the context and its
 * environments are then unchanged.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (two host threads, two contexts) race
 * on it.  Same arguments, ownership and other errors as ctm_free_energy. */
ctm_status ctm_free_energy_noalloc(ctm_ctx* c, double* f, double* log_kappa3, double* log_kappa2);

/* g = -(2/beta) (E3/n1_3 - E2/n1_2), the environment of the bra tensor in the
 * 3x3 patch of each network normalised by that patch's value, projected onto
 * the D4-symmetric subspace (Eq. gradient expression).  g has 2 D^4 entries in
 * the layout of A (host or device per CTM_FLAG_DEVICE_PTRS). */
ctm_status ctm_grad(ctm_ctx* c, double* g);

/* Singular values of C1 C2 C3 C4 / |Tr(C1 C2 C3 C4)| of the current
 * environment for network which = 3 (triple layer) or 2 (double layer),
 * descending, computed on the call with converged Jacobi sweeps (a move far
 * from convergence estimates its spectrum change with fewer); *n receives the
 * count (<= cap).  Host buffer.  Synchronises. */
ctm_status ctm_corner_spectrum(ctm_ctx* c, int which, double* s, int cap, int* n);

/* Replace beta and A and keep the converged environments as the starting
 * point of the next ctm_iterate (warm restart); max_iter of ctm_iterate(0)
 * counts from here, and a reduced-precision context starts its
 * reduced-precision phase again. */
ctm_status ctm_reset_tensor(ctm_ctx* c, double beta, const double* A);

/* Iterations done so far, and the device bytes the context holds. */
ctm_status ctm_query(const ctm_ctx* c, int* total_iters, long long* device_bytes);

/* Magnetisation <sigma> of a spin of the PEPO layer (Sec. IV B: local
 * observables as impurity tensors in the converged environment): the 3x3
 * patch of the triple-layer network with the centre PEPO replaced by the
 * impurity PEPO Oz (the spin's value +1 / -1 for s = 0 / 1 under the sum over
 * s), divided by the same patch with O.  Both methods (split and reduced).
 * *m receives the host double.  CTM_ESTATE before any iteration,
 * CTM_ENUMERIC when the patch value is zero or non-finite. */
ctm_status ctm_magnetization(ctm_ctx* c, double* m);

/* In-plane nearest-neighbour correlation <sigma sigma'> of two PEPO-layer
 * spins (the bond energy of Sec. IV B, -J <sigma sigma'> per in-plane bond):
 * the 3x4 patch of the triple-layer network around two horizontally adjacent
 * sites, both with the impurity PEPO Oz, divided by the same patch with O.
 * Both methods (split: two edge columns and two sites absorbed layer by layer;
 * reduced: left and right half of the fused-site patch).  *zz receives the
 * host double.  CTM_ESTATE
 * before any iteration, CTM_ENUMERIC when the patch value is zero or
 * non-finite. */
ctm_status ctm_bond_correlation(ctm_ctx* c, double* zz);

/* Internal energy per site U (Sec. IV B: U from an impurity tensor in the
 * converged environment; J = 1, three links per site):
 * U = -n1(dO/dbeta) / n1(O), the 3x3 patch of the triple-layer network with
 * the centre PEPO replaced by its beta derivative (product rule over the six
 * sqrt(W) legs), divided by the same patch with O.  This is -d ln kappa3 /
 * d beta at fixed A, i.e. d(beta f)/d beta wherever f is stationary in A (at
 * the variational optimum).  Both methods.  *u receives the host double.
 * CTM_ESTATE before any iteration, CTM_ENUMERIC when the patch value is zero
 * or non-finite. */
ctm_status ctm_energy(ctm_ctx* c, double* u);

/* Launch statistics of a context built with CTM_FLAG_PROFILE: which = 0 the
 * FP64 MFMA GEMM kernel, 1 the Jacobi SVD kernels, 2 the Cholesky QR kernels,
 * 3 the FP32 / BF16 MFMA GEMM kernel, 4 the split-K reduction of the GEMMs,
 * 5 the part of class 0 issued by the factorisations (subspace iteration,
 * Cholesky-QR Gram and triangular products, Rayleigh-Ritz, projector
 * assembly P_B = rho_T V S^-1/2, P_T = S^-1/2 U^T rho_B); class 0 minus
 * class 5 are the contraction products.
 * launches, summed kernel time in ms (HIP events on the context's streams
 * around each launch; the two network streams may overlap) and algorithmic
 * flops: 2 M N K per GEMM; per Jacobi sweep and column pair 12 m (+ 6 n with
 * V); 2 k^3 / 3 per Cholesky-QR factor; none for the reduction.  bytes: the
 * algorithmic operand and result bytes, 8 (M K + K N + M N) per GEMM (0 for
 * the other classes).  Synchronises.  Any output may be NULL.  CTM_ESTATE
 * without CTM_FLAG_PROFILE. */
ctm_status ctm_kernel_stats(ctm_ctx* c, int which, long long* launches, double* ms, double* flops,
                            double* bytes);

/* Release a context.  NULL-safe. */
void ctm_destroy(ctm_ctx* c);

/* Message of the last failing call on c (or of the last failing ctm_init when
 * c is NULL).  Never NULL. */
const char* ctm_last_error(const ctm_ctx* c);

const char* ctm_status_string(int status);

int ctm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CTM_H */
