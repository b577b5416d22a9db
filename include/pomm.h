/*
 * pomm.h -- C ABI of libpomm: preconditioned orbital minimization (OMM) for a
 * planewave (Fourier pseudospectral) Hamiltonian on one AMD MI355X (gfx950).
 *
 * Problem (Section 1, eq. tracemin): the span of the N lowest eigenvectors of
 * the n x n Hermitian matrix H = -Laplacian/2 + V discretized on a periodic
 * grid (Section 4.1: kinetic part diagonal in Fourier space, V diagonal in
 * real space).  The library minimizes the unconstrained OMM energy
 * E_omm(X) = 1/2 tr((2I - X*X)(X* H_sigma X)) (eq. omm) for the shifted,
 * negative definite H_sigma = H - sigma I (Section 1), by preconditioned
 * nonlinear conjugate gradients (Algorithm 1) with an exact quartic line
 * search, preconditioned by the pole expansion of the Fermi projector
 * (eq. dFOP) whose resolvents are applied by rough GMRES solves (eqs. direct,
 * lst) with the sparsifying preconditioner (Section 3.2, eq. P) or the
 * inverse shifted Laplacian as inner preconditioner.
 *
 * Conventions shared by every entry point
 *   - Domain [0, 2*pi)^dim, m points per axis (m even), n = m^dim, grid
 *     coordinate x_j = 2*pi*j/m; flat grid index j = j1 + m*j2 (+ m*m*j3).
 *     Frequencies k_i in {-m/2, ..., m/2-1}; kinetic symbol |k|^2/2.
 *   - Orbital blocks are column-major n x ncols arrays (leading dimension n)
 *     of interleaved complex numbers: complex128 (double re, double im) for
 *     OMM_PREC_FP64, complex64 for OMM_PREC_FP32.
 *   - Pointers named "device" must be device memory on the handle's GPU; the
 *     caller owns them.  V is read from host memory and copied at setup.
 *   - Every call is enqueued on the handle's HIP stream.  ommApplyH and
 *     ommPrecondition return without waiting; ommSolve and ommSetup return
 *     after their device work is complete.
 *   - Every entry point returns an omm status code and never throws.  After a
 *     failure ommLastError(h) holds a message (for ommSetup failures, use
 *     ommLastError(NULL)).  A handle must not be used from two host threads
 *     at once; distinct handles are independent.
 */
#ifndef POMM_H
#define POMM_H

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define OMM_OK            0
#define OMM_EINVAL        1  /* bad grid / size / NULL pointer / option out of range      */
#define OMM_ENOTNEGDEF    2  /* shift does not make H - shift*I negative definite          */
#define OMM_ESPECTRUM     3  /* spectral window inconsistent: need lo < homo < lumo        */
#define OMM_ENOMEM        4  /* device allocation failed                                   */
#define OMM_EHIP          5  /* HIP runtime error                                          */
#define OMM_ENOCONV       6  /* iteration cap reached; X still holds the last iterate      */
#define OMM_EBREAKDOWN    7  /* line search breakdown: quartic leading coefficient <= 0    */
#define OMM_EUNSUPPORTED  8  /* valid request that this build does not implement          */

/* Precision of an orbital block at the boundary. */
#define OMM_PREC_FP64     0  /* complex128 */
#define OMM_PREC_FP32     1  /* complex64  */

/* omm_opts_t.precision: arithmetic of the solve. */
#define OMM_FP64          0  /* everything in FP64                                          */
#define OMM_MIXED         1  /* FFT, H.X and Krylov in FP32; Gram, energy, line search FP64 */

/* omm_opts_t.inner: inner preconditioner of the GMRES solves. */
#define OMM_INNER_SPP     0  /* sparsifying preconditioner (Section 3.2)                    */
#define OMM_INNER_PP      1  /* inverse shifted Laplacian (Section 3.2, first paragraph)    */

/* omm_opts_t.poles: contour quadrature of eq. dFOP. */
#define OMM_POLES_ELLIPTIC 0 /* conformal-map (Hale-Higham-Trefethen type) rule             */
#define OMM_POLES_CIRCLE   1 /* trapezoid rule on a circle through lo - (homo - lo) and homo */

/* omm_opts_t.gmres_side: preconditioning side of the rough GMRES solves
 * (Section 3.1 leaves it open). */
#define OMM_SIDE_AUTO      0 /* right for OMM_FP64, left for OMM_MIXED                       */
#define OMM_SIDE_RIGHT     1 /* GMRES on A M^{-1}; stop on ||g - A y|| <= rtol ||g||          */
#define OMM_SIDE_LEFT      2 /* GMRES on M^{-1} A; stop on ||M^{-1}(g - A y)|| <= rtol times
                                its value at y0 (in FP32 the true residual of the stiff
                                operator carries round-off that M^{-1} damps)               */

/* omm_opts_t.outer: preconditioner of Algorithm 1.  FERMI is the paper's pole
 * expansion (Section 3); LAPLACE and TPA are the Fourier-diagonal comparison
 * preconditioners of Section 3.1 (eqs. Lap and TPA) with scale opts.tau:
 * 1/(1 + |k|^2/tau) and q(s)/(q(s) + 16 s^4), q(s) = 27 + 18s + 12s^2 + 8s^3,
 * s = |k|^2/tau.  With LAPLACE or TPA the start is not filtered and
 * ommPrecompute is not available. */
#define OMM_OUTER_FERMI   0
#define OMM_OUTER_LAPLACE 1
#define OMM_OUTER_TPA     2

/* omm_opts_t.spp_products: arithmetic of the dense block products of the sparse
 * direct solve (block cyclic reduction levels >= 1) in the OMM_MIXED form. */
#define OMM_PRODUCTS_SPLIT16 0 /* each complex64 operand as fp16 hi + lo with a power-of-two
                                  scale, three fp16 products per real product, fp32
                                  accumulation: about complex64 accuracy              */
#define OMM_PRODUCTS_FP32    1 /* complex64 products on the fp32 matrix cores          */
#define OMM_PRODUCTS_F16     2 /* factor blocks rounded once to fp16 (with a power-of-two
                                  scale per block), right-hand sides split as in SPLIT16:
                                  two fp16 products per real product and half the factor
                                  bytes.  The sparse solve stays a fixed linear operator
                                  (its factors within 2^-12 per element of the exact
                                  ones), so GMRES still reaches its tolerance on
                                  (H - z_j); only the preconditioner's quality changes  */

/* Stop rule reported in omm_info_t.stop_rule. */
#define OMM_STOP_GRAD     1  /* rel_grad <= tol                                             */
#define OMM_STOP_ENERGY   2  /* energy unchanged to 8 eps |E| for `stall` iterations         */
#define OMM_STOP_MAXIT    3  /* maxit line searches                                         */

typedef struct {
    int dim;      /* 2 or 3                                                    */
    int m[3];     /* points per axis; this build requires m[0]=m[1](=m[2]),    */
                  /* m even, m = 2^a * 3^b with b <= 1, 8 <= m <= 128           */
} omm_grid_t;

/* Spectral window of the UNSHIFTED H (Section 4: the contour is built from
 * spectral information).  Occupied eigenvalues lambda_1..lambda_N must lie in
 * [lo, homo] and unoccupied ones in [lumo, +inf), lo < homo < lumo. */
typedef struct {
    double lo;    /* lower bound of lambda_1 (min V is always valid)          */
    double homo;  /* upper bound of lambda_N                                   */
    double lumo;  /* lower bound of lambda_{N+1}                               */
} omm_spectrum_t;

typedef struct {
    int    precision;      /* OMM_FP64 | OMM_MIXED                      default OMM_FP64   */
    int    inner;          /* OMM_INNER_SPP | OMM_INNER_PP              default SPP        */
    int    poles;          /* OMM_POLES_ELLIPTIC | OMM_POLES_CIRCLE     default ELLIPTIC   */
    int    npoles;         /* even, 2..64; 0 = automatic (see pole_tol)  default 30         */
    double gmres_rtol;     /* relative residual of the rough solves     default 1e-5       */
    int    gmres_restart;  /* Krylov dimension per cycle, 1..32          default 15         */
    int    gmres_cycles;   /* restart cycles, >= 1                       default 5          */
    double filter_rtol;    /* GMRES tolerance of the initial filter     default 1e-5       */
    double tol;            /* stop when ||G(X)||_F / ||H_sigma X||_F <= tol, default 1e-10  */
    int    maxit;          /* line searches cap                          default 4000       */
    int    stall;          /* energy-stagnation window, 0 disables      default 3          */
    int    filter;         /* 1: X1 = P X0 before Algorithm 1           default 1          */
    double pole_tol;       /* npoles = 0 with the elliptic rule: the smallest even p >= 30
                              whose quadrature error rate exp(-pi K' p / (4K)) is at most
                              pole_tol (the rate of the conformal map, see ommSetup)
                                                                        default 1e-9       */
    int    gmres_side;     /* OMM_SIDE_AUTO | _RIGHT | _LEFT             default AUTO       */
    int    spp_products;   /* OMM_PRODUCTS_SPLIT16 | _FP32 | _F16 (OMM_MIXED) default SPLIT16 */
    int    outer;          /* OMM_OUTER_FERMI | _LAPLACE | _TPA          default FERMI      */
    double tau;            /* kinetic scale of OMM_OUTER_LAPLACE / _TPA (> 0 there)   default 0 */
    int    gmres_verify;   /* 1: a restart cycle whose systems all met rtol by the Arnoldi
                              residual estimate is followed by a recomputed residual check
                              (a system that fails it keeps iterating); 0: the estimates
                              are accepted (equal in exact arithmetic)       default 1 */
} omm_opts_t;

typedef struct {
    int       iters;        /* line searches performed                             */
    int       status;       /* OMM_OK or OMM_ENOCONV / OMM_EBREAKDOWN              */
    int       stop_rule;    /* OMM_STOP_*                                          */
    double    energy;       /* E_omm(X) for H_sigma at exit                        */
    double    rel_grad;     /* ||G(X)||_F / ||H_sigma X||_F at exit                */
    long long gmres_steps;  /* Arnoldi steps summed over all systems               */
    long long precond_calls;/* preconditioner applications (filter included)      */
    double    sigma;        /* shift used                                          */
} omm_info_t;

typedef struct omm_ctx* omm_handle_t;

typedef struct {
    int    iters;        /* filter + Rayleigh-Ritz rounds after the first Rayleigh-Ritz */
    int    applies;      /* H.X applies on the whole block                           */
    int    converged;    /* 1 when the residuals of Ritz pairs 1..N+1 met tol          */
    double res_homo;     /* |H x_N - theta_N x_N|                                      */
    double res_lumo;     /* |H x_{N+1} - theta_{N+1} x_{N+1}|                          */
} omm_estimate_info_t;

/* Fill *opts with the defaults listed above (the paper's Section 4 settings:
 * 30 poles, GMRES tolerance 1e-5, restart 15, 5 cycles, maxit 4000). */
void ommDefaultOptions(omm_opts_t* opts);

/* Create a handle for H = -Laplacian/2 + V on `grid` with N orbitals.
 *   V      host, n doubles, flat grid order; copied.
 *   N      1 <= N < n.
 *   shift  sigma of H_sigma = H - sigma I.  NaN selects sigma = hi + 1 with
 *          hi = dim*(m/2)^2/2 + max V, an upper bound of lambda_n (Section 1:
 *          the shift leaves the eigenspace unchanged).  A finite shift must
 *          exceed hi (else OMM_ENOTNEGDEF).
 *   spec   spectral window for the pole set (OMM_ESPECTRUM if inconsistent or
 *          spec->lo > min V).  NULL: estimated on the device as by
 *          ommEstimateSpectrum with its defaults, on min(N + 8, n/2) columns
 *          started from a SplitMix64 block (entries uniform in [-1, 1)); the
 *          window used is returned by ommGetSpectrum.  OMM_ESPECTRUM if that
 *          estimate does not converge.
 *   opts   NULL for defaults.
 *   stream hipStream_t to enqueue on (NULL = default stream).
 * Builds the pole set (eq. dFOP), the inner preconditioners (for SPP: the
 * stencil Q, the sparse matrix P of eq. P and its direct factorization, one
 * per pole) and all workspace of ommSolve for this N.  On success *out owns
 * all of it until ommDestroy. */
int ommSetup(const omm_grid_t* grid, const double* V, int N, double shift,
             const omm_spectrum_t* spec, const omm_opts_t* opts, void* stream,
             omm_handle_t* out);

/* HX = H_sigma X for ncols columns (Section 4.1: F^{-1} diag(|k|^2/2) F X +
 * (V - sigma) X).  X, HX: device, n x ncols, precision `prec`; may not alias.
 * 1 <= ncols.  Asynchronous. */
int ommApplyH(omm_handle_t h, const void* X, void* HX, int ncols, int prec);

/* PG = sum_j w_j Y_j with (H - z_j I) Y_j = G solved by GMRES from Y_j = G
 * (eqs. direct, lst), each column and pole an independent system, at relative
 * tolerance rtol (<= 0 selects opts.gmres_rtol).  G, PG: device complex128,
 * n x ncols, 1 <= ncols <= N; may not alias.  Asynchronous; the Arnoldi step
 * count is accumulated into the handle (ommGetCounters). */
int ommPrecondition(omm_handle_t h, const void* G, void* PG, int ncols, double rtol);

/* Precompute the preconditioner as U U^H (Section 3.3, Algorithm 2).  B: device,
 * n x ncols real FP64, column major (ld n), a Gaussian random block supplied by
 * the caller, N <= ncols <= 2N (ncols - N oversampling columns).  For every pole,
 * (H - z_j I) Y_j = B is solved by the GMRES of ommPrecondition started from B,
 * at rtol (<= 0: opts.gmres_rtol); Y = sum_j w_j Y_j; a rank-revealing QR of Y
 * (column pivoting, taken as pivoted Cholesky of the ncols x ncols Gram matrix
 * on the host, then one Cholesky re-orthogonalization on the device) gives U,
 * its first N orthonormal columns (n x N complex128, owned by the handle).  From
 * then on ommPrecondition and ommSolve apply G -> U (U^H G) (two products of
 * n x N by N x N; rtol is ignored) and the filter of ommSolve is U U^H X0.
 * B = NULL with ncols = 0 returns to the pole expansion.  Errors: OMM_EINVAL
 * (NULL B, ncols outside N..2N), OMM_ESPECTRUM (the filtered block has rank
 * below N); the handle then stays on the pole expansion.  Synchronous. */
int ommPrecompute(omm_handle_t h, const double* B, int ncols, double rtol);

/* Estimate the spectral window that ommSetup takes (Section 4 builds the contour
 * from spectral information, which the paper supplies exactly).  No handle is
 * needed.  Chebyshev-filtered subspace iteration on the device: a block of ncols
 * columns, started from B (device, n x ncols real FP64, ld n, supplied by the
 * caller, e.g. Gaussian), is filtered by the Chebyshev polynomial of degree at most
 * `degree` (<= 0: 100; lowered per round so that the filtered block stays
 * well conditioned) that damps [largest Ritz value, dim (m/2)^2/2 + max V], then
 * orthonormalized (CholeskyQR2) and rotated to its Ritz vectors (Rayleigh-Ritz,
 * complex128, the small eigenproblem on the host), until the Ritz pairs 1..N+1
 * have residual norms <= tol max(1, |theta|) (tol <= 0: 1e-6) or maxit rounds
 * (<= 0: 50) have run.  Output: spec->lo = min V (T is positive semidefinite),
 * spec->homo = theta_N (an upper bound of lambda_N: the i-th Ritz value is at
 * least lambda_i), spec->lumo = theta_{N+1} - res_{N+1} (a lower bound of the
 * eigenvalue nearest theta_{N+1}, which is lambda_{N+1} once the block holds the
 * lowest N+1 eigenvectors).  V: host, n doubles.  N + 2 <= ncols <= n/2.  info
 * may be NULL.  Returns OMM_OK, OMM_ENOCONV (maxit reached; spec and info hold
 * the last round), OMM_ESPECTRUM (the block lost rank, or no gap between the
 * N-th and (N+1)-th Ritz values) or OMM_EINVAL.  Synchronous on `stream`. */
int ommEstimateSpectrum(const omm_grid_t* grid, const double* V, int N, const double* B, int ncols, int degree,
                        double tol, int maxit, void* stream, omm_spectrum_t* spec, omm_estimate_info_t* info);

/* Y = M_j^{-1} B, the inner preconditioner of pole j = `pole` (0-based) alone:
 * for OMM_INNER_SPP the sparsifying preconditioner P_j^{-1} (Q G_j B)
 * (Section 3.2, eq. P; the sparse solve is the handle's exact direct
 * factorization), for OMM_INNER_PP the Fourier diagonal (T + <V> - z_j)^{-1}
 * (Section 3.2).  Computed at the handle's Krylov precision (complex64 under
 * OMM_MIXED).  B, Y: device complex128, n x ncols, 1 <= ncols <= N; may not
 * alias.  Uses the GMRES workspace: do not overlap with ommPrecondition or
 * ommSolve on the same handle.  Asynchronous. */
int ommApplyInner(omm_handle_t h, int pole, const void* B, void* Y, int ncols);

/* Minimize E_omm from X (device complex128, n x N, in: X0, out: the final
 * iterate, which spans the approximate lowest-N eigenspace).  With
 * opts.filter = 1 the start is first filtered, X1 = P X0 (Section 4).
 * info may be NULL.  Returns after completion. */
int ommSolve(omm_handle_t h, void* X, omm_info_t* info);

/* Independent solves of `count` instances (many-instance batches): ommSolve(hs[i], Xs[i],
 * &infos[i]) for every i, from up to 16 host threads, so that the instances' kernels
 * overlap on the device when their handles were set up on distinct streams.  Each
 * instance's result is the one ommSolve gives it alone (the kernels of one handle do not
 * depend on the others).  hs: distinct handles on the current device; Xs: their
 * orbital blocks; infos may be NULL.  Returns OMM_OK or the first failing status in
 * index order (every instance is still attempted; ommLastError(hs[i]) holds the
 * messages).  Returns after all have completed. */
int ommSolveBatched(omm_handle_t* hs, int count, void* const* Xs, omm_info_t* infos);

/* Pole set: z (2*npoles doubles, re/im interleaved) and w (same), in the
 * unshifted frame: P ~= sum_j w_j (H - z_j I)^{-1}.  Host pointers. */
int ommGetPoles(omm_handle_t h, double* z, double* w);

/* Sparsifying-preconditioner stencil of pole `pole` (0-based): q and
 * t_s = (Q G_j)(0, s) on the 3x3 neighbourhood, s = (s1, s2) in {-1,0,1}^2 at
 * index (s1+1) + 3 (s2+1); 9 complex values each, re/im interleaved (18
 * doubles), host pointers (Section 3.2, eq. P).  OMM_EUNSUPPORTED unless the
 * handle uses OMM_INNER_SPP. */
int ommGetStencil(omm_handle_t h, int pole, double* q, double* t);

/* Shift sigma in use, n, N, npoles. */
int ommGetInfo(omm_handle_t h, double* sigma, int* n, int* N, int* npoles);
/* The spectral window the handle's pole set was built from (given or estimated). */
int ommGetSpectrum(omm_handle_t h, omm_spectrum_t* spec);

/* Accumulated counters since setup: Arnoldi steps and preconditioner calls. */
int ommGetCounters(omm_handle_t h, long long* gmres_steps, long long* precond_calls);

/* Kernel-class profiling with HIP events on the handle's stream (library
 * tracing).  Classes: 0 spectral applies (FFT-based H.X and friends), 1 sparse
 * direct solve GEMMs, 2 preconditioner setup, 3 Arnoldi steps, 4 other GMRES
 * kernels, 5 outer OMM kernels, 6 sparse direct solve, first level (line
 * tridiagonal solves and stencil products).  ommSetProfiling(h, 1) clears the counters
 * and starts recording every class; ommSetProfilingClasses(h, mask) records only
 * the classes whose bit is set (mask 0 stops recording; every event pair costs host
 * and queue time, so a timing run records few classes).  The consecutive GEMM
 * launches of one sparse solve share one event pair (their launch gaps count as
 * kernel time).  ommGetProfile fills arrays of OMM_PROF_CLASSES entries (any may
 * be NULL): total milliseconds, algorithmic bytes and flops, and kernel launches
 * per class. */
#define OMM_PROF_CLASSES 7
int ommSetProfiling(omm_handle_t h, int on);
int ommSetProfilingClasses(omm_handle_t h, unsigned mask);
int ommGetProfile(omm_handle_t h, double* ms, double* bytes, double* flops, long long* launches);
const char* ommProfileClassName(int cls);

/* Release everything the handle owns (waits for its stream first). */
int ommDestroy(omm_handle_t h);

const char* ommStatusString(int status);
const char* ommLastError(omm_handle_t h);

#ifdef __cplusplus
}
#endif
#endif /* POMM_H */
